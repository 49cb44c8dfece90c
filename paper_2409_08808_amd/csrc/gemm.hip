// Matrix-core products of the library (gfx950 MFMA):
//   dgemm_nt        C = alpha A B^T + beta C in FP64 (v_mfma_f64_16x16x4f64): the
//                   reciprocal-space Ewald sum, FP64 population energies and the
//                   FP64 re-anchoring of the Monte Carlo field.
//   k_pop_bf16      Phi = dQ (V_hi + V_lo) with bf16 inputs and FP32 accumulation
//                   (v_mfma_f32_32x32x16_bf16) and a fused FP64 row-dot epilogue:
//                   the mixed-precision population energies.
#include <algorithm>

#include "common.h"

namespace goac {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ FP64 NT GEMM
// C = alpha A B^T + beta C, A: M x K (lda), B: N x K (ldb), FP64.
// Tile 64 x 64 x 16, 256 threads = 4 waves in a 2 x 2 grid, each wave a 32 x 32
// block of four 16 x 16 MFMA accumulators. Operands are staged k-major in two LDS
// buffers; the next K-slice is loaded into registers while the matrix cores work
// on the current one (one barrier per slice). Rows beyond M (or *M_dev) and
// columns beyond N are skipped; K is zero-padded. With split-K (gridDim.z > 1)
// each z-slice writes its partial product to `part`, reduced in slice order by
// k_dgemm_reduce (deterministic). With sym (A = B, M = N: C += alpha A A^T), only
// the tiles on and above the diagonal are computed; each mirrors its result (or
// its partial) into the transposed tile (each element keeping its own beta C term).
constexpr int DG_BM = 64, DG_BN = 64, DG_BK = 16;
static_assert(DG_BM == DG_BN, "the symmetric product mirrors square tiles");

__global__ __launch_bounds__(256) void k_dgemm_nt(int64_t M, int64_t N, int64_t K, const double* __restrict__ A,
                                                  int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                  double* __restrict__ C, int64_t ldc, double alpha, double beta,
                                                  const int32_t* __restrict__ M_dev, int64_t k_per_split,
                                                  double* __restrict__ part, int32_t sym) {
    __shared__ double As[2][DG_BK][DG_BM + 2];
    __shared__ double Bs[2][DG_BK][DG_BN + 2];
    if (M_dev) M = *M_dev;
    if (sym && blockIdx.y > blockIdx.x) return;
    const int64_t m0 = (int64_t)blockIdx.y * DG_BM;
    const int64_t n0 = (int64_t)blockIdx.x * DG_BN;
    if (m0 >= M) return;
    const int64_t kbeg = (int64_t)blockIdx.z * k_per_split;
    const int64_t kend = kbeg + k_per_split < K ? kbeg + k_per_split : K;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    f64x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    // loader mapping: each thread moves 4 consecutive k of one row of A and of B
    const int lr = tid >> 2;          // 0..63
    const int lk = (tid & 3) * 4;     // 0, 4, 8, 12
    const int64_t gm = m0 + lr, gn = n0 + lr;
    const double* pa = A + gm * lda;
    const double* pb = B + gn * ldb;
    double ra[4], rb[4];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gk = k0 + lk + q;
            ra[q] = (gm < M && gk < kend) ? pa[gk] : 0.0;
            rb[q] = (gn < N && gk < kend) ? pb[gk] : 0.0;
        }
    };
    if (kbeg < kend) fetch(kbeg);
    int buf = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += DG_BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[buf][lk + q][lr] = ra[q];
            Bs[buf][lk + q][lr] = rb[q];
        }
        __syncthreads();
        if (k0 + DG_BK < kend) fetch(k0 + DG_BK);
#pragma unroll
        for (int ks = 0; ks < DG_BK; ks += 4) {
            const int kk = ks + (lane >> 4);
            const double a0 = As[buf][kk][wm * 32 + (lane & 15)];
            const double a1 = As[buf][kk][wm * 32 + 16 + (lane & 15)];
            const double b0 = Bs[buf][kk][wn * 32 + (lane & 15)];
            const double b1 = Bs[buf][kk][wn * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        buf ^= 1;
    }
    // FP64 16x16 accumulators interleave rows: D[row = lane / 16 + 4 v][col = lane % 16]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t r = m0 + wm * 32 + a * 16 + (lane >> 4) + 4 * v;
                const int64_t cix = n0 + wn * 32 + b * 16 + (lane & 15);
                if (r < M && cix < N) {
                    if (part) {
                        part[((int64_t)blockIdx.z * M + r) * N + cix] = acc[a][b][v];
                        if (sym && blockIdx.y < blockIdx.x) part[((int64_t)blockIdx.z * M + cix) * N + r] = acc[a][b][v];
                    } else {
                        double* c = C + r * ldc + cix;
                        const double val = alpha * acc[a][b][v];
                        *c = (beta == 0.0) ? val : val + beta * *c;
                        if (sym && blockIdx.y < blockIdx.x) {
                            double* ct = C + cix * ldc + r;
                            *ct = (beta == 0.0) ? val : val + beta * *ct;
                        }
                    }
                }
            }
}

// C = alpha sum_z part[z] + beta C, slices summed in order
__global__ void k_dgemm_reduce(int64_t M, int64_t N, int32_t splits, const double* __restrict__ part,
                               double* __restrict__ C, int64_t ldc, double alpha, double beta) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * N) return;
    const int64_t r = idx / N, c = idx - r * N;
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * M * N + idx];
    double* o = C + r * ldc + c;
    const double val = alpha * s;
    *o = (beta == 0.0) ? val : val + beta * *o;
}

// split K when the tile grid leaves most compute units idle and K is long
int dgemm_splits(const goac_ctx* ctx, int64_t M, int64_t N, int64_t K, const int32_t* M_dev, bool sym) {
    const int64_t tn = (N + DG_BN - 1) / DG_BN;
    const int64_t tiles = sym ? tn * (tn + 1) / 2 : tn * ((M + DG_BM - 1) / DG_BM);
    int splits = 1;
    const int64_t want = 2 * (int64_t)ctx->num_cus;
    while (!M_dev && tiles * splits < want && K / (splits * 2) >= 256 && splits < 32) splits *= 2;
    return splits;
}

goac_status dgemm_nt(goac_ctx* ctx, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                     const double* B, int64_t ldb, double* C, int64_t ldc, double alpha, double beta,
                     const int32_t* M_dev, bool sym, WsSource* ws) {
    if (M <= 0 || N <= 0) return GOAC_OK;
    if (sym && (M != N || A != B || lda != ldb || M_dev))
        return fail(ctx, GOAC_EINVAL, "dgemm_nt: a symmetric product needs A = B and M = N");
    const int splits = dgemm_splits(ctx, M, N, K, M_dev, sym);
    const int64_t kps = round_up((K + splits - 1) / splits, DG_BK);
    double* part = nullptr;
    if (splits > 1) {
        WsSource own{ctx};
        void* w = nullptr;
        GOAC_TRY((ws ? ws : &own)->get(1, (size_t)splits * M * N * sizeof(double), &w));
        part = (double*)w;
    }
    dim3 grid((unsigned)((N + DG_BN - 1) / DG_BN), (unsigned)((M + DG_BM - 1) / DG_BM), (unsigned)splits);
    hipLaunchKernelGGL(k_dgemm_nt, grid, dim3(256), 0, ctx->stream, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta,
                       M_dev, kps, part, sym ? 1 : 0);
    GOAC_CHECK_LAUNCH(ctx);
    if (splits > 1) {
        hipLaunchKernelGGL(k_dgemm_reduce, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, ctx->stream, M, N,
                           splits, part, C, ldc, alpha, beta);
        GOAC_CHECK_LAUNCH(ctx);
    }
    return GOAC_OK;
}

// ------------------------------------------------------------------ bf16 hi+lo population GEMM
// E_p - lin_p - E~ = 1/2 dQ_p^T V dQ_p. With the mobile positions in 128-wide
// tiles, 1/2 dQ^T V dQ = sum over n-tiles j and k-tiles i <= j of
//   sum_{n in j} dQ_pn sum_{k in i} W_nk dQ_pk,
// W = V for i < j and V / 2 for i = j (stored so, hi and lo in bf16: k_extract),
// so every (p-tile, n-tile j, k-tile i <= j) unit has weight one and the symmetric
// half of the matrix work is all there is. The units are enumerated p-tile, then
// j, then i (i fastest), and a grid of G workgroups takes equal contiguous shares
// of them (stream-K: no partial last wave however the units fall). A share splits
// into runs, one per (p-tile, j) it touches; a run accumulates its k-tiles on the
// matrix cores (bf16 inputs, v_mfma_f32_32x32x16_bf16, FP32 accumulation) and its
// fused epilogue adds the run's row sums sum_{n in j} dQ_pn Phi_pn (FP32 within the
// tile, dQ a small integer) into the row's 64-bit fixed-point accumulator (scale
// 2^sc, a power of two chosen per problem so that no sum of absolute terms of a row
// reaches 2^61). Integer addition is associative, so the energies do not depend on
// the order in which the runs finish (for a given grid, the same bits every call);
// k_pop_finalize then writes E[p] = E~ + acc[p] / 2^sc.
//
// Tile 256 (p) x 128 (n) x 32 (k), 256 threads = 2 x 2 waves, each wave 128 x 64 =
// 4 x 2 accumulators fed by the hi and the lo operand: 16 MFMAs per 8 LDS operand
// reads. The next K stage is fetched into registers while the matrix cores work
// on the current one; double-buffered LDS (80 KiB, two workgroups per compute
// unit), one barrier per stage.
constexpr int PB_BM = 256, PB_BN = 128, PB_BK = 32, PB_LD = PB_BK + 8, PB_DLD = PB_BN + 8;
constexpr int kPopLds = 2 * (PB_BM + 2 * PB_BN) * PB_LD * 2;   // 80 KiB
static_assert(PB_BM * PB_DLD * 2 + PB_BM * 2 * 8 <= kPopLds, "epilogue staging exceeds the stage buffers");

__global__ __launch_bounds__(256, 2) void k_pop_bf16(int64_t P, int32_t Mp, const __hip_bfloat16* __restrict__ dQ,
                                                     const __hip_bfloat16* __restrict__ Vhi,
                                                     const __hip_bfloat16* __restrict__ Vlo,
                                                     unsigned long long* __restrict__ rowacc, int32_t NT, int64_t U,
                                                     int32_t G, const double* __restrict__ Ed) {
    // operand stages during the K loop; the epilogue reuses the same bytes for the
    // tile's dQ block and the row sums
    __shared__ __align__(16) unsigned char smem[kPopLds];
    auto As = reinterpret_cast<__hip_bfloat16 (*)[PB_BM][PB_LD]>(smem);
    auto Hs = reinterpret_cast<__hip_bfloat16 (*)[PB_BN][PB_LD]>(smem + 2 * PB_BM * PB_LD * 2);
    auto Ls = reinterpret_cast<__hip_bfloat16 (*)[PB_BN][PB_LD]>(smem + 2 * (PB_BM + PB_BN) * PB_LD * 2);
    auto Ds = reinterpret_cast<__hip_bfloat16 (*)[PB_DLD]>(smem);
    auto red = reinterpret_cast<double (*)[2]>(smem + PB_BM * PB_DLD * 2);
    const int g = (int)blockIdx.x;
    const int64_t u_end = U * (g + 1) / G;
    const int64_t Umt = (int64_t)NT * (NT + 1) / 2;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const double scale = Ed[2];
    for (int64_t u = U * g / G; u < u_end;) {
        // the run from unit u: p-tile mt, n-tile j, k-tiles i0 .. i0 + len - 1 of j
        const int mt = (int)(u / Umt);
        const int64_t rem = u - (int64_t)mt * Umt;
        int j = (int)((sqrt(8.0 * (double)rem + 1.0) - 1.0) * 0.5);
        while ((int64_t)j * (j + 1) / 2 > rem) --j;
        while ((int64_t)(j + 1) * (j + 2) / 2 <= rem) ++j;
        const int i0 = (int)(rem - (int64_t)j * (j + 1) / 2);
        const int len = (int)std::min<int64_t>(u_end - u, (int64_t)(j + 1 - i0));
        u += len;
        const int kbeg = i0 * PB_BN;
        const int kend = (i0 + len) * PB_BN < Mp ? (i0 + len) * PB_BN : Mp;
        const int64_t m0 = (int64_t)mt * PB_BM;
        const int n0 = j * PB_BN;
        f32x16 acc[4][2];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = f32x16{};
        // loader: the p-tile is 256 rows x 32 k = 1024 chunks of 8 bf16 (four per
        // thread), each n-tile 128 rows x 32 k (two per thread)
        // Thread tid loads rows tid / 4 + 64 q at columns 8 (tid % 4) of each operand;
        // dQ and W share the row stride Mp, so one 32-bit element offset serves every
        // load beside a uniform base. dQ has rows up to the next multiple of 256 and W
        // is Mq x Mq, so every load lies inside its buffer and none is conditional.
        v4u32 ra[4], rh[2], rl[2];
        const uint32_t to = (uint32_t)(tid >> 2) * (uint32_t)Mp + (uint32_t)(tid & 3) * 8u;
        const int64_t slab = (int64_t)64 * Mp;
        auto fetch = [&](int k0) {
            const __hip_bfloat16* a0 = dQ + m0 * Mp + k0;
            const __hip_bfloat16* h0 = Vhi + (int64_t)n0 * Mp + k0;
            const __hip_bfloat16* l0 = Vlo + (int64_t)n0 * Mp + k0;
#pragma unroll
            for (int q = 0; q < 4; ++q) ra[q] = *reinterpret_cast<const v4u32*>(a0 + q * slab + to);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                rh[q] = *reinterpret_cast<const v4u32*>(h0 + q * slab + to);
                rl[q] = *reinterpret_cast<const v4u32*>(l0 + q * slab + to);
            }
        };
        auto stash = [&](int buf) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = tid + q * 256;
                *reinterpret_cast<v4u32*>(&As[buf][idx >> 2][(idx & 3) * 8]) = ra[q];
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int idx = tid + q * 256;
                *reinterpret_cast<v4u32*>(&Hs[buf][idx >> 2][(idx & 3) * 8]) = rh[q];
                *reinterpret_cast<v4u32*>(&Ls[buf][idx >> 2][(idx & 3) * 8]) = rl[q];
            }
        };
        fetch(kbeg);
        stash(0);
        __syncthreads();
        int buf = 0;
        for (int k0 = kbeg; k0 < kend; k0 += PB_BK) {
            const bool more = k0 + PB_BK < kend;
            if (more) fetch(k0 + PB_BK);
#pragma unroll
            for (int ks = 0; ks < PB_BK; ks += 16) {
                const int kk = ks + 8 * (lane >> 5);
                bf16x8 av[4], hv[2], lv[2];
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    av[a] = *reinterpret_cast<const bf16x8*>(&As[buf][wm * 128 + a * 32 + (lane & 31)][kk]);
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    hv[b] = *reinterpret_cast<const bf16x8*>(&Hs[buf][wn * 64 + b * 32 + (lane & 31)][kk]);
                    lv[b] = *reinterpret_cast<const bf16x8*>(&Ls[buf][wn * 64 + b * 32 + (lane & 31)][kk]);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], hv[b], acc[a][b], 0, 0, 0);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], lv[b], acc[a][b], 0, 0, 0);
            }
            if (more) stash(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
        // epilogue. The tile's dQ block (256 p x 128 n) is staged in LDS with 16-byte
        // loads. Lane holds D[i][j] of each 32 x 32 block, j = lane % 32,
        // i = 8 (v / 4) + 4 (lane / 32) + v % 4; per 32-row block the lane forms
        // x_v = sum_b dQ[i][j_b] D_b[i][j] and a halving butterfly over the 32 lanes of
        // its half (masks 16, 8, 4, 2, 1, each step keeping half of the rows) leaves
        // row v(lane) summed over all 32 columns in lanes 2c and 2c + 1 (fixed order,
        // deterministic).
        {
            const __hip_bfloat16* d0 = dQ + m0 * Mp + n0;
            for (int x = tid; x < PB_BM * (PB_BN / 8); x += 256) {
                const int rr = x / (PB_BN / 8), c = (x % (PB_BN / 8)) * 8;
                *reinterpret_cast<uint4*>(&Ds[rr][c]) =
                    *reinterpret_cast<const uint4*>(d0 + ((uint32_t)rr * (uint32_t)Mp + (uint32_t)c));
            }
        }
        __syncthreads();
        const int c32 = lane & 31, h = lane >> 5;
        const int vkeep = ((c32 >> 4) & 1) * 8 + ((c32 >> 3) & 1) * 4 + ((c32 >> 2) & 1) * 2 + ((c32 >> 1) & 1);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            float x[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 8 * (v >> 2) + 4 * h + (v & 3);
                const int rr = wm * 128 + a * 32 + i;
                float s2 = 0.0f;
#pragma unroll
                for (int b = 0; b < 2; ++b) s2 += __bfloat162float(Ds[rr][wn * 64 + b * 32 + c32]) * acc[a][b][v];
                x[v] = s2;
            }
#pragma unroll
            for (int w = 8; w >= 1; w >>= 1) {
                const bool low = (c32 & (2 * w)) == 0;   // keep rows v < w of the current block
#pragma unroll
                for (int v = 0; v < w; ++v) {
                    const float send = low ? x[v + w] : x[v];
                    const float recv = __shfl_xor(send, 2 * w, 64);
                    x[v] = (low ? x[v] : x[v + w]) + recv;
                }
            }
            const float tot = x[0] + __shfl_xor(x[0], 1, 64);
            if ((c32 & 1) == 0) {
                const int i = 8 * (vkeep >> 2) + 4 * h + (vkeep & 3);
                red[wm * 128 + a * 32 + i][wn] = (double)tot;
            }
        }
        __syncthreads();
        if (m0 + tid < P)
            atomicAdd(rowacc + m0 + tid, (unsigned long long)__double2ll_rn((red[tid][0] + red[tid][1]) * scale));
        __syncthreads();   // the LDS is the next run's stage buffer
    }
}

// E[p] = E~ + acc[p] / 2^sc, unless the gate is set
__global__ __launch_bounds__(256) void k_pop_finalize(int64_t P, const long long* __restrict__ acc,
                                                      const double* __restrict__ Ed, double* __restrict__ E,
                                                      const int32_t* __restrict__ gate) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P || (gate && *gate)) return;
    E[p] = Ed[1] + (double)acc[p] * Ed[3];
}

// Rows of the population product (Mq columns), one workgroup of T threads (64 to
// 512) per row p, each thread taking 8 consecutive mobile positions per step:
//   dQ[p][k] = bf16(charge[occ[p][mob[k]]] - c_{s(k)}), zero beyond M (16-byte stores);
//   acc[p] = round(2^sc lin_p), lin_p = sum_k dQ[p][k] ht[k] in FP64 (each thread in
//   order, then a fixed butterfly, then the waves in order).
// With chk, the occupancy constraints of Eq. 2 are checked on the way: a species id
// >= E, or (sublattice, species) counts over the row's mobile positions that differ
// from the problem's, or 1 into *chk. With at most 16 (sublattice, species) pairs
// the counts stay in registers, 8-bit fields of two 64-bit words moved to 32-bit
// counters every 16 steps (before a field can pass 128); more pairs count in an LDS
// histogram.
constexpr int kPrepMaxT = 512;

__global__ __launch_bounds__(kPrepMaxT) void k_prep_rows(int64_t P, int64_t n, int32_t M, int32_t Mq, int32_t S,
                                                         int32_t E, const uint8_t* __restrict__ occ,
                                                         const int32_t* __restrict__ mob,
                                                         const uint8_t* __restrict__ msub,
                                                         const double* __restrict__ dq,
                                                         const double* __restrict__ ht,
                                                         const int32_t* __restrict__ tab,
                                                         const double* __restrict__ Ed,
                                                         __hip_bfloat16* __restrict__ dQ,
                                                         unsigned long long* __restrict__ acc,
                                                         int32_t* __restrict__ chk) {
    __shared__ int hist[kMaxSub * kMaxSpecies];
    __shared__ double wsum[kPrepMaxT / 64];
    const int64_t p = blockIdx.x;
    const int tid = threadIdx.x, T = blockDim.x;
    const int nb = S * E;
    // loads off the row's dependency chain go out first
    const double scale = Ed[2];
    const int32_t* cnt = tab + 2 + 2 * S;
    const int want = chk && tid < nb ? cnt[tid] : 0;
    for (int x = tid; x < nb; x += T) hist[x] = 0;
    if (chk && nb > 16) __syncthreads();   // the loop counts into the histogram
    const uint8_t* row = occ + p * n;
    double lin = 0.0;
    bool bad = false;
    uint32_t tot[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) tot[b] = 0;
    uint64_t lo = 0, hi = 0;
    int steps = 0;
    auto flush = [&]() {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            tot[b] += (uint32_t)((lo >> (8 * b)) & 0xffu);
            tot[b + 8] += (uint32_t)((hi >> (8 * b)) & 0xffu);
        }
        lo = hi = 0;
    };
    for (int k0 = tid * 8; k0 < Mq; k0 += T * 8) {
        int site[8];
        uint2 sb = make_uint2(0, 0);
        double h[8];
        if (k0 + 8 <= M) {
            const int4 a = *reinterpret_cast<const int4*>(mob + k0);
            const int4 b = *reinterpret_cast<const int4*>(mob + k0 + 4);
            site[0] = a.x; site[1] = a.y; site[2] = a.z; site[3] = a.w;
            site[4] = b.x; site[5] = b.y; site[6] = b.z; site[7] = b.w;
            sb = *reinterpret_cast<const uint2*>(msub + k0);
#pragma unroll
            for (int q = 0; q < 8; q += 2) {
                const double2 t = *reinterpret_cast<const double2*>(ht + k0 + q);
                h[q] = t.x;
                h[q + 1] = t.y;
            }
        } else {
            // the tail: the position tables hold M (mobile sites) and Mp entries
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool in = k0 + q < M;
                site[q] = in ? mob[k0 + q] : -1;
                h[q] = in ? ht[k0 + q] : 0.0;
                if (in) (q < 4 ? sb.x : sb.y) |= (uint32_t)msub[k0 + q] << (8 * (q & 3));
            }
        }
        __hip_bfloat16 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            double x = 0.0;
            if (site[q] >= 0) {
                const int e = row[site[q]];
                const int sl = (int)(((q < 4 ? sb.x : sb.y) >> (8 * (q & 3))) & 0xffu);
                if (e >= E) {
                    bad = true;
                } else {
                    const int b = sl * E + e;
                    x = dq[b];
                    if (nb <= 16) {
                        lo += b < 8 ? 1ull << (8 * (b & 7)) : 0ull;
                        hi += b >= 8 ? 1ull << (8 * (b & 7)) : 0ull;
                    } else if (chk) {
                        atomicAdd(&hist[b], 1);
                    }
                }
                lin += x * h[q];
            }
            v[q] = __float2bfloat16((float)x);
        }
        *reinterpret_cast<uint4*>(dQ + p * Mq + k0) = *reinterpret_cast<const uint4*>(v);
        if (nb <= 16 && ++steps == 16) {
            flush();
            steps = 0;
        }
    }
    const int lane = tid & 63, wave = tid >> 6;
    if (chk && nb <= 16) {
        __syncthreads();   // the histogram is cleared
        flush();
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            if (b < nb) {
                uint32_t c = tot[b];
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) c += __shfl_xor(c, o, 64);
                if (lane == 0) atomicAdd(&hist[b], (int)c);
            }
        }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) lin += __shfl_xor(lin, o, 64);
    if (lane == 0) wsum[wave] = lin;
    __syncthreads();
    if (tid == 0) {
        double l = 0.0;
        for (int w = 0; w < T / 64; ++w) l += wsum[w];
        acc[p] = (unsigned long long)__double2ll_rn(l * scale);
    }
    if (!chk) return;
    if (tid < nb && hist[tid] != want) bad = true;
    for (int x = tid + T; x < nb; x += T)
        if (hist[x] != cnt[x]) bad = true;
    if (bad) atomicOr(chk, 1);
}

// Q[p][k] = charge[occ[p][mob[k]]] (FP64), zero beyond M
__global__ void k_build_q64(int64_t P, int64_t n, int32_t M, int32_t Mp, int32_t E, const uint8_t* __restrict__ occ,
                            const int32_t* __restrict__ mob, const double* __restrict__ charge,
                            double* __restrict__ out, const int32_t* __restrict__ gate) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * (int64_t)Mp || (gate && *gate)) return;
    const int64_t p = idx / Mp;
    const int k = (int)(idx - p * Mp);
    double v = 0.0;
    if (k < M) {
        const int e = occ[p * n + mob[k]];
        v = charge[e < E ? e : E - 1];
    }
    out[idx] = v;
}

// E[p] = E_ff + sum_k q_k (h_k + Phi_k / 2): one wavefront per row, lanes stride
// over k, fixed-order butterfly sum (deterministic)
__global__ __launch_bounds__(256) void k_pop_fp64_finalize(int64_t P, int32_t M, int32_t Mp,
                                                           const double* __restrict__ Q,
                                                           const double* __restrict__ Phi,
                                                           const double* __restrict__ h, const double* __restrict__ Ed,
                                                           double* __restrict__ E, const int32_t* __restrict__ gate) {
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= P || (gate && *gate)) return;
    double s = 0.0;
    for (int k = lane; k < M; k += 64) s += Q[p * Mp + k] * (h[k] + 0.5 * Phi[p * Mp + k]);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) E[p] = Ed[0] + s;
}

goac_status build_q64(goac_ctx* ctx, int64_t P, int64_t n, int32_t M, int32_t Mp, int32_t E, const uint8_t* occ,
                      const int32_t* mob, const double* charge, double* Q, const int32_t* gate) {
    const int64_t tot = P * (int64_t)Mp;
    hipLaunchKernelGGL(k_build_q64, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, P, n, M, Mp, E,
                       occ, mob, charge, Q, gate);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

// Grid of the mixed product for P rows: U units (p-tile, n-tile j, k-tile i <= j)
// shared by G workgroups. G is the number of units up to two workgroups per compute
// unit (more workgroups measured faster at every population size tried), divided by
// the tile setting kt when one is set or tuned. G moves the run boundaries, so the
// energies differ between settings by the FP32 accumulation order only.
struct PopPlan {
    int32_t NT = 0, MT = 0, G = 0;
    int64_t U = 0;
};

static PopPlan pop_plan(const goac_problem* pb, int64_t P, int32_t kt_req) {
    PopPlan pl;
    pl.NT = pb->d.Mq / PB_BN;
    pl.MT = (int32_t)((P + PB_BM - 1) / PB_BM);
    const int64_t Umt = (int64_t)pl.NT * (pl.NT + 1) / 2;
    pl.U = Umt * pl.MT;
    if (kt_req <= 0) {
        const auto it = pb->pop_kt.find(P);
        kt_req = it != pb->pop_kt.end() ? it->second : 1;
    }
    const int64_t slots = 2 * (int64_t)std::max(1, pb->ctx->num_cus);
    pl.G = (int32_t)std::min<int64_t>(pl.U, std::max<int64_t>(1, slots / kt_req));
    return pl;
}

// threads per row of the row kernel: 8 positions per thread and step, 64 to 512
static int prep_threads(int32_t Mq) {
    const int t = (int)std::min<int64_t>(kPrepMaxT, ((int64_t)Mq / 8 + 63) / 64 * 64);
    return std::max(64, t);
}

size_t energies_scratch_bytes(const goac_problem* pb, int64_t P, goac_precision prec) {
    const ProblemDev& d = pb->d;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    if (prec == GOAC_MIXED)
        return al((size_t)round_up(P, PB_BM) * d.Mq * sizeof(__hip_bfloat16)) + al((size_t)P * sizeof(long long));
    const size_t qb = al((size_t)P * d.Mp * sizeof(double));
    const int splits = dgemm_splits(pb->ctx, P, d.M, d.Mp, nullptr, false);
    return al(2 * qb) + (splits > 1 ? al((size_t)splits * P * d.M * sizeof(double)) : 0);
}

goac_status energies_mixed(goac_problem* pb, int64_t P, const uint8_t* occ, double* E, int32_t kt_req,
                           int32_t* chk, WsSource* src, int32_t* host, hipEvent_t ev) {
    goac_ctx* ctx = pb->ctx;
    const ProblemDev& d = pb->d;
    const PopPlan pl = pop_plan(pb, P, kt_req);
    if (pl.U > ((int64_t)1 << 40)) return fail(ctx, GOAC_EINVAL, "energies: population too large for one launch");
    // dQ rows up to the product's next p-tile boundary (the rows past P are read,
    // never written, and only feed product rows that are discarded)
    const size_t dq_bytes = round_up((size_t)round_up(P, PB_BM) * d.Mq * sizeof(__hip_bfloat16), 256);
    WsSource own{ctx};
    void* ws = nullptr;
    GOAC_TRY((src ? src : &own)->get(0, dq_bytes + round_up((size_t)P * sizeof(long long), 256), &ws));
    __hip_bfloat16* dQ = (__hip_bfloat16*)ws;
    unsigned long long* acc = (unsigned long long*)((char*)ws + dq_bytes);
    hipLaunchKernelGGL(k_prep_rows, dim3((unsigned)P), dim3(prep_threads(d.Mq)), 0, ctx->stream, P, d.n, d.M, d.Mq,
                       d.S, d.E, occ, d.mob, d.msub, d.dq, d.ht, d.tab, d.Ed, dQ, acc, chk);
    GOAC_CHECK_LAUNCH(ctx);
    if (host) GOAC_HIP(ctx, hipMemcpyAsync(host, chk, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    if (ev) GOAC_HIP(ctx, hipEventRecord(ev, ctx->stream));
    hipLaunchKernelGGL(k_pop_bf16, dim3((unsigned)pl.G), dim3(256), 0, ctx->stream, P, d.Mq, dQ, d.Vhi, d.Vlo,
                       acc, pl.NT, pl.U, pl.G, d.Ed);
    GOAC_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(k_pop_finalize, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, ctx->stream, P,
                       (const long long*)acc, d.Ed, E, chk);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

goac_status energies_fp64(goac_problem* pb, int64_t P, const uint8_t* occ, double* E, const int32_t* gate,
                          WsSource* src) {
    goac_ctx* ctx = pb->ctx;
    const ProblemDev& d = pb->d;
    const size_t qb = round_up((size_t)P * d.Mp * sizeof(double), 256);
    WsSource own{ctx};
    void* ws = nullptr;
    goac_status st = (src ? src : &own)->get(0, 2 * qb, &ws);
    if (st != GOAC_OK) return st;
    double* Q = (double*)ws;
    double* Phi = (double*)((char*)ws + qb);
    GOAC_TRY(build_q64(ctx, P, d.n, d.M, d.Mp, d.E, occ, d.mob, d.charge, Q, gate));
    st = dgemm_nt(ctx, P, d.M, d.Mp, Q, d.Mp, d.V64, d.Mp, Phi, d.Mp, 1.0, 0.0, nullptr, false, src);
    if (st != GOAC_OK) return st;
    hipLaunchKernelGGL(k_pop_fp64_finalize, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, ctx->stream, P, d.M,
                       d.Mp, Q, Phi, d.h, d.Ed, E, gate);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

}  // namespace goac

namespace goac {
goac_status energies_enqueue(goac_problem* pb, int64_t P, const uint8_t* occ, goac_precision prec, double* E) {
    return prec == GOAC_MIXED ? energies_mixed(pb, P, occ, E) : energies_fp64(pb, P, occ, E);
}
}  // namespace goac
