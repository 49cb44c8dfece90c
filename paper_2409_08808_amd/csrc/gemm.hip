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
// fused epilogue writes the run's row sums sum_{n in j} dQ_pn Phi_pn (FP32 within
// the tile, dQ a small integer) to part, the run's p-tile to run_mt. k_pop_finalize
// adds a row's runs in a fixed order, so a given grid gives the same sums always.
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
                                                     double* __restrict__ part, int32_t* __restrict__ run_mt,
                                                     int32_t NT, int64_t U, int32_t G, int32_t R) {
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
    int r = 0;
    for (int64_t u = U * g / G; u < u_end; ++r) {
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
        uint4 ra[4], rh[2], rl[2];
        auto fetch = [&](int k0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = tid + q * 256;
                const int rr = idx >> 2;
                const int c = (idx & 3) * 8;
                const int64_t gp = m0 + rr;
                ra[q] = gp < P ? *reinterpret_cast<const uint4*>(dQ + gp * Mp + k0 + c) : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int idx = tid + q * 256;
                const int rr = idx >> 2;
                const int c = (idx & 3) * 8;
                const int gn = n0 + rr;
                rh[q] = gn < Mp ? *reinterpret_cast<const uint4*>(Vhi + (int64_t)gn * Mp + k0 + c)
                                : make_uint4(0, 0, 0, 0);
                rl[q] = gn < Mp ? *reinterpret_cast<const uint4*>(Vlo + (int64_t)gn * Mp + k0 + c)
                                : make_uint4(0, 0, 0, 0);
            }
        };
        auto stash = [&](int buf) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = tid + q * 256;
                *reinterpret_cast<uint4*>(&As[buf][idx >> 2][(idx & 3) * 8]) = ra[q];
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int idx = tid + q * 256;
                *reinterpret_cast<uint4*>(&Hs[buf][idx >> 2][(idx & 3) * 8]) = rh[q];
                *reinterpret_cast<uint4*>(&Ls[buf][idx >> 2][(idx & 3) * 8]) = rl[q];
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
        for (int x = tid; x < PB_BM * (PB_BN / 8); x += 256) {
            const int rr = x / (PB_BN / 8), c = (x % (PB_BN / 8)) * 8;
            const int64_t gp = m0 + rr;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (gp < P && n0 + c < Mp) v = *reinterpret_cast<const uint4*>(dQ + gp * Mp + n0 + c);
            *reinterpret_cast<uint4*>(&Ds[rr][c]) = v;
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
        const int64_t slot = (int64_t)g * R + r;
        part[slot * PB_BM + tid] = red[tid][0] + red[tid][1];
        if (tid == 0) run_mt[slot] = mt;
        __syncthreads();   // the LDS is the next run's stage buffer
    }
    for (; r < R; ++r)
        if (tid == 0) run_mt[(int64_t)g * R + r] = -1;
}

// E[p] = E~ + lin[p] + the row sums of the runs on p's p-tile, with lin[p] =
// sum_k dQ[p][k] ht[k] (FP64) from the row builder or, when it did not form it,
// here: one wavefront per row, each lane sums its strided share in order, then a
// fixed butterfly
__global__ __launch_bounds__(256) void k_pop_finalize(int64_t P, int32_t M, int32_t Mp, int32_t runs,
                                                      const __hip_bfloat16* __restrict__ dQ,
                                                      const double* __restrict__ ht, const double* __restrict__ part,
                                                      const int32_t* __restrict__ run_mt,
                                                      const double* __restrict__ lin, const double* __restrict__ Ed,
                                                      double* __restrict__ E, const int32_t* __restrict__ gate) {
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= P || (gate && *gate)) return;
    const int mt = (int)(p / PB_BM), loc = (int)(p - (int64_t)mt * PB_BM);
    double s = 0.0;
    if (!lin)
        for (int k = lane; k < M; k += 64) s += (double)__bfloat162float(dQ[p * Mp + k]) * ht[k];
    for (int t = lane; t < runs; t += 64)
        if (run_mt[t] == mt) s += part[(int64_t)t * PB_BM + loc];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) E[p] = Ed[1] + (lin ? lin[p] + s : s);
}

// dQ[p][k] = bf16(charge[occ[p][mob[k]]] - c_{s(k)}), zero beyond M; grid (Mp/512, P),
// 8 consecutive k per thread written as one 16-byte store
__global__ void k_build_dq(int64_t P, int64_t n, int32_t M, int32_t Mp, int32_t E, const uint8_t* __restrict__ occ,
                           const int32_t* __restrict__ mob, const uint8_t* __restrict__ msub,
                           const double* __restrict__ dq, __hip_bfloat16* __restrict__ out,
                           const int32_t* __restrict__ gate) {
    const int64_t p = blockIdx.y;
    const int k0 = (blockIdx.x * blockDim.x + threadIdx.x) * 8;
    if (k0 >= Mp || (gate && *gate)) return;
    __hip_bfloat16 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = k0 + q;
        float x = 0.0f;
        if (k < M) {
            const int e = occ[p * n + mob[k]];
            x = (float)dq[msub[k] * E + (e < E ? e : E - 1)];   // ids are checked; the clamp keeps reads in bounds
        }
        v[q] = __float2bfloat16(x);
    }
    *reinterpret_cast<uint4*>(out + p * Mp + k0) = *reinterpret_cast<const uint4*>(v);
}

// The same for rows of at most kDqStageMax sites: one workgroup takes R rows, reads
// them into LDS with coalesced 16-byte loads and gathers from LDS, reading the
// position tables (site, sublattice, h~) once for the R rows. It also forms each
// row's linear term lin[p] = sum_k dQ[p][k] ht[k] in FP64 (each thread sums its k
// in order, then a fixed butterfly and the four waves in order).
constexpr int64_t kDqStageMax = 48 * 1024;

template <int R>
__global__ __launch_bounds__(256) void k_build_dq_staged(int64_t P, int64_t n, int32_t M, int32_t Mp, int32_t E,
                                                         const uint8_t* __restrict__ occ,
                                                         const int32_t* __restrict__ mob,
                                                         const uint8_t* __restrict__ msub,
                                                         const double* __restrict__ dq,
                                                         const double* __restrict__ ht,
                                                         __hip_bfloat16* __restrict__ out,
                                                         double* __restrict__ lin,
                                                         const int32_t* __restrict__ gate) {
    extern __shared__ __align__(16) uint8_t rows[];
    __shared__ double wsum[R][4];
    if (gate && *gate) return;
    const int64_t p0 = (int64_t)blockIdx.x * R;
    const int64_t ld = round_up(n, 16);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t p = p0 + r;
        if (p >= P) break;
        const uint8_t* src = occ + p * n;
        uint8_t* row = rows + r * ld;
        // rows start at p * n bytes: 16-byte loads only when that is aligned
        if ((((uintptr_t)src) & 15) == 0) {
            for (int64_t x = threadIdx.x * 16; x < n; x += 256 * 16) {
                if (x + 16 <= n) *reinterpret_cast<uint4*>(row + x) = *reinterpret_cast<const uint4*>(src + x);
                else
                    for (int64_t y = x; y < n; ++y) row[y] = src[y];
            }
        } else {
            for (int64_t x = threadIdx.x; x < n; x += 256) row[x] = src[x];
        }
    }
    __syncthreads();
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    for (int k0 = threadIdx.x * 8; k0 < Mp; k0 += 256 * 8) {
        // the position tables are read once for the R rows
        int site[8], sub[8];
        double h[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = k0 + q;
            site[q] = k < M ? mob[k] : 0;
            sub[q] = k < M ? msub[k] : 0;
            h[q] = k < M ? ht[k] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t p = p0 + r;
            if (p >= P) break;
            const uint8_t* row = rows + r * ld;
            __hip_bfloat16 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int k = k0 + q;
                double x = 0.0;
                if (k < M) {
                    const int e = row[site[q]];
                    x = dq[sub[q] * E + (e < E ? e : E - 1)];   // ids are checked; the clamp keeps reads in bounds
                    acc[r] += x * h[q];
                }
                v[q] = __float2bfloat16((float)x);
            }
            *reinterpret_cast<uint4*>(out + p * Mp + k0) = *reinterpret_cast<const uint4*>(v);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double a = acc[r];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) a += __shfl_xor(a, o, 64);
        if ((threadIdx.x & 63) == 0) wsum[r][threadIdx.x >> 6] = a;
    }
    __syncthreads();
    if (threadIdx.x < R && p0 + threadIdx.x < P)
        lin[p0 + threadIdx.x] = ((wsum[threadIdx.x][0] + wsum[threadIdx.x][1]) + wsum[threadIdx.x][2]) +
                                wsum[threadIdx.x][3];
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
// shared by G workgroups, and R, the most runs one share splits into. G is the
// number of units up to two workgroups per compute unit (more workgroups measured
// faster at every population size tried), divided by the tile setting kt when one
// is set or tuned.
struct PopPlan {
    int32_t NT = 0, MT = 0, G = 0, R = 0;
    int64_t U = 0;
};

static int32_t pop_max_runs(int64_t U, int64_t Umt, int64_t G) {
    int32_t R = 1;
    for (int64_t g = 0; g < G; ++g) {
        const int64_t u0 = U * g / G, u1 = U * (g + 1) / G;
        int32_t r = 0;
        for (int64_t u = u0; u < u1; ++r) {
            const int64_t mt = u / Umt, rem = u - mt * Umt;
            int64_t j = (int64_t)((std::sqrt(8.0 * (double)rem + 1.0) - 1.0) * 0.5);
            while (j * (j + 1) / 2 > rem) --j;
            while ((j + 1) * (j + 2) / 2 <= rem) ++j;
            u += std::min<int64_t>(u1 - u, j + 1 - (rem - j * (j + 1) / 2));
        }
        R = std::max(R, r);
    }
    return R;
}

static PopPlan pop_plan(const goac_problem* pb, int64_t P, int32_t kt_req) {
    PopPlan pl;
    pl.NT = (pb->d.Mp + PB_BN - 1) / PB_BN;
    pl.MT = (int32_t)((P + PB_BM - 1) / PB_BM);
    const int64_t Umt = (int64_t)pl.NT * (pl.NT + 1) / 2;
    pl.U = Umt * pl.MT;
    if (kt_req <= 0) {
        const auto it = pb->pop_kt.find(P);
        kt_req = it != pb->pop_kt.end() ? it->second : 1;
    }
    const int64_t slots = 2 * (int64_t)std::max(1, pb->ctx->num_cus);
    pl.G = (int32_t)std::min<int64_t>(pl.U, std::max<int64_t>(1, slots / kt_req));
    pl.R = pop_max_runs(pl.U, Umt, pl.G);
    return pl;
}

size_t energies_scratch_bytes(const goac_problem* pb, int64_t P, goac_precision prec) {
    const ProblemDev& d = pb->d;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    if (prec == GOAC_MIXED) {
        const PopPlan pl = pop_plan(pb, P, 0);
        const size_t runs = (size_t)pl.G * pl.R;
        const size_t dq_bytes = al((size_t)P * d.Mp * sizeof(__hip_bfloat16));
        const size_t part_bytes = al(runs * PB_BM * sizeof(double));
        const size_t mt_bytes = al(runs * sizeof(int32_t));
        return al(dq_bytes + part_bytes + mt_bytes + (size_t)P * sizeof(double));
    }
    const size_t qb = al((size_t)P * d.Mp * sizeof(double));
    const int splits = dgemm_splits(pb->ctx, P, d.M, d.Mp, nullptr, false);
    return al(2 * qb) + (splits > 1 ? al((size_t)splits * P * d.M * sizeof(double)) : 0);
}

goac_status energies_mixed(goac_problem* pb, int64_t P, const uint8_t* occ, double* E, int32_t kt_req,
                           const int32_t* gate, WsSource* src) {
    goac_ctx* ctx = pb->ctx;
    const ProblemDev& d = pb->d;
    const PopPlan pl = pop_plan(pb, P, kt_req);
    const int64_t runs = (int64_t)pl.G * pl.R;
    if (pl.U > ((int64_t)1 << 40) || runs > ((int64_t)1 << 30))
        return fail(ctx, GOAC_EINVAL, "energies: population too large for one launch");
    const size_t dq_bytes = round_up((size_t)P * d.Mp * sizeof(__hip_bfloat16), 256);
    const size_t part_bytes = round_up((size_t)runs * PB_BM * sizeof(double), 256);
    const size_t mt_bytes = round_up((size_t)runs * sizeof(int32_t), 256);
    WsSource own{ctx};
    void* ws = nullptr;
    GOAC_TRY((src ? src : &own)->get(0, dq_bytes + part_bytes + mt_bytes + (size_t)P * sizeof(double), &ws));
    __hip_bfloat16* dQ = (__hip_bfloat16*)ws;
    double* part = (double*)((char*)ws + dq_bytes);
    int32_t* run_mt = (int32_t*)((char*)ws + dq_bytes + part_bytes);
    double* lin = nullptr;
    if (d.n <= kDqStageMax) {
        lin = (double*)((char*)ws + dq_bytes + part_bytes + mt_bytes);
        // rows per workgroup: the position tables are read once for all of them
        const int64_t ld = round_up(d.n, 16);
        const int R = (P >= 4 * 2 * (int64_t)ctx->num_cus && 4 * ld <= 64 * 1024) ? 4
                      : (P >= 2 * 2 * (int64_t)ctx->num_cus && 2 * ld <= 64 * 1024) ? 2 : 1;
        const unsigned g = (unsigned)((P + R - 1) / R);
        if (R == 4)
            hipLaunchKernelGGL(k_build_dq_staged<4>, dim3(g), dim3(256), 4 * ld, ctx->stream, P, d.n, d.M, d.Mp, d.E,
                               occ, d.mob, d.msub, d.dq, d.ht, dQ, lin, gate);
        else if (R == 2)
            hipLaunchKernelGGL(k_build_dq_staged<2>, dim3(g), dim3(256), 2 * ld, ctx->stream, P, d.n, d.M, d.Mp, d.E,
                               occ, d.mob, d.msub, d.dq, d.ht, dQ, lin, gate);
        else
            hipLaunchKernelGGL(k_build_dq_staged<1>, dim3(g), dim3(256), ld, ctx->stream, P, d.n, d.M, d.Mp, d.E,
                               occ, d.mob, d.msub, d.dq, d.ht, dQ, lin, gate);
    } else
        hipLaunchKernelGGL(k_build_dq, dim3((unsigned)((d.Mp + 511) / 512), (unsigned)P), dim3(64), 0, ctx->stream,
                           P, d.n, d.M, d.Mp, d.E, occ, d.mob, d.msub, d.dq, dQ, gate);
    GOAC_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(k_pop_bf16, dim3((unsigned)pl.G), dim3(256), 0, ctx->stream, P, d.Mp, dQ, d.Vhi, d.Vlo, part,
                       run_mt, pl.NT, pl.U, pl.G, pl.R);
    GOAC_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(k_pop_finalize, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, ctx->stream, P, d.M, d.Mp,
                       (int32_t)runs, dQ, d.ht, part, run_mt, lin, d.Ed, E, gate);
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
