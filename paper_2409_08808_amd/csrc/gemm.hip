// Matrix-core products of the library (gfx950 MFMA):
//   dgemm_nt        C = alpha A B^T + beta C in FP64 (v_mfma_f64_16x16x4f64): the
//                   reciprocal-space Ewald sum, FP64 population energies and the
//                   FP64 re-anchoring of the Monte Carlo field.
//   k_pop_bf16      Phi = dQ (V_hi + V_lo) with bf16 inputs and FP32 accumulation
//                   (v_mfma_f32_32x32x16_bf16) and a fused FP64 row-dot epilogue:
//                   the mixed-precision population energies.
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
// k_dgemm_reduce (deterministic).
constexpr int DG_BM = 64, DG_BN = 64, DG_BK = 16;

__global__ __launch_bounds__(256) void k_dgemm_nt(int64_t M, int64_t N, int64_t K, const double* __restrict__ A,
                                                  int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                  double* __restrict__ C, int64_t ldc, double alpha, double beta,
                                                  const int32_t* __restrict__ M_dev, int64_t k_per_split,
                                                  double* __restrict__ part) {
    __shared__ double As[2][DG_BK][DG_BM + 2];
    __shared__ double Bs[2][DG_BK][DG_BN + 2];
    if (M_dev) M = *M_dev;
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
                    } else {
                        double* c = C + r * ldc + cix;
                        const double val = alpha * acc[a][b][v];
                        *c = (beta == 0.0) ? val : val + beta * *c;
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

goac_status dgemm_nt(goac_ctx* ctx, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                     const double* B, int64_t ldb, double* C, int64_t ldc, double alpha, double beta,
                     const int32_t* M_dev) {
    if (M <= 0 || N <= 0) return GOAC_OK;
    const int64_t tiles = ((N + DG_BN - 1) / DG_BN) * ((M + DG_BM - 1) / DG_BM);
    // split K when the tile grid leaves most compute units idle and K is long
    int splits = 1;
    const int64_t want = 2 * (int64_t)ctx->num_cus;
    while (!M_dev && tiles * splits < want && K / (splits * 2) >= 512 && splits < 32) splits *= 2;
    const int64_t kps = round_up((K + splits - 1) / splits, DG_BK);
    double* part = nullptr;
    if (splits > 1) {
        void* w = nullptr;
        goac_status st = workspace(ctx, 1, (size_t)splits * M * N * sizeof(double), &w);
        if (st != GOAC_OK) return st;
        part = (double*)w;
    }
    dim3 grid((unsigned)((N + DG_BN - 1) / DG_BN), (unsigned)((M + DG_BM - 1) / DG_BM), (unsigned)splits);
    hipLaunchKernelGGL(k_dgemm_nt, grid, dim3(256), 0, ctx->stream, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta,
                       M_dev, kps, part);
    GOAC_CHECK_LAUNCH(ctx);
    if (splits > 1) {
        hipLaunchKernelGGL(k_dgemm_reduce, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, ctx->stream, M, N,
                           splits, part, C, ldc, alpha, beta);
        GOAC_CHECK_LAUNCH(ctx);
    }
    return GOAC_OK;
}

// ------------------------------------------------------------------ bf16 hi+lo population GEMM
// Phi[p][n] = sum_k dQ[p][k] (Vhi[n][k] + Vlo[n][k]) (V is symmetric, so its rows
// serve as columns), bf16 inputs, FP32 accumulation on v_mfma_f32_32x32x16_bf16.
// Fused epilogue per output tile, in FP64 (linear in Phi, so K may be split):
//   part[p][t] = sum_{n in tile} dQ[p][n] (ht[n] [first K slice only] + Phi_slice[p][n] / 2)
// Tile 128 (p) x 128 (n) x 32 (k), 256 threads = 2 x 2 waves, each wave 64 x 64 =
// 2 x 2 accumulators, each fed by the hi and the lo operand: 8 MFMAs per 6 LDS
// operand reads. The next K stage is fetched into registers while the matrix
// cores work on the current one; double-buffered LDS, one barrier per stage.
constexpr int PB_BM = 128, PB_BN = 128, PB_BK = 32, PB_LD = PB_BK + 8;

__global__ __launch_bounds__(256) void k_pop_bf16(int64_t P, int32_t M, int32_t Mp,
                                                  const __hip_bfloat16* __restrict__ dQ,
                                                  const __hip_bfloat16* __restrict__ Vhi,
                                                  const __hip_bfloat16* __restrict__ Vlo,
                                                  const double* __restrict__ ht, double* __restrict__ part,
                                                  int32_t n_tiles_total, int32_t k_per_split) {
    __shared__ __align__(16) __hip_bfloat16 As[2][PB_BM][PB_LD];
    __shared__ __align__(16) __hip_bfloat16 Hs[2][PB_BN][PB_LD];
    __shared__ __align__(16) __hip_bfloat16 Ls[2][PB_BN][PB_LD];
    __shared__ double red[PB_BM][2];
    const int64_t m0 = (int64_t)blockIdx.y * PB_BM;
    const int n0 = blockIdx.x * PB_BN;
    const int split = blockIdx.z;
    const int kbeg = split * k_per_split;
    const int kend = kbeg + k_per_split < Mp ? kbeg + k_per_split : Mp;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x16{};
    // loader: each matrix tile is 128 rows x 32 k = 512 chunks of 8 bf16; two per thread
    uint4 ra[2], rh[2], rl[2];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int idx = tid + q * 256;
            const int r = idx >> 2;
            const int c = (idx & 3) * 8;
            const int64_t gp = m0 + r;
            const int gn = n0 + r;
            ra[q] = gp < P ? *reinterpret_cast<const uint4*>(dQ + gp * Mp + k0 + c) : make_uint4(0, 0, 0, 0);
            rh[q] = gn < Mp ? *reinterpret_cast<const uint4*>(Vhi + (int64_t)gn * Mp + k0 + c) : make_uint4(0, 0, 0, 0);
            rl[q] = gn < Mp ? *reinterpret_cast<const uint4*>(Vlo + (int64_t)gn * Mp + k0 + c) : make_uint4(0, 0, 0, 0);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int idx = tid + q * 256;
            const int r = idx >> 2;
            const int c = (idx & 3) * 8;
            *reinterpret_cast<uint4*>(&As[buf][r][c]) = ra[q];
            *reinterpret_cast<uint4*>(&Hs[buf][r][c]) = rh[q];
            *reinterpret_cast<uint4*>(&Ls[buf][r][c]) = rl[q];
        }
    };
    if (kbeg < kend) {
        fetch(kbeg);
        stash(0);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += PB_BK) {
        const bool more = k0 + PB_BK < kend;
        if (more) fetch(k0 + PB_BK);
#pragma unroll
        for (int ks = 0; ks < PB_BK; ks += 16) {
            const int kk = ks + 8 * (lane >> 5);
            bf16x8 av[2], hv[2], lv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                av[a] = *reinterpret_cast<const bf16x8*>(&As[buf][wm * 64 + a * 32 + (lane & 31)][kk]);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                hv[b] = *reinterpret_cast<const bf16x8*>(&Hs[buf][wn * 64 + b * 32 + (lane & 31)][kk]);
                lv[b] = *reinterpret_cast<const bf16x8*>(&Ls[buf][wn * 64 + b * 32 + (lane & 31)][kk]);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], hv[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], lv[b], acc[a][b], 0, 0, 0);
                }
        }
        if (more) stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // epilogue: lane holds D[i][j] of each 32 x 32 block, j = lane % 32,
    // i = 8 (v / 4) + 4 (lane / 32) + v % 4
    const double first = split == 0 ? 1.0 : 0.0;
    double rows[2][16];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) rows[a][v] = 0.0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int gn = n0 + wn * 64 + b * 32 + (lane & 31);
        const bool okn = gn < M;
        const double htn = okn ? first * ht[gn] : 0.0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int64_t gp = m0 + wm * 64 + a * 32 + i;
                const double dqv = (okn && gp < P) ? (double)__bfloat162float(dQ[gp * Mp + gn]) : 0.0;
                rows[a][v] += dqv * (htn + 0.5 * (double)acc[a][b][v]);
            }
    }
    // sum over the 32 columns of the wave (lanes with equal lane / 32), fixed order
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            double x = rows[a][v];
#pragma unroll
            for (int o = 1; o < 32; o <<= 1) x += __shfl_xor(x, o, 64);
            rows[a][v] = x;
        }
    if ((lane & 31) == 0) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                red[wm * 64 + a * 32 + i][wn] = rows[a][v];
            }
    }
    __syncthreads();
    if (tid < PB_BM) {
        const int64_t gp = m0 + tid;
        if (gp < P) part[gp * n_tiles_total + (int64_t)blockIdx.x * gridDim.z + split] = red[tid][0] + red[tid][1];
    }
}

// E[p] = E~ + sum over column tiles of part[p][t], in tile order
__global__ void k_pop_finalize(int64_t P, int32_t n_tiles, const double* __restrict__ part, double E_t,
                               double* __restrict__ E) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double s = 0.0;
    for (int t = 0; t < n_tiles; ++t) s += part[p * n_tiles + t];
    E[p] = E_t + s;
}

// dQ[p][k] = bf16(charge[occ[p][mob[k]]] - c_{s(k)}), zero beyond M; grid (Mp/512, P),
// 8 consecutive k per thread written as one 16-byte store
__global__ void k_build_dq(int64_t P, int64_t n, int32_t M, int32_t Mp, int32_t E, const uint8_t* __restrict__ occ,
                           const int32_t* __restrict__ mob, const uint8_t* __restrict__ msub,
                           const double* __restrict__ dq, __hip_bfloat16* __restrict__ out) {
    const int64_t p = blockIdx.y;
    const int k0 = (blockIdx.x * blockDim.x + threadIdx.x) * 8;
    if (k0 >= Mp) return;
    __hip_bfloat16 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = k0 + q;
        float x = 0.0f;
        if (k < M) {
            const int e = occ[p * n + mob[k]];
            x = (float)dq[msub[k] * E + (e < E ? e : E - 1)];   // out-of-range ids read the last species
        }
        v[q] = __float2bfloat16(x);
    }
    *reinterpret_cast<uint4*>(out + p * Mp + k0) = *reinterpret_cast<const uint4*>(v);
}

// Q[p][k] = charge[occ[p][mob[k]]] (FP64), zero beyond M
__global__ void k_build_q64(int64_t P, int64_t n, int32_t M, int32_t Mp, int32_t E, const uint8_t* __restrict__ occ,
                            const int32_t* __restrict__ mob, const double* __restrict__ charge,
                            double* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * (int64_t)Mp) return;
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
                                                           const double* __restrict__ h, double E_ff,
                                                           double* __restrict__ E) {
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= P) return;
    double s = 0.0;
    for (int k = lane; k < M; k += 64) s += Q[p * Mp + k] * (h[k] + 0.5 * Phi[p * Mp + k]);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) E[p] = E_ff + s;
}

goac_status build_q64(goac_ctx* ctx, int64_t P, int64_t n, int32_t M, int32_t Mp, int32_t E, const uint8_t* occ,
                      const int32_t* mob, const double* charge, double* Q) {
    const int64_t tot = P * (int64_t)Mp;
    hipLaunchKernelGGL(k_build_q64, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, P, n, M, Mp, E,
                       occ, mob, charge, Q);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

goac_status energies_mixed(goac_problem* pb, int64_t P, const uint8_t* occ, double* E) {
    goac_ctx* ctx = pb->ctx;
    const ProblemDev& d = pb->d;
    const int32_t n_ntiles = (d.Mp + PB_BN - 1) / PB_BN;
    const int64_t m_tiles = (P + PB_BM - 1) / PB_BM;
    // split K until the grid covers the compute units (the epilogue is linear in Phi)
    int splits = 1;
    while ((int64_t)n_ntiles * m_tiles * splits < ctx->num_cus && d.Mp / (splits * 2) >= 256 && splits < 8)
        splits *= 2;
    const int32_t kps = (int32_t)round_up((d.Mp + splits - 1) / splits, PB_BK);
    const int32_t n_tiles_total = n_ntiles * splits;
    const size_t dq_bytes = round_up((size_t)P * d.Mp * sizeof(__hip_bfloat16), 256);
    const size_t part_bytes = (size_t)P * n_tiles_total * sizeof(double);
    void* ws = nullptr;
    goac_status st = workspace(ctx, 0, dq_bytes + part_bytes, &ws);
    if (st != GOAC_OK) return st;
    __hip_bfloat16* dQ = (__hip_bfloat16*)ws;
    double* part = (double*)((char*)ws + dq_bytes);
    hipLaunchKernelGGL(k_build_dq, dim3((unsigned)((d.Mp + 511) / 512), (unsigned)P), dim3(64), 0, ctx->stream, P,
                       d.n, d.M, d.Mp, d.E, occ, d.mob, d.msub, d.dq, dQ);
    GOAC_CHECK_LAUNCH(ctx);
    dim3 grid((unsigned)n_ntiles, (unsigned)m_tiles, (unsigned)splits);
    hipLaunchKernelGGL(k_pop_bf16, grid, dim3(256), 0, ctx->stream, P, d.M, d.Mp, dQ, d.Vhi, d.Vlo, d.ht, part,
                       n_tiles_total, kps);
    GOAC_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(k_pop_finalize, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, ctx->stream, P,
                       n_tiles_total, part, d.E_t, E);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

#define GOAC_TRY_(expr)                \
    do {                               \
        goac_status s_ = (expr);       \
        if (s_ != GOAC_OK) return s_;  \
    } while (0)

goac_status energies_fp64(goac_problem* pb, int64_t P, const uint8_t* occ, double* E) {
    goac_ctx* ctx = pb->ctx;
    const ProblemDev& d = pb->d;
    const size_t qb = round_up((size_t)P * d.Mp * sizeof(double), 256);
    void* ws = nullptr;
    goac_status st = workspace(ctx, 0, 2 * qb, &ws);
    if (st != GOAC_OK) return st;
    double* Q = (double*)ws;
    double* Phi = (double*)((char*)ws + qb);
    GOAC_TRY_(build_q64(ctx, P, d.n, d.M, d.Mp, d.E, occ, d.mob, d.charge, Q));
    st = dgemm_nt(ctx, P, d.M, d.Mp, Q, d.Mp, d.V64, d.Mp, Phi, d.Mp, 1.0, 0.0, nullptr);
    if (st != GOAC_OK) return st;
    hipLaunchKernelGGL(k_pop_fp64_finalize, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, ctx->stream, P, d.M,
                       d.Mp, Q, Phi, d.h, d.E_ff, E);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

}  // namespace goac
