// Best-swap descent to a local minimum on gfx950 (SI, "Gradient Descent").
//
// One workgroup per configuration. The mobile occupation, charges and the FP64
// field phi = h + V_mm q of the configuration live in LDS. A step scores every
// swap of two positions of one site class holding different species,
//   dE = d (phi_i - phi_j) + 1/2 d^2 (V_ii + V_jj - 2 V_ij),  d = q_j - q_i,
// streaming the upper triangle of V_mm row by row (the threads stride over the
// pairs numbered row by row, so rows are read coalesced and no lane idles): a
// first pass finds the lowest dE, a second pass the lexicographically first pair
// (i, j) whose dE lies within tol of it. The step
// applies that swap with the rank-2 field update; descent stops when the lowest
// dE is >= -tol or after max_steps swaps.
#include <climits>

#include "common.h"

namespace goac {

constexpr int kGdThreads = 256;

__device__ inline double gd_wave_sum(double x) {
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) x += __shfl_xor(x, s, 64);
    return x;
}

__global__ __launch_bounds__(kGdThreads) void k_gd(int64_t n, int32_t M, int32_t Mp, int32_t E,
                                                   const int32_t* __restrict__ mob,
                                                   const uint8_t* __restrict__ msub_g,
                                                   const double* __restrict__ V64, const double* __restrict__ diag,
                                                   const double* __restrict__ h, const double* __restrict__ charge,
                                                   const double* __restrict__ Ed, int64_t max_steps, double tol,
                                                   uint8_t* __restrict__ occ, int64_t* __restrict__ steps_out,
                                                   double* __restrict__ E_out) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ double s_red[kGdThreads / 64];
    __shared__ long long s_key[kGdThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = kGdThreads / 64;
    double* q = reinterpret_cast<double*>(lds);
    double* phi = q + Mp;
    uint8_t* om = reinterpret_cast<uint8_t*>(phi + Mp);
    uint8_t* ms = om + Mp;
    const int64_t p = blockIdx.x;
    uint8_t* row = occ + p * n;
    for (int k = tid; k < M; k += kGdThreads) {
        const uint8_t e = row[mob[k]];
        om[k] = e;
        ms[k] = msub_g[k];
        q[k] = charge[e < E ? e : E - 1];
    }
    __syncthreads();
    // phi_k = h_k + sum_l V_kl q_l: a wavefront per row, lanes over l, fixed butterfly
    for (int k = wave; k < M; k += NW) {
        const double* Vk = V64 + (int64_t)k * Mp;
        double s = 0.0;
        for (int l = lane; l < M; l += 64) s += Vk[l] * q[l];
        s = gd_wave_sum(s);
        if (lane == 0) phi[k] = h[k] + s;
    }
    __syncthreads();
    // E = E_ff + 1/2 sum_k q_k (phi_k + h_k)
    double e_part = 0.0;
    for (int k = tid; k < M; k += kGdThreads) e_part += q[k] * (phi[k] + h[k]);
    e_part = gd_wave_sum(e_part);
    if (lane == 0) s_red[wave] = e_part;
    __syncthreads();
    double Ecur = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) Ecur += s_red[w];
    Ecur = Ed[0] + 0.5 * Ecur;
    __syncthreads();

    auto score = [&](int i, int j, double& dE) -> bool {
        if (ms[i] != ms[j] || om[i] == om[j]) return false;
        const double d = q[j] - q[i];
        dE = d * (phi[i] - phi[j]) + 0.5 * d * d * (diag[i] + diag[j] - 2.0 * V64[(int64_t)i * Mp + j]);
        return true;
    };

    // pair (i, i + 1 + r): carry r past the end of row i into the next rows; false
    // once the rows are exhausted
    auto next_pair = [&](int& i, int& r) -> bool {
        while (i < M - 1 && r > M - 2 - i) {
            r -= M - 1 - i;
            ++i;
        }
        return i < M - 1;
    };

    int64_t st = 0;
    while (st < max_steps) {
        // pass 1: lowest dE. The pairs i < j are numbered row by row and the threads
        // stride over that numbering, so every lane has a pair in every iteration.
        double lo = INFINITY;
        for (int i = 0, r = tid; next_pair(i, r);) {
            double dE;
            if (score(i, i + 1 + r, dE)) lo = fmin(lo, dE);
            r += kGdThreads;
        }
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) lo = fmin(lo, __shfl_xor(lo, s, 64));
        if (lane == 0) s_red[wave] = lo;
        __syncthreads();
        lo = s_red[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) lo = fmin(lo, s_red[w]);
        __syncthreads();
        if (!(lo < -tol)) break;
        // pass 2: lexicographically first pair within tol of the lowest
        const double thr = lo + tol;
        long long key = LLONG_MAX;
        for (int i = 0, r = tid; next_pair(i, r);) {   // a thread's pairs in order
            double dE;
            const int j = i + 1 + r;
            if (score(i, j, dE) && dE <= thr) {
                key = (long long)i * M + j;
                break;
            }
            r += kGdThreads;
        }
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) {
            const long long o = __shfl_xor(key, s, 64);
            key = o < key ? o : key;
        }
        if (lane == 0) s_key[wave] = key;
        __syncthreads();
        key = s_key[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) key = s_key[w] < key ? s_key[w] : key;
        const int bi = (int)(key / M), bj = (int)(key % M);
        double dEb = 0.0;
        score(bi, bj, dEb);
        const double d = q[bj] - q[bi];
        __syncthreads();
        // apply: swap the species and charges, rank-2 field update
        for (int k = tid; k < M; k += kGdThreads)
            phi[k] += d * (V64[(int64_t)bi * Mp + k] - V64[(int64_t)bj * Mp + k]);
        if (tid == 0) {
            const uint8_t t = om[bi];
            om[bi] = om[bj];
            om[bj] = t;
            const double tq = q[bi];
            q[bi] = q[bj];
            q[bj] = tq;
        }
        Ecur += dEb;
        ++st;
        __syncthreads();
    }
    for (int k = tid; k < M; k += kGdThreads) row[mob[k]] = om[k];
    if (tid == 0) {
        if (steps_out) steps_out[p] = st;
        if (E_out) E_out[p] = Ecur;
    }
}

}  // namespace goac

using namespace goac;

extern "C" goac_status goac_gd_run(goac_problem* pb, int64_t P, uint8_t* occ_dev, int64_t max_steps, double tol,
                                   int64_t* steps_dev, double* E_dev) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (P < 0 || (P > 0 && !occ_dev) || max_steps < 0 || !(tol >= 0.0))
        return fail(ctx, GOAC_EINVAL, "gd_run: bad arguments");
    if (P == 0) return GOAC_OK;
    if (P >= (int64_t)1 << 31) return fail(ctx, GOAC_EINVAL, "gd_run: population too large");
    const ProblemDev& d = pb->d;
    const size_t lds = (size_t)d.Mp * (2 * sizeof(double) + 2);
    if (lds > 160 * 1024 - 1024) return fail(ctx, GOAC_EINVAL, "gd_run: too many mobile positions for one workgroup");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    GOAC_TRY(rows_check(pb, P, occ_dev, "gd_run"));
    if (lds > 64 * 1024)
        GOAC_HIP(ctx, hipFuncSetAttribute((const void*)k_gd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_gd, dim3((unsigned)P), dim3(kGdThreads), lds, ctx->stream, d.n, d.M, d.Mp, d.E, d.mob,
                       d.msub, d.V64, d.diag, d.h, d.charge, d.Ed, max_steps, tol, occ_dev, steps_dev, E_dev);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}
