// Metropolis swap Monte Carlo on gfx950 (SI, "Monte Carlo", "Simulated annealing").
//
// One workgroup runs one chain at a time; a persistent grid pulls chains from a
// work counter in longest-first order. A chain's field phi, its occupation and
// its per-sublattice position lists live in LDS for the whole launch.
//
// Trials are evaluated speculatively: the WG lanes score the next WG trial
// indices t, t+1, ... against the current state at once (Philox draw, partner
// pick, dE from phi and three gathered matrix entries, Metropolis test). Since
// rejected trials leave the state unchanged, every trial up to the first one that
// may be accepted (found with a wavefront ballot) is final; that trial is
// resolved, applied (rank-2 field update streaming rows i and j of V_mm), and
// the window restarts after it. The result is exactly the sequential chain.
//
// MIXED keeps phi' = phi - phibar_s (a per-instance constant per sublattice that
// cancels in every same-sublattice swap) in FP32 and streams FP32 rows; a running
// rigorous bound eps on |phi'32 - phi'| makes the FP32 decision final only when
// the FP64 decision cannot differ; otherwise phi_i - phi_j is recomputed in FP64.
// The field is re-anchored in FP64 after reanchor_every field updates.
#include "common.h"

namespace goac {

template <typename T>
struct Bcast {
    int i, j;
    int unsure, pad;
    double d, dE, u, kT;
};

__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) x += __shfl_xor(x, s, 64);
    return x;
}
__device__ inline double wave_max(double x) {
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) x = fmax(x, __shfl_xor(x, s, 64));
    return x;
}
__device__ inline uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) x += __shfl_xor(x, s, 64);
    return x;
}

// WG reductions through a small LDS scratch (NW doubles per value); all threads
// return the result. Callers are uniform.
template <int WG>
__device__ inline double wg_sum(double x, double* scr) {
    constexpr int NW = WG / 64;
    x = wave_sum(x);
    if (NW == 1) return x;
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scr[w] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) s += scr[q];
    return s;
}
template <int WG>
__device__ inline double wg_max(double x, double* scr) {
    constexpr int NW = WG / 64;
    x = wave_max(x);
    if (NW == 1) return x;
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scr[w] = x;
    __syncthreads();
    double s = scr[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) s = fmax(s, scr[q]);
    return s;
}

constexpr double kU32 = 0x1p-24;      // unit roundoff of FP32
constexpr double kMargin = 1e-8;      // eV: covers the reference FP64 chain's own rounding

// FP64 anchor of a chain: phi_k = h_k + sum_l V64[l][k] q_l (V symmetric, so the
// column walk is coalesced), phi' = phi - phibar_s stored as FP32; returns the new
// energy E = E_ff + 1/2 sum q_k (phi_k + h_k) and the error bound eps of phi'32.
template <int WG>
__device__ void anchor_chain(const McInst& I, const uint8_t* occ, const uint8_t* msub, const double* chg,
                             const double* phibar, float* phi, double* scr, double& E_out, double& eps_out,
                             float& phib_out) {
    const int M = I.M;
    const GOAC_GLOBAL double* V64 = gptr(I.V64);
    const GOAC_GLOBAL double* hv = gptr(I.h);
    double esum = 0.0, pmax = 0.0, amax = 0.0;
    for (int k0 = 0; k0 < M; k0 += WG) {
        const int k = k0 + threadIdx.x;
        const bool ok = k < M;
        double acc = ok ? hv[k] : 0.0;
        double aab = ok ? fabs(acc) : 0.0;
        for (int l = 0; l < M; ++l) {
            const double ql = chg[occ[l]];
            if (ok) {
                const double v = V64[(int64_t)l * I.Mp + k];
                acc += v * ql;
                aab += fabs(v * ql);
            }
        }
        if (ok) {
            const double hk = hv[k];
            const double qk = chg[occ[k]];
            esum += qk * (acc + hk);
            const float p = (float)(acc - phibar[msub[k]]);
            phi[k] = p;
            pmax = fmax(pmax, fabs((double)p));
            amax = fmax(amax, aab);
        }
    }
    esum = wg_sum<WG>(esum, scr);
    pmax = wg_max<WG>(pmax, scr);
    amax = wg_max<WG>(amax, scr);
    E_out = I.E_ff + 0.5 * esum;
    // FP64 dot error (gamma_M times the absolute sum) plus FP32 rounding of phi'
    const double gM = (double)(M + 2) * 0x1p-53 * 1.01;
    eps_out = kU32 * pmax * 1.0001 + gM * amax * 2.0;
    float pb = 1.0f;
    while ((double)pb < 2.0 * pmax) pb *= 2.0f;
    phib_out = pb;
}

template <bool MIXED, int WG, bool TRACE>
__global__ __launch_bounds__(WG) void k_mc(McArgs a) {
    using T = typename std::conditional<MIXED, float, double>::type;
    constexpr int NW = WG / 64;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int s_item;
    __shared__ int s_first[2][NW];
    __shared__ Bcast<T> s_b;
    __shared__ double s_scr[NW > 1 ? NW : 1];
    __shared__ double s_phibar[kMaxSub];
    __shared__ int s_flag;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    T* phi = reinterpret_cast<T*>(lds);
    uint8_t* occ = lds + a.lds_phi_bytes;
    uint8_t* msub = occ + a.Mp_max;
    uint16_t* perm = reinterpret_cast<uint16_t*>(msub + a.Mp_max);
    uint16_t* where = perm + a.Mp_max;
    int32_t* tab = reinterpret_cast<int32_t*>(where + a.Mp_max);
    double* chg = reinterpret_cast<double*>(tab + a.tab_max);

    if (tid == 0) s_flag = 0;
    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = atomicAdd(a.queue, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= a.n_items) return;
        const int c = a.order ? a.order[item] : item;
        ChainScalars* sc = a.sc + c;
        const int inst = sc->inst;
        const McInst I = a.insts[inst];
        const int M = I.M, Mp = I.Mp, S = I.S, E = I.E;
        const int64_t off = sc->off;
        GOAC_GLOBAL T* gphi = gptr_rw(reinterpret_cast<T*>(a.phi) + off);
        GOAC_GLOBAL uint8_t* gocc = gptr_rw(a.occ + off);
        GOAC_GLOBAL uint16_t* gperm = gptr_rw(a.perm + off);
        GOAC_GLOBAL uint8_t* gbest = gptr_rw(a.best + off);
        const GOAC_GLOBAL double* V64 = gptr(I.V64);
        const GOAC_GLOBAL float* V32 = gptr(I.V32);
        const GOAC_GLOBAL double* diag = gptr(I.diag);
        const GOAC_GLOBAL float* rowmax = gptr(I.rowmax);
        const GOAC_GLOBAL double* hv = gptr(I.h);
        const int ntab = tab_words(S, E);
        // ---- load the chain into LDS
        for (int k = tid; k < Mp; k += WG) {
            phi[k] = gphi[k];
            occ[k] = gocc[k];
            msub[k] = gptr(I.msub)[k];
            const uint16_t p = gperm[k];
            perm[k] = p;
        }
        for (int k = tid; k < ntab; k += WG) tab[k] = gptr(I.tab)[k];
        for (int k = tid; k < E; k += WG) chg[k] = gptr(I.charge)[k];
        __syncthreads();
        for (int k = tid; k < M; k += WG) where[perm[k]] = (uint16_t)k;
        if (MIXED && tid < S) s_phibar[tid] = gptr(I.phibar)[tid];
        __syncthreads();
        const int32_t* subsize = tab + 2;
        const int32_t* suboff = subsize + S;
        const int32_t* cnt = suboff + S;
        const int32_t* offs = cnt + S * E;

        uint64_t t = sc->t;
        const uint64_t t_end = t + a.n_trials;
        double Ecur = sc->E, best = sc->best_E;
        uint64_t n_acc = sc->accepts, n_upd = sc->updates, n_fb = sc->fallbacks, n_anc = sc->anchors;
        double eps = sc->eps;
        float phib = sc->phibound;
        uint32_t since = sc->since_anchor;
        int status = sc->status;
        const GOAC_GLOBAL double* kTrow = gptr(a.kT + (int64_t)sc->row * a.n_blocks);
        const uint32_t chain_id = sc->chain_id;
        const uint32_t w3 = (I.instance << 8) | TAG_MC;
        uint64_t hsum = 0;
        int parity = 0;

        // temperature block of the window start; a window of WG <= block_len trials
        // crosses at most one block boundary (otherwise each lane divides)
        uint64_t blk0 = t / a.block_len;
        uint64_t bnd = (blk0 + 1) * a.block_len;
        const bool wide_blocks = a.block_len >= (uint64_t)WG;
        const uint64_t nb1 = (uint64_t)(a.n_blocks - 1);
        while (t < t_end) {
            const uint64_t tl = t + (uint64_t)tid;
            const bool valid = tl < t_end;
            double kT;
            if (wide_blocks) {
                const double kT0 = kTrow[blk0 < nb1 ? blk0 : nb1];
                const double kT1 = kTrow[blk0 + 1 < nb1 ? blk0 + 1 : nb1];
                kT = tl >= bnd ? kT1 : kT0;
            } else {
                const uint64_t blk = tl / a.block_len;
                kT = kTrow[blk < nb1 ? blk : nb1];
            }
            const u32x4 r = philox((uint32_t)tl, (uint32_t)(tl >> 32), chain_id, w3, a.seed);
            const int i = (int)mulshift(r.x, (uint32_t)M);
            const int s = S == 1 ? 0 : msub[i];
            const int sa = occ[i];
            const int na = cnt[s * E + sa];
            const int csz = subsize[s] - na;
            int j = i;
            bool stop = false, unsure = false;
            double d = 0.0, dE = 0.0;
            if (valid && csz > 0) {
                const int k = (int)mulshift(r.y, (uint32_t)csz);
                const int idx = k < offs[s * E + sa] ? k : k + na;
                j = perm[suboff[s] + idx];
                const int sb = occ[j];
                d = chg[sb] - chg[sa];
                const double phi_i = (double)phi[i], phi_j = (double)phi[j];
                const double Vii = diag[i], Vjj = diag[j];
                const double Vij = V64[(int64_t)i * Mp + j];
                dE = d * (phi_i - phi_j) + 0.5 * d * d * (Vii + Vjj - 2.0 * Vij);
                // Metropolis threshold L = -kT ln u, first in FP32 from the top 24 bits
                // of u: |L32 - L| <= m32 (u32 within 2^-25 of u, log within 2^-20 relative);
                // tests closer than m32 to the threshold use the exact FP64 rule
                const uint32_t ub = r.z >> 8;
                const float u32 = ((float)ub + 0.5f) * 0x1p-24f;
                const float lg = __logf(u32);
                const float kTf = (float)kT;
                const double L32 = (double)(-kTf * lg);
                const double m32 = ub < 2 ? INFINITY : (double)(kTf * (0x1p-24f / u32 + 0x1p-20f * (1.0f - lg)));
                if constexpr (MIXED) {
                    const double e = d != 0.0 ? 2.0 * fabs(d) * eps + kMargin : 0.0;
                    const double hi = dE + e, lo = dE - e;
                    const bool sure_acc = (hi <= 0.0) || (hi - L32 < -m32);
                    const bool sure_rej = (lo > 0.0) && (lo - L32 > m32);
                    unsure = !sure_acc && !sure_rej;
                    stop = sure_acc || unsure;
                } else {
                    bool acc;
                    if (dE <= 0.0) acc = true;
                    else if (dE - L32 < -m32) acc = true;
                    else if (dE - L32 > m32) acc = false;
                    else acc = unit_open(r.z, r.w) < exp(-dE / kT);
                    stop = acc;
                }
            }
            // first trial of the window that may be accepted
            const uint64_t mask = __ballot(stop);
            int f;
            if (NW == 1) {
                f = mask ? (int)__ffsll((long long)mask) - 1 : WG;
            } else {
                if (lane == 0) s_first[parity][wave] = mask ? wave * 64 + (int)__ffsll((long long)mask) - 1 : WG;
                __syncthreads();
                f = WG;
#pragma unroll
                for (int q = 0; q < NW; ++q) f = min(f, s_first[parity][q]);
                parity ^= 1;
            }
            const uint64_t left = t_end - t;
            const int nvalid = left < (uint64_t)WG ? (int)left : WG;
            if (TRACE && valid && tid < f) hsum += trial_hash(tl, (uint32_t)i, (uint32_t)j, 0u);
            if (f >= nvalid) {
                t += (uint64_t)nvalid;
                while (t >= bnd) { ++blk0; bnd += a.block_len; }
                continue;
            }
            if (tid == f) {
                s_b.i = i; s_b.j = j; s_b.unsure = unsure ? 1 : 0;
                s_b.d = d; s_b.dE = dE; s_b.u = unit_open(r.z, r.w); s_b.kT = kT;
            }
            __syncthreads();
            const int bi = s_b.i, bj = s_b.j;
            const double bd = s_b.d;
            double bdE = s_b.dE;
            bool accf = true;
            if (MIXED && s_b.unsure) {  // (never true for FP64)
                // exact FP64 difference phi_i - phi_j from the occupation
                double part = 0.0;
                for (int k = tid; k < M; k += WG)
                    part += (V64[(int64_t)bi * Mp + k] - V64[(int64_t)bj * Mp + k]) * chg[occ[k]];
                const double diff = wg_sum<WG>(part, s_scr) + (hv[bi] - hv[bj]);
                const double Vii = diag[bi], Vjj = diag[bj];
                const double Vij = V64[(int64_t)bi * Mp + bj];
                bdE = bd * diff + 0.5 * bd * bd * (Vii + Vjj - 2.0 * Vij);
                accf = (bdE <= 0.0) || (s_b.u < exp(-bdE / s_b.kT));
                ++n_fb;
            }
            if (TRACE && tid == f) hsum += trial_hash(tl, (uint32_t)bi, (uint32_t)bj, accf ? 1u : 0u);
            if (accf) {
                if (bd != 0.0) {
                    const T dd = (T)bd;
                    const GOAC_GLOBAL T* Vi;
                    const GOAC_GLOBAL T* Vj;
                    if constexpr (MIXED) {
                        Vi = V32 + (int64_t)bi * Mp;
                        Vj = V32 + (int64_t)bj * Mp;
                    } else {
                        Vi = V64 + (int64_t)bi * Mp;
                        Vj = V64 + (int64_t)bj * Mp;
                    }
                    bool over = false;
                    constexpr int VEC = MIXED ? 4 : 2;
                    for (int k = tid * VEC; k < Mp; k += WG * VEC) {
#pragma unroll
                        for (int q = 0; q < VEC; ++q) {
                            T p = phi[k + q];
                            if constexpr (MIXED) {
                                p = fmaf(dd, Vi[k + q], p);
                                p = fmaf(-dd, Vj[k + q], p);
                                over |= fabsf(p) > phib;
                            } else {
                                p = p + dd * (Vi[k + q] - Vj[k + q]);
                            }
                            phi[k + q] = p;
                        }
                    }
                    if (MIXED && over) s_flag = 1;
                    ++n_upd;
                    ++since;
                }
                if (tid == 0) {
                    const uint8_t sa = occ[bi], sb = occ[bj];
                    occ[bi] = sb;
                    occ[bj] = sa;
                    const uint16_t wi = where[bi], wj = where[bj];
                    perm[wi] = (uint16_t)bj;
                    perm[wj] = (uint16_t)bi;
                    where[bi] = wj;
                    where[bj] = wi;
                }
                Ecur += bdE;
                ++n_acc;
                __syncthreads();
                if constexpr (MIXED) if (bd != 0.0) {
                    const int flag = s_flag;
                    if (flag) {
                        // |phi'| grew past the bound: take the exact maximum
                        double pm = 0.0;
                        for (int k = tid; k < M; k += WG) pm = fmax(pm, fabs((double)phi[k]));
                        pm = wg_max<WG>(pm, s_scr);
                        float pb = phib;
                        while ((double)pb < 2.0 * pm) pb *= 2.0f;
                        phib = pb;
                        __syncthreads();
                        if (tid == 0) s_flag = 0;
                    }
                    // two fused multiply-adds per element, each rounding <= u |intermediate|,
                    // plus the FP32 rounding of the two V entries
                    const double rmi = (double)rowmax[bi], rmj = (double)rowmax[bj];
                    const double ad = fabs(bd);
                    eps += kU32 * (2.0 * (double)phib + ad * (rmi + 2.0 * (rmi + rmj))) * 1.0001;
                    if (!(eps < 1e3)) status = 1;
                    if (since >= (uint32_t)a.reanchor_every) {
                        __syncthreads();
                        anchor_chain<WG>(I, occ, msub, chg, s_phibar, reinterpret_cast<float*>(phi), s_scr, Ecur,
                                         eps, phib);
                        since = 0;
                        ++n_anc;
                        __syncthreads();
                    }
                }
                if (Ecur < best) {
                    best = Ecur;
                    for (int k = tid; k < Mp; k += WG) gbest[k] = occ[k];
                }
            }
            t += (uint64_t)(f + 1);
            while (t >= bnd) { ++blk0; bnd += a.block_len; }
        }
        // ---- write the chain back
        __syncthreads();
        for (int k = tid; k < Mp; k += WG) {
            gphi[k] = phi[k];
            gocc[k] = occ[k];
            gperm[k] = perm[k];
        }
        if (TRACE) {
            uint64_t hs = wave_sum_u64(hsum);
            if (NW > 1) {
                __shared__ uint64_t s_h[NW > 1 ? NW : 1];
                if (lane == 0) s_h[wave] = hs;
                __syncthreads();
                hs = 0;
                for (int q = 0; q < NW; ++q) hs += s_h[q];
            }
            hsum = hs;
        }
        if (tid == 0) {
            sc->t = t;
            sc->E = Ecur;
            sc->best_E = best;
            sc->accepts = n_acc;
            sc->updates = n_upd;
            sc->fallbacks = n_fb;
            sc->anchors = n_anc;
            sc->eps = eps;
            sc->phibound = phib;
            sc->since_anchor = since;
            sc->status = status;
            if (TRACE) sc->hash += hsum;
        }
    }
}

// ------------------------------------------------------------------ launch
template <bool MIXED, int WG, bool TRACE>
static goac_status launch_mc(goac_ctx* ctx, const McArgs& a, size_t lds, int grid) {
    auto kern = k_mc<MIXED, WG, TRACE>;
    if (lds > 64 * 1024) GOAC_HIP(ctx, hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(WG), lds, ctx->stream, a);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

goac_status mc_launch(goac_ctx* ctx, const McArgs& a, bool mixed, bool trace, int wg, size_t lds, int grid) {
#define GOAC_MC_CASE(MX, W, TR) \
    if (mixed == MX && wg == W && trace == TR) return launch_mc<MX, W, TR>(ctx, a, lds, grid);
    GOAC_MC_CASE(false, 64, false)
    GOAC_MC_CASE(false, 64, true)
    GOAC_MC_CASE(true, 64, false)
    GOAC_MC_CASE(true, 64, true)
    GOAC_MC_CASE(false, 256, false)
    GOAC_MC_CASE(false, 256, true)
    GOAC_MC_CASE(true, 256, false)
    GOAC_MC_CASE(true, 256, true)
#undef GOAC_MC_CASE
    return fail(ctx, GOAC_EINVAL, "unsupported Monte Carlo workgroup size");
}

}  // namespace goac
