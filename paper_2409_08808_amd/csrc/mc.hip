// Metropolis swap Monte Carlo on gfx950 (SI, "Monte Carlo", "Simulated annealing").
//
// One workgroup runs one chain at a time; a persistent grid pulls chains from a
// work counter in longest-first order. A chain's field phi, its occupation and
// its per-sublattice position lists live in LDS for the whole launch (one-wave
// chains also keep the diagonal V_kk there, two of the three per-trial gathers).
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
// The field is re-anchored in FP64 after reanchor_every field updates: inside the
// kernel for small cells (one pass over V_mm per chain), or, for large cells, by a
// batched FP64 matrix-core product between chunks of trials (k_anchor_* below),
// which reads V_mm once for all due chains. The error bound stays rigorous while a
// chain waits for its anchor; only the fallback rate grows.
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

// Bounds of the Metropolis threshold L = -kT ln u (u = unit_open(r.z, r.w)) from
// the top 24 bits ub of u, in FP32:
//   thr = kT32 (-lg2 kLn2Up + b) >= L,   lo = kT32 (-lg2 kLn2Dn - b) <= L (ub >= 2)
// with u32 = (ub + 1/2) 2^-24, lg2 the hardware log2(u32), ri >= 1/u32 the power of
// two read off u32's exponent and b = 2^-24 ri + 2^-20. For ub >= 2, u lies within
// 2^-25 of u32, so |ln u - ln u32| <= 0.625 2^-24 / u32, which the 2^-24 ri term
// covers; the relative errors (log2 within 2^-23, kT32, the fma and the product,
// 2^-24 each) stay below the 2^-20 of kLn2Up / kLn2Dn around ln 2, and the
// absolute 2^-20 kT32 covers the log near u = 1. Trials with ub < 2 always stop.
constexpr float kLn2Up = 0x1.62e448p-1f;  // >= ln 2 (1 + 2^-20)
constexpr float kLn2Dn = 0x1.62e418p-1f;  // <= ln 2 (1 - 2^-20)
// a uniform pointer held in scalar registers
template <typename P>
__device__ __forceinline__ P* sptr(P* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (P*)(((uint64_t)hi << 32) | lo);
}

// element x of a global array; with OFF32 through a 32-bit byte offset (arrays
// below 4 GiB, which the host guarantees for one-wave chains)
template <bool OFF32, typename T>
__device__ __forceinline__ T gather(const GOAC_GLOBAL T* base, uint32_t x) {
    if constexpr (OFF32)
        return *reinterpret_cast<const GOAC_GLOBAL T*>(reinterpret_cast<const GOAC_GLOBAL char*>(base) +
                                                       (uint32_t)(x * (uint32_t)sizeof(T)));
    else
        return base[(uint64_t)x];
}

// kT of the filter in FP32; below 2^-100 the bounds could lose their range, so the
// filter then passes every trial to the exact rule
__device__ __forceinline__ float kt_filter(double kT) { return kT >= 0x1p-100 ? (float)kT : INFINITY; }
__device__ __forceinline__ void metropolis_band(uint32_t ub, float& lg2, float& b) {
    const float u32 = fmaf((float)ub, 0x1p-24f, 0x1p-25f);
    lg2 = __builtin_amdgcn_logf(u32);
    const float ri = __uint_as_float(0x7f000000u - (__float_as_uint(u32) & 0x7f800000u));
    b = fmaf(ri, 0x1p-24f, 0x1p-20f);
}

// FP64 anchor of a chain: phi_k = h_k + sum_l V64[l][k] q_l (V symmetric, so the
// column walk is coalesced), phi' = phi - phibar_s stored as FP32; returns the new
// energy E = E_ff + 1/2 sum q_k (phi_k + h_k) and the error bound eps of phi'32.
template <int WG>
__device__ void anchor_chain(const McInst& I, const uint8_t* occ, const uint8_t* msub, const double* chg,
                             const double* phibar, float* phi, double* scr, double& E_out, double& eps_out,
                             float& phib_out) {
    const int M = I.M;
    const GOAC_GLOBAL double* V64 = gptr(sptr(I.V64));
    const GOAC_GLOBAL double* hv = gptr(I.h);
    // in-kernel anchors run for cells of at most 1024 positions: 32-bit byte offsets
    const uint32_t rs = (uint32_t)I.Mp;
    double esum = 0.0, pmax = 0.0, amax = 0.0;
    for (int k0 = 0; k0 < M; k0 += WG) {
        const int k = k0 + threadIdx.x;
        const bool ok = k < M;
        double acc = ok ? hv[k] : 0.0;
        double aab = ok ? fabs(acc) : 0.0;
        // the sum runs over l in order; U rows are loaded ahead of it so that a
        // one-wave chain keeps U loads in flight (one more U-fold unroll costs the
        // trial loop scalar registers)
        constexpr int U = 4;
        int l = 0;
        uint32_t o = (uint32_t)k;   // element (l, k)
        for (; l + U <= M; l += U) {
            double v[U], q[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                q[u] = chg[occ[l + u]];
                v[u] = ok ? gather<true>(V64, o) : 0.0;
                o += rs;
            }
            if (ok) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    acc += v[u] * q[u];
                    aab += fabs(v[u] * q[u]);
                }
            }
        }
        for (; l < M; ++l) {
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
            const float p = (float)(acc - phibar[I.S == 1 ? 0 : msub[k]]);
            phi[k] = p;
            pmax = fmax(pmax, fabs((double)p));
            amax = fmax(amax, aab);
        }
    }
    esum = wg_sum<WG>(esum, scr);
    pmax = wg_max<WG>(pmax, scr);
    amax = wg_max<WG>(amax, scr);
    E_out = I.Ed[0] + 0.5 * esum;
    // FP64 dot error (gamma_M times the absolute sum) plus FP32 rounding of phi'
    const double gM = (double)(M + 2) * 0x1p-53 * 1.01;
    eps_out = kU32 * pmax * 1.0001 + gM * amax * 2.0;
    float pb = 1.0f;
    while ((double)pb < 2.0 * pmax) pb *= 2.0f;
    phib_out = pb;
}

// small cells run one wave per chain and want 4 resident waves per SIMD (<= 128
// VGPRs); large cells run 4 waves per chain and are bounded by LDS
template <bool MIXED, int WG, bool TRACE>
__global__ __launch_bounds__(WG, WG == 64 ? 4 : 2) void k_mc(McArgs a) {
    using T = typename std::conditional<MIXED, float, double>::type;
    constexpr int NW = WG / 64;
    // several waves per chain (large cells, where accepted trials are frequent and
    // a window's scoring costs the most) go on within a window after an accepted
    // trial; one-wave chains start the next window instead (fewer live registers)
    constexpr bool INWIN = NW > 1;
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
    // site-class ids take LDS only when some instance has more than one class
    uint8_t* msub = occ + a.Mp_max;
    uint16_t* perm = reinterpret_cast<uint16_t*>(msub + (a.msub_lds ? a.Mp_max : 0));
    uint16_t* where = perm + a.Mp_max;
    int32_t* tab = reinterpret_cast<int32_t*>(where + a.Mp_max);
    double* chg = reinterpret_cast<double*>(tab + a.tab_max);
    double* dgl = chg + kMaxSpecies;   // one-wave chains: the diagonal V_kk of the instance
    // multi-wave chains: the accepted swaps since the last best-occupation copy
    uint32_t* blog = reinterpret_cast<uint32_t*>(chg + kMaxSpecies);

    if (tid == 0) s_flag = 0;
    for (int round = 0;; ++round) {
        // a workgroup's first chain is its block index; later ones come from the
        // work counter, used only when there are more chains than workgroups
        int item = (int)blockIdx.x;
        if (round > 0) {
            if ((int)gridDim.x >= a.n_items) return;
            __syncthreads();
            if (tid == 0) s_item = (int)gridDim.x + atomicAdd(a.queue, 1);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_item);
        }
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
        // the per-trial gathers take their bases from scalar registers
        const GOAC_GLOBAL double* V64 = gptr(sptr(I.V64));
        const GOAC_GLOBAL float* V32 = gptr(sptr(I.V32));
        const GOAC_GLOBAL double* diag = gptr(sptr(I.diag));
        const GOAC_GLOBAL float* rowmax = gptr(I.rowmax);
        const GOAC_GLOBAL double* hv = gptr(I.h);
        const int ntab = tab_words(S, E);
        // ---- load the chain into LDS
        for (int k = tid; k < Mp; k += WG) {
            phi[k] = gphi[k];
            occ[k] = gocc[k];
            if (S > 1) msub[k] = gptr(I.msub)[k];
            const uint16_t p = gperm[k];
            perm[k] = p;
        }
        for (int k = tid; k < ntab; k += WG) tab[k] = gptr(I.tab)[k];
        for (int k = tid; k < E; k += WG) chg[k] = gptr(I.charge)[k];
        if constexpr (WG == 64) for (int k = tid; k < M; k += WG) dgl[k] = diag[k];
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
        bool best_dirty = false;   // occ is the best occupation and gbest not yet updated
        // occ -> gbest. One-wave chains (small cells) copy all of it in 32-bit words
        // (M_p is a multiple of 64, both 16-byte aligned). Multi-wave chains log the
        // accepted swaps since the last copy and write only the positions they
        // touched; the first copy of a launch, or one after the log overflowed, is
        // a full one.
        int blog_n = 0;
        bool blog_full = true;
        auto copy_best = [&]() {
            if (NW == 1 || blog_full) {
                const uint32_t* src = reinterpret_cast<const uint32_t*>(occ);
                GOAC_GLOBAL uint32_t* dst = reinterpret_cast<GOAC_GLOBAL uint32_t*>(gbest);
                for (int k = tid; k < Mp / 4; k += WG) dst[k] = src[k];
            } else {
                for (int e = tid; e < blog_n; e += WG) {
                    const uint32_t u = blog[e];
                    const uint32_t p = u & 0xffffu, q = u >> 16;
                    gbest[p] = occ[p];
                    gbest[q] = occ[q];
                }
            }
            blog_n = 0;
            blog_full = false;
        };
        uint64_t n_acc = sc->accepts, n_upd = sc->updates, n_fb = sc->fallbacks, n_anc = sc->anchors;
        double eps = sc->eps;
        float phib = sc->phibound;
        // MIXED: the largest |V_kl| of any row, for the error bound of an update
        double rmax = 0.0;
        if constexpr (MIXED) {
            for (int k = tid; k < M; k += WG) rmax = fmax(rmax, (double)rowmax[k]);
            rmax = wg_max<WG>(rmax, s_scr);
        }
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
        double kT0 = 0.0, kT1 = 0.0;   // temperatures of blocks blk0 and blk0 + 1
        float kTf0 = 0.0f, kTf1 = 0.0f;
        uint64_t kblk = ~(uint64_t)0;
        double eps2 = 2.0 * eps;
        while (t < t_end) {
            const uint64_t left = t_end - t;
            const int nvalid = left < (uint64_t)WG ? (int)left : WG;
            // lanes from `split` on lie in block blk0 + 1
            int split = WG;
            float kTf;
            if (wide_blocks) {
                if (blk0 != kblk) {
                    kT0 = kTrow[blk0 < nb1 ? blk0 : nb1];
                    kT1 = kTrow[blk0 + 1 < nb1 ? blk0 + 1 : nb1];
                    kTf0 = kt_filter(kT0);
                    kTf1 = kt_filter(kT1);
                    kblk = blk0;
                }
                const uint64_t rel = bnd - t;
                split = rel < (uint64_t)WG ? (int)rel : WG;
                kTf = tid < split ? kTf0 : kTf1;
            } else {
                const uint64_t blk = (t + (uint64_t)tid) / a.block_len;
                kTf = kt_filter(kTrow[blk < nb1 ? blk : nb1]);
            }
            const u32x4 r = [&] {
                const uint64_t tl = t + (uint64_t)tid;
                return philox((uint32_t)tl, (uint32_t)(tl >> 32), chain_id, w3, a.seed);
            }();
            // Metropolis threshold L = -kT ln u: FP32 bounds lo <= L <= thr from the
            // top 24 bits of u (metropolis_band); trials with ub < 2 always stop
            const uint32_t ub = r.z >> 8;
            float thr, lo;
            {
                float lg2, b;
                metropolis_band(ub, lg2, b);
                thr = kTf * fmaf(-lg2, kLn2Up, b);
                lo = (ub >= 2 && kTf < INFINITY) ? kTf * fmaf(-lg2, kLn2Dn, -b) : -INFINITY;
            }
            // the trial's swap (i, j) against the current state: d = q_j - q_i and
            // dE = d (phi_i - phi_j) + quad, quad = 1/2 d^2 (V_ii + V_jj - 2 V_ij).
            // Scored without a branch: with csz == 0 the pick reads an in-range slot
            // (perm is followed by where in LDS) and j falls back to i; such lanes and
            // lanes past the end never stop.
            int i, j, csz;
            double d, quad, dE;
            auto score = [&]() {
                i = (int)mulshift(r.x, (uint32_t)M);
                // the loads that need only i go out first
                double Vii;
                if constexpr (WG == 64) Vii = dgl[i];
                else Vii = gather<false>(diag, (uint32_t)i);
                const double phi_i = (double)phi[i];
                const int s = S == 1 ? 0 : msub[i];
                const int sa = occ[i];
                const double qa = chg[sa];
                // s < 16, E < 256, positions < 2^16: 24-bit products run at the full
                // vector rate (32-bit integer products run at a quarter of it)
                const int se = (int)__umul24((unsigned)s, (unsigned)E) + sa;
                const int na = cnt[se];
                csz = subsize[s] - na;
                const int k = (int)mulshift(r.y, (uint32_t)csz);
                const int idx = k < offs[se] ? k : k + na;
                const int jp = perm[suboff[s] + idx];
                j = csz > 0 ? jp : i;
                double Vjj;
                if constexpr (WG == 64) Vjj = dgl[j];
                else Vjj = gather<false>(diag, (uint32_t)j);
                const double Vij = gather<WG == 64>(V64, __umul24((unsigned)i, (unsigned)Mp) + (unsigned)j);
                const double phi_j = (double)phi[j];
                const int sb = occ[j];
                d = chg[sb] - qa;
                quad = 0.5 * d * d * (Vii + Vjj - 2.0 * Vij);
                dE = d * (phi_i - phi_j) + quad;
            };
            score();
            // The window's trials are decided in order: every trial before the first
            // one that may be accepted is rejected; that one is resolved and, when
            // accepted, applied. INWIN then scores the trials after it again against
            // the new state (their draws are unchanged) and goes on within the window;
            // otherwise the next window starts after it. A trial is surely rejected
            // when dE - e > thr, e bounding the FP32 field's error in dE (MIXED).
            int from = 0, used = nvalid;
            for (;;) {
                double e = 0.0;
                if constexpr (MIXED) e = fma(fabs(d), eps2, kMargin);
                const bool stop = tid >= from && tid < nvalid && csz > 0 && (ub < 2 || !(dE - e > (double)thr));
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
                if (TRACE && tid >= from && tid < nvalid && tid < f)
                    hsum += trial_hash(t + (uint64_t)tid, (uint32_t)i, (uint32_t)j, 0u);
                if (f >= nvalid) break;
                if (tid == f) {
                    double kT;
                    if (wide_blocks) {
                        kT = f < split ? kT0 : kT1;
                    } else {
                        const uint64_t blk = (t + (uint64_t)tid) / a.block_len;
                        kT = kTrow[blk < nb1 ? blk : nb1];
                    }
                    // sure accept: even dE + e lies below the lower bound of L
                    const bool sure = d == 0.0 || dE + e <= 0.0 || dE + e < (double)lo;
                    s_b.i = i; s_b.j = j; s_b.unsure = sure ? 0 : 1;
                    s_b.d = d; s_b.dE = dE; s_b.u = unit_open(r.z, r.w); s_b.kT = kT;
                }
                __syncthreads();
                const int bi = s_b.i, bj = s_b.j;
                const double bd = s_b.d;
                double bdE = s_b.dE;
                bool accf = true;
                if (s_b.unsure) {
                    if constexpr (MIXED) {
                        // exact FP64 difference phi_i - phi_j from the occupation
                        double part = 0.0;
                        for (int k = tid; k < M; k += WG)
                            part += (V64[(int64_t)bi * Mp + k] - V64[(int64_t)bj * Mp + k]) * chg[occ[k]];
                        const double diff = wg_sum<WG>(part, s_scr) + (hv[bi] - hv[bj]);
                        const double Vii = diag[bi], Vjj = diag[bj];
                        const double Vij = V64[(int64_t)bi * Mp + bj];
                        bdE = bd * diff + 0.5 * bd * bd * (Vii + Vjj - 2.0 * Vij);
                        ++n_fb;
                    }
                    // the exact rule (the FP64 field's dE is exact already)
                    accf = (bdE <= 0.0) || (s_b.u < exp(-bdE / s_b.kT));
                }
                if (TRACE && tid == f) hsum += trial_hash(t + (uint64_t)tid, (uint32_t)bi, (uint32_t)bj, accf ? 1u : 0u);
                if (accf) {
                    bool grew = false;   // MIXED: some |phi'| passed phib
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
                        // rows i and j streamed as 16-byte vectors, U vectors per thread in
                        // flight before the field is touched
                        constexpr int VEC = MIXED ? 4 : 2;
                        constexpr int U = WG >= 256 ? 8 : 1;   // one wave per chain: keep registers low
                        typedef float f32x4v __attribute__((ext_vector_type(4)));
                        typedef double f64x2v __attribute__((ext_vector_type(2)));
                        using V16 = typename std::conditional<MIXED, f32x4v, f64x2v>::type;
                        const GOAC_GLOBAL V16* Vi16 = reinterpret_cast<const GOAC_GLOBAL V16*>(Vi);
                        const GOAC_GLOBAL V16* Vj16 = reinterpret_cast<const GOAC_GLOBAL V16*>(Vj);
                        const int nv = Mp / VEC;
                        for (int v0 = tid; v0 < nv; v0 += WG * U) {
                            V16 av4[U], bv4[U];
#pragma unroll
                            for (int u = 0; u < U; ++u) {
                                const int v = v0 + u * WG;
                                if (v < nv) {
                                    av4[u] = Vi16[v];
                                    bv4[u] = Vj16[v];
                                }
                            }
#pragma unroll
                            for (int u = 0; u < U; ++u) {
                                const int v = v0 + u * WG;
                                if (v < nv) {
                                    const T* av = reinterpret_cast<const T*>(&av4[u]);
                                    const T* bv = reinterpret_cast<const T*>(&bv4[u]);
#pragma unroll
                                    for (int q = 0; q < VEC; ++q) {
                                        const int k = v * VEC + q;
                                        T p = phi[k];
                                        if constexpr (MIXED) {
                                            p = fmaf(dd, av[q], p);
                                            p = fmaf(-dd, bv[q], p);
                                            over |= fabsf(p) > phib;
                                        } else {
                                            p = p + dd * (av[q] - bv[q]);
                                        }
                                        phi[k] = p;
                                    }
                                }
                            }
                        }
                        if constexpr (MIXED) {
                            if constexpr (NW == 1) grew = __ballot(over) != 0;
                            else if (over) s_flag = 1;
                        }
                        ++n_upd;
                        ++since;
                    }
                    // the best occupation is copied lazily: only before an accepted swap
                    // that does not lower the best energy again (or one after which the
                    // field is re-anchored), and at the end of the launch, so a run of
                    // improving swaps costs one copy
                    {
                        bool anchor_due = false;
                        if constexpr (MIXED)
                            anchor_due = bd != 0.0 && a.inline_anchor && since >= (uint32_t)a.reanchor_every;
                        if (best_dirty && (anchor_due || !(Ecur + bdE < best))) {
                            copy_best();
                            best_dirty = false;
                            __syncthreads();   // the copy reads occ before the swap below
                        }
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
                        if (NW > 1 && blog_n < kBestLog) blog[blog_n] = (uint32_t)bi | ((uint32_t)bj << 16);
                    }
                    if constexpr (NW > 1) {
                        if (blog_n < kBestLog) ++blog_n;
                        else blog_full = true;
                    }
                    Ecur += bdE;
                    ++n_acc;
                    __syncthreads();
                    if constexpr (MIXED) if (bd != 0.0) {
                        if constexpr (NW > 1) grew = s_flag != 0;
                        if (grew) {
                            // |phi'| grew past the bound: take the exact maximum
                            double pm = 0.0;
                            for (int k = tid; k < M; k += WG) pm = fmax(pm, fabs((double)phi[k]));
                            pm = wg_max<WG>(pm, s_scr);
                            float pb = phib;
                            while ((double)pb < 2.0 * pm) pb *= 2.0f;
                            phib = pb;
                            if constexpr (NW > 1) {
                                __syncthreads();
                                if (tid == 0) s_flag = 0;
                            }
                        }
                        // two fused multiply-adds per element, each rounding <= u |intermediate|,
                        // plus the FP32 rounding of the two V entries (rows bounded by rmax)
                        eps += kU32 * (2.0 * (double)phib + fabs(bd) * (5.0 * rmax)) * 1.0001;
                        if (!(eps < 1e3)) status = 1;
                        if (a.inline_anchor && since >= (uint32_t)a.reanchor_every) {
                            __syncthreads();
                            anchor_chain<WG>(I, occ, msub, chg, s_phibar, reinterpret_cast<float*>(phi), s_scr,
                                             Ecur, eps, phib);
                            since = 0;
                            ++n_anc;
                            __syncthreads();
                        }
                        eps2 = 2.0 * eps;
                    }
                    if (Ecur < best) {
                        best = Ecur;
                        best_dirty = true;
                    }
                    // the trials after f against the new state: a trial touching i or j
                    // (its species, its partner list) is scored afresh, the others only
                    // take the new field
                    if constexpr (INWIN) {
                        if (tid > f && tid < nvalid) {
                            if (i == bi || i == bj || j == bi || j == bj)
                                score();
                            else
                                dE = d * ((double)phi[i] - (double)phi[j]) + quad;
                        }
                    }
                }
                if constexpr (!INWIN) {
                    used = f + 1;
                    break;
                }
                from = f + 1;
            }
            t += (uint64_t)used;
            while (t >= bnd) { ++blk0; bnd += a.block_len; }
        }
        // ---- write the chain back
        __syncthreads();
        if (best_dirty) copy_best();
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

// ------------------------------------------------------------------ batched FP64 anchor
// chains of one instance with since_anchor >= R: compacted list (row order is
// immaterial: every row is computed independently) and their FP64 charges Q
__global__ void k_anchor_select(int64_t first, int64_t C, uint32_t R, const ChainScalars* __restrict__ sc,
                                int32_t* __restrict__ due) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    if (sc[first + c].since_anchor >= R) {
        const int slot = atomicAdd(&due[0], 1);
        due[1 + slot] = (int32_t)c;
    }
}

__global__ void k_anchor_gather(int32_t M, int32_t Mp, int64_t first, const int32_t* __restrict__ due,
                                const ChainScalars* __restrict__ sc, const uint8_t* __restrict__ occ_m,
                                const double* __restrict__ charge, double* __restrict__ Q) {
    const int r = blockIdx.x;
    if (r >= due[0]) return;
    const int64_t c = first + due[1 + r];
    const uint8_t* o = occ_m + sc[c].off;
    for (int k = threadIdx.x; k < Mp; k += blockDim.x) Q[(int64_t)r * Mp + k] = k < M ? charge[o[k]] : 0.0;
}

// phi' = fl32(Phi + h - phibar_s), E = E_ff + 1/2 sum q (phi + h), error bound
__global__ __launch_bounds__(256) void k_anchor_apply(int32_t M, int32_t Mp, int64_t first,
                                                      const int32_t* __restrict__ due, const double* __restrict__ Q,
                                                      const double* __restrict__ Phi, const double* __restrict__ h,
                                                      const double* __restrict__ rowabs, double qmax,
                                                      const uint8_t* __restrict__ msub,
                                                      const double* __restrict__ phibar, const double* __restrict__ Ed,
                                                      ChainScalars* __restrict__ sc, float* __restrict__ phi) {
    __shared__ double s_a[256], s_b[256], s_c[256];
    const int r = blockIdx.x;
    if (r >= due[0]) return;
    ChainScalars* S = sc + first + due[1 + r];
    const int64_t off = S->off;
    double es = 0.0, pm = 0.0, am = 0.0;
    for (int k = threadIdx.x; k < M; k += 256) {
        const double q = Q[(int64_t)r * Mp + k];
        const double pk = Phi[(int64_t)r * Mp + k] + h[k];
        es += q * (pk + h[k]);
        const float v = (float)(pk - phibar[msub[k]]);
        phi[off + k] = v;
        pm = fmax(pm, fabs((double)v));
        am = fmax(am, fabs(h[k]) + qmax * rowabs[k]);
    }
    s_a[threadIdx.x] = es;
    s_b[threadIdx.x] = pm;
    s_c[threadIdx.x] = am;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_a[threadIdx.x] += s_a[threadIdx.x + w];
            s_b[threadIdx.x] = fmax(s_b[threadIdx.x], s_b[threadIdx.x + w]);
            s_c[threadIdx.x] = fmax(s_c[threadIdx.x], s_c[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        S->E = Ed[0] + 0.5 * s_a[0];
        const double gM = (double)(M + 2) * 0x1p-53 * 1.01;
        S->eps = kU32 * s_b[0] * 1.0001 + gM * s_c[0] * 2.0;
        float pb = 1.0f;
        while ((double)pb < 2.0 * s_b[0]) pb *= 2.0f;
        S->phibound = pb;
        S->since_anchor = 0;
        S->anchors += 1;
    }
}

__global__ void k_zero_one(int32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = 0;
}

// batched anchor of the due chains of one instance (MIXED, large cells)
goac_status anchor_batched(goac_ctx* ctx, goac_chains* ch, int inst, uint32_t R) {
    goac_problem* pb = ch->pbs[inst];
    const ProblemDev& d = pb->d;
    const int64_t Ci = ch->count[inst];
    const int64_t first = ch->first_chain[inst];
    if (Ci == 0) return GOAC_OK;
    const size_t b_due = round_up((Ci + 1) * 4, 256), b_q = round_up((size_t)Ci * d.Mp * 8, 256);
    void* ws = nullptr;
    goac_status st = workspace(ctx, 0, b_due + 2 * b_q, &ws);
    if (st != GOAC_OK) return st;
    int32_t* due = (int32_t*)ws;
    double* Q = (double*)((char*)ws + b_due);
    double* Phi = (double*)((char*)ws + b_due + b_q);
    hipLaunchKernelGGL(k_zero_one, dim3(1), dim3(64), 0, ctx->stream, due);
    hipLaunchKernelGGL(k_anchor_select, dim3((unsigned)((Ci + 255) / 256)), dim3(256), 0, ctx->stream, first, Ci, R,
                       ch->sc, due);
    hipLaunchKernelGGL(k_anchor_gather, dim3((unsigned)Ci), dim3(256), 0, ctx->stream, d.M, d.Mp, first, due, ch->sc,
                       ch->occ, d.charge, Q);
    GOAC_CHECK_LAUNCH(ctx);
    st = dgemm_nt(ctx, Ci, d.M, d.Mp, Q, d.Mp, d.V64, d.Mp, Phi, d.Mp, 1.0, 0.0, due);
    if (st != GOAC_OK) return st;
    hipLaunchKernelGGL(k_anchor_apply, dim3((unsigned)Ci), dim3(256), 0, ctx->stream, d.M, d.Mp, first, due, Q, Phi,
                       d.h, d.rowabs, d.qmax, d.msub, d.phibar, d.Ed, ch->sc, (float*)ch->phi);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
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
