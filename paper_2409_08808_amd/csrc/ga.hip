// Genetic-algorithm generation, random starts and top-k selection on gfx950
// (SI, "Genetic Algorithm" and "Random"; Methodology: output of the n lowest
// configurations).
#include <algorithm>

#include "common.h"

namespace goac {

// ------------------------------------------------------------------ random starts
// One workgroup per (chain, sublattice): the canonical species sequence of the
// sublattice is shuffled by Fisher-Yates. The draws m_k = (r_k (k+1)) >> 32 are
// independent (counter-based), so the lanes compute them in parallel; the swaps,
// which are order-dependent, run on one lane.
__global__ void k_init(int64_t n, int32_t S, int32_t E, const int32_t* __restrict__ tab,
                       const int32_t* __restrict__ spos, const int32_t* __restrict__ mob,
                       const int32_t* __restrict__ fixed_idx, int32_t n_fixed, const uint8_t* __restrict__ ref_occ,
                       uint64_t seed, uint32_t chain_base, uint32_t instance, uint8_t* __restrict__ occ) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int64_t c = blockIdx.x / S;
    const int s = (int)(blockIdx.x - c * S);
    const int32_t* subsize = tab + 2;
    const int32_t* suboff = subsize + S;
    const int32_t* cnt = suboff + S;
    const int32_t* offs = cnt + S * E;
    const int Ps = subsize[s];
    uint8_t* arr = lds;
    uint16_t* mk = reinterpret_cast<uint16_t*>(lds + round_up(Ps, 16));
    const uint32_t chain = chain_base + (uint32_t)c;
    for (int x = threadIdx.x; x < Ps; x += blockDim.x) {
        int e = 0;
        while (!(x < offs[s * E + e] + cnt[s * E + e])) ++e;
        arr[x] = (uint8_t)e;
        if (x >= 1) {
            const u32x4 r = philox((uint32_t)x, (uint32_t)s, chain, (instance << 8) | TAG_INIT, seed);
            mk[x] = (uint16_t)mulshift(r.x, (uint32_t)(x + 1));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = Ps - 1; k >= 1; --k) {
            const int m = mk[k];
            const uint8_t t = arr[k];
            arr[k] = arr[m];
            arr[m] = t;
        }
    __syncthreads();
    uint8_t* row = occ + c * n;
    for (int x = threadIdx.x; x < Ps; x += blockDim.x) row[mob[spos[suboff[s] + x]]] = arr[x];
    if (s == 0)
        for (int f = threadIdx.x; f < n_fixed; f += blockDim.x) row[fixed_idx[f]] = ref_occ[fixed_idx[f]];
}

// ------------------------------------------------------------------ GA: selection tables
// One workgroup: E_max, integer roulette weights round((E_max - E_p) 2^30) and
// their inclusive prefix sums (exact, so the order of the additions does not
// matter). The elites come from rank_select.
__global__ __launch_bounds__(1024) void k_ga_prep(int64_t P, const double* __restrict__ E,
                                                  uint64_t* __restrict__ cum, int32_t* __restrict__ err) {
    __shared__ double s_red[1024];
    __shared__ uint64_t s_tot[1024];
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    double mx = -INFINITY;
    for (int64_t p = tid; p < P; p += nt) mx = fmax(mx, E[p]);
    s_red[tid] = mx;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
        if (tid < w) s_red[tid] = fmax(s_red[tid], s_red[tid + w]);
        __syncthreads();
    }
    const double emax = s_red[0];
    const double lim = 0x1p62 / (double)P;
    // contiguous chunk per thread
    const int64_t chunk = (P + nt - 1) / nt;
    const int64_t lo = tid * chunk, hi = lo + chunk < P ? lo + chunk : P;
    uint64_t run = 0;
    bool bad = false;
    for (int64_t p = lo; p < hi; ++p) {
        const double w = (emax - E[p]) * 0x1p30;
        if (!(w < lim)) bad = true;
        run += bad ? 0 : (uint64_t)(w + 0.5);
        cum[p] = run;
    }
    if (bad) atomicOr(err, 1);
    // exclusive scan of the per-thread totals (Hillis-Steele, exact integers)
    s_tot[tid] = run;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const uint64_t v = tid >= off ? s_tot[tid - off] : 0;
        __syncthreads();
        s_tot[tid] += v;
        __syncthreads();
    }
    const uint64_t incl = s_tot[tid];
    __syncthreads();
    s_tot[tid] = incl - run;
    __syncthreads();
    const uint64_t base = s_tot[tid];
    for (int64_t p = lo; p < hi; ++p) cum[p] += base;
}

__device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// smallest p with cum[p] > target
__device__ inline int64_t upper_bound_u64(const uint64_t* cum, int64_t P, uint64_t target) {
    int64_t lo = 0, hi = P - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cum[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// ------------------------------------------------------------------ GA: one child per wavefront
constexpr int kInf = 0x7fffffff;

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// A wave's LDS operations complete in issue order, so ordering them across the
// lanes of one wave needs no wait, only that the compiler keeps their order.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// first position >= from (in the sublattice's ascending list [0, len)) whose
// predicate holds, scanning 64 at a time with a ballot; len if none
template <typename Pred>
__device__ inline int wave_find(int from, int len, Pred pred) {
    const int lane = threadIdx.x & 63;
    for (int base = from; base < len; base += 64) {
        const int x = base + lane;
        const bool hit = x < len && pred(x);
        const uint64_t m = __ballot(hit);
        if (m) return base + (int)__ffsll((long long)m) - 1;
    }
    return len;
}

// sublattices up to this length take the byte walk (crossover_bytes), longer ones
// the row walk (crossover_rows) when its rows fit in LDS, else the scan walk
constexpr int kByteMaxLen = 1024;

__device__ __forceinline__ uint32_t byte_of(uint32_t v, int k) { return (v >> (8 * k)) & 0xffu; }

// Crossover walk of a sublattice with bit rows in LDS, one 64-bit word per 64
// positions (nw words each): dis, the positions of the path copy ref that differ
// from B; coin, the coin bit of every differing position (all drawn up front, 64
// positions per ballot); and for each species e, hold[e], the positions holding e
// in ref and differing from B. Every position before the walk's p agrees with B
// in ref, so p's partner q is the first position of hold[B[p]].
// The walk keeps its current window of 64 positions in registers: lane l holds
// ref, B and the child at position 64 w + l, and lane e the window's word of
// hold[e]. A step whose partner lies in the window reads and writes only those
// registers (readlane / writelane with uniform indices); a partner further on is
// found with 64-word ballots over LDS, where its updates go too. Leaving a window
// writes its child bytes back (its ref and rows are no longer needed: every
// position of it then agrees with B).
__device__ __forceinline__ uint32_t lane_get(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

__device__ void crossover_rows(uint8_t* rs, uint8_t* cs, const uint8_t* bs, int len, const int32_t* spos_s, int E,
                               uint64_t* rows, uint32_t c, uint32_t g, uint64_t seed, int lane) {
    const int nw = (len + 63) >> 6;
    uint64_t* dis = rows;
    uint64_t* coin = rows + nw;
    uint64_t* hold = rows + 2 * nw;
    for (int x = lane; x < E * nw; x += 64) hold[x] = 0;
    wave_lds_order();
    for (int w = 0; w < nw; ++w) {
        const int x = w * 64 + lane;
        const bool in = x < len;
        const int a = in ? rs[x] : 0;
        const bool d = in && a != bs[x];
        const uint32_t sp = in ? (uint32_t)spos_s[x] : 0u;
        const bool cn = d && (philox(sp, c, g, TAG_X, seed).x >> 31) != 0;
        const uint64_t dm = __ballot(d), cm = __ballot(cn);
        if (d) atomicOr(reinterpret_cast<unsigned long long*>(&hold[a * nw + w]), 1ull << lane);
        if (lane == 0) {
            dis[w] = dm;
            coin[w] = cm;
        }
    }
    wave_lds_order();
    int w = -1;
    uint64_t cur = 0, cw = 0;
    uint32_t rv = 0, bv = 0, cv = 0;   // the window: ref, B and the child at 64 w + lane
    uint64_t hw = 0;                   // lane e: the window's word of hold[e]
    for (;;) {
        if (!cur) {
            // leave the window (child bytes back to LDS), then find the next word
            // with a differing position and load its window
            if (w >= 0 && w * 64 + lane < len) cs[w * 64 + lane] = (uint8_t)cv;
            int nxt = nw;
            for (int base = w + 1; base < nw; base += 64) {
                const int y = base + lane;
                const uint64_t m = __ballot(y < nw && dis[y] != 0);
                if (m) {
                    nxt = base + (int)__ffsll((long long)m) - 1;
                    break;
                }
            }
            wave_lds_order();
            if (nxt >= nw) break;
            w = nxt;
            const int x = w * 64 + lane;
            const bool in = x < len;
            rv = in ? rs[x] : 0u;
            bv = in ? bs[x] : 0u;
            cv = in ? cs[x] : 0u;
            hw = lane < E ? hold[lane * nw + w] : 0ull;
            cur = dis[w];
            cw = coin[w];
            wave_lds_order();
        }
        const int po = (int)__ffsll((long long)cur) - 1;
        cur &= cur - 1;
        const int a = (int)lane_get(rv, po);
        const int b = (int)lane_get(bv, po);
        const uint32_t cp = lane_get(cv, po);
        const bool take = (cw >> po) & 1ull;   // the child takes this swap of the path
        const uint64_t bitp = 1ull << po;
        // partner: the first holder of b, in the window or further on
        const uint64_t hv = readlane64(hw, b);
        // p now agrees: it leaves hold[a]
        hw = lane == a ? hw & ~bitp : hw;
        if (hv) {
            // in the window: registers only, no branches
            const int qo = (int)__ffsll((long long)hv) - 1;
            const uint64_t bitq = 1ull << qo;
            const int bq = (int)lane_get(bv, qo);
            const uint32_t cq = lane_get(cv, qo);
            const bool carry = bq != a;   // q keeps differing from B after taking a
            hw = lane == b ? hw & ~bitq : hw;
            hw = (carry && lane == a) ? hw | bitq : hw;
            rv = (carry && lane == qo) ? (uint32_t)a : rv;
            cur = carry ? cur : cur & ~bitq;
            cv = (take && lane == po) ? cq : ((take && lane == qo) ? cp : cv);
        } else {
            int qw = nw;
            uint64_t hq = 0;
            const uint64_t* hb = hold + b * nw;
            for (int base = w + 1; base < nw; base += 64) {
                const int y = base + lane;
                const uint64_t v = y < nw ? hb[y] : 0ull;
                const uint64_t m = __ballot(v != 0);
                if (m) {
                    const int l = (int)__ffsll((long long)m) - 1;
                    qw = base + l;
                    hq = readlane64(v, l);
                    break;
                }
            }
            if (qw >= nw) break;   // cannot happen: ref and B share the composition
            const int qo = (int)__ffsll((long long)hq) - 1;
            const int q = qw * 64 + qo;
            const int bq = bs[q];
            const uint8_t cq = cs[q];
            const bool carry = bq != a;
            if (lane == 0) {
                hold[b * nw + qw] = hq & ~(1ull << qo);
                rs[q] = (uint8_t)a;
                if (carry) atomicOr(reinterpret_cast<unsigned long long*>(&hold[a * nw + qw]), 1ull << qo);
                else atomicAnd(reinterpret_cast<unsigned long long*>(&dis[qw]), ~(1ull << qo));
                if (take) cs[q] = (uint8_t)cp;
            }
            cv = (take && lane == po) ? (uint32_t)cq : cv;
            wave_lds_order();
        }
    }
    if (w >= 0 && w * 64 + lane < len) cs[w * 64 + lane] = (uint8_t)cv;   // (already written on the normal exit)
    wave_lds_order();
}

// Crossover walk of one sublattice of at most 256 NR positions held in registers,
// any species count: lane l holds position l + 64 k of chunk k in byte k & 3 of
// dword k >> 2 of R (the path copy), Bv (parent B) and Cv (the child). The coin
// of every position is drawn up front, all lanes in parallel (bit k of coin). A
// step finds the next disagreeing position p and its partner q with a ballot over
// one chunk at a time and moves single bytes between lanes with readlane, so the
// walk touches no memory between the loads and the final stores of the child.
template <int NR>
__device__ void crossover_bytes(uint8_t* cs, const uint8_t* bs, int len, const int32_t* spos_s, uint32_t c,
                                uint32_t g, uint64_t seed, int lane) {
    uint32_t R[NR], Bv[NR], Cv[NR];
#pragma unroll
    for (int d = 0; d < NR; ++d) {
        uint32_t r = 0xffffffffu, b = 0xffffffffu;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = (4 * d + k) * 64 + lane;
            if (x < len) {
                const uint32_t sh = 8u * (uint32_t)k;
                r = (r & ~(0xffu << sh)) | ((uint32_t)cs[x] << sh);
                b = (b & ~(0xffu << sh)) | ((uint32_t)bs[x] << sh);
            }
        }
        R[d] = r;  // padding bytes agree with B, so the walk never visits them
        Bv[d] = b;
        Cv[d] = r;
    }
    const int nk = (len + 63) >> 6;
    uint32_t coin = 0;
    for (int k = 0; k < nk; ++k) {
        const int x = k * 64 + lane;
        if (x < len && (philox((uint32_t)spos_s[x], c, g, TAG_X, seed).x >> 31)) coin |= 1u << k;
    }
    auto chunk = [](const uint32_t(&v)[NR], int k) -> uint32_t { return byte_of(v[k >> 2], k & 3); };
    auto put = [lane](uint32_t(&v)[NR], int k, int l, uint32_t b) {
        const uint32_t sh = 8u * (uint32_t)(k & 3);
        const uint32_t old = v[k >> 2];
        const uint32_t nv = (old & ~(0xffu << sh)) | (b << sh);
        v[k >> 2] = lane == l ? nv : old;
    };
    int p = 0;
    while (p < len) {
        // next disagreeing position from p
        int k = p >> 6;
        uint64_t m = __ballot(chunk(R, k) != chunk(Bv, k)) & (~0ull << (p & 63));
        while (!m && ++k < nk) m = __ballot(chunk(R, k) != chunk(Bv, k));
        if (!m) break;
        const int lp = (int)__ffsll((long long)m) - 1;
        p = k * 64 + lp;
        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)chunk(R, k), lp);
        const uint32_t want = (uint32_t)__builtin_amdgcn_readlane((int)chunk(Bv, k), lp);
        // partner: first q > p holding want in the path copy and disagreeing with B
        int kq = k;
        uint64_t mq = __ballot(chunk(R, kq) == want && chunk(R, kq) != chunk(Bv, kq));
        mq = lp == 63 ? 0ull : mq & (~0ull << (lp + 1));
        while (!mq && ++kq < nk) mq = __ballot(chunk(R, kq) == want && chunk(R, kq) != chunk(Bv, kq));
        if (!mq) break;  // cannot happen: the path copy and B share the composition
        const int lq = (int)__ffsll((long long)mq) - 1;
        put(R, k, lp, want);
        put(R, kq, lq, a);
        if (((uint32_t)__builtin_amdgcn_readlane((int)coin, lp) >> k) & 1u) {
            const uint32_t cp = (uint32_t)__builtin_amdgcn_readlane((int)chunk(Cv, k), lp);
            const uint32_t cq = (uint32_t)__builtin_amdgcn_readlane((int)chunk(Cv, kq), lq);
            put(Cv, k, lp, cq);
            put(Cv, kq, lq, cp);
        }
        ++p;
    }
#pragma unroll
    for (int d = 0; d < NR; ++d)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = (4 * d + k) * 64 + lane;
            if (x < len) cs[x] = (uint8_t)byte_of(Cv[d], k);
        }
    wave_lds_order();
}

// Child c of generation g (SI, "Genetic Algorithm"). Children below n_elite copy
// the elites. Every other child draws parents A and B by roulette, crosses them
// and may mutate:
//   crossover: the canonical swap path from A to B is walked on a copy ref of A.
//     Per sublattice, positions p ascending with ref[p] != B[p] take B[p] from
//     the smallest later position q of the sublattice that holds B[p] and also
//     disagrees with B; ref swaps p and q. The child (a second copy of A) takes
//     each swap of the path iff the top bit of Philox(p_mobile, c, g, X) is set.
//   mutation: with probability p_mut one valid swap, drawn as an MC proposal
//     with the sublattice's positions ordered by (species, position).
// Sublattices of up to 1024 positions take the byte walk (crossover_bytes); longer
// ones the row walk (crossover_rows) when rows_words > 0 (the LDS of its rows, in
// 64-bit words), else the scan walk, which finds p and q with 64-position ballots
// over the path copy in LDS.
__global__ __launch_bounds__(64) void k_ga_child(
    int64_t n, int32_t M, int32_t S, int32_t E, const int32_t* __restrict__ tab, const int32_t* __restrict__ spos,
    const int32_t* __restrict__ spos_inv, const uint8_t* __restrict__ msub, const int32_t* __restrict__ ssite,
    const int32_t* __restrict__ fixed_idx, int32_t n_fixed, const uint8_t* __restrict__ ref_occ, int64_t P,
    const uint8_t* __restrict__ pop_in, const uint64_t* __restrict__ cum, const int32_t* __restrict__ elite,
    int32_t n_elite, uint64_t seed, uint32_t g, const uint32_t* __restrict__ g_dev, double p_mut,
    int32_t rows_words, uint8_t* __restrict__ pop_out) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int64_t c = blockIdx.x;
    if (g_dev) g += *g_dev;   // a captured generation: the index is base + offset
    const int lane = threadIdx.x;
    uint8_t* out = pop_out + c * n;
    if (c < n_elite) {
        int64_t ep = elite[c];
        if (ep < 0 || ep >= P) ep = 0;   // unranked (NaN energies); the call reports the error
        const uint8_t* src = pop_in + ep * n;
        for (int64_t x = lane; x < n; x += 64) out[x] = src[x];
        return;
    }
    const int32_t* subsize = tab + 2;
    const int32_t* suboff = subsize + S;
    const int32_t* cnt = suboff + S;
    const int32_t* offs = cnt + S * E;
    // parents
    const u32x4 r = philox((uint32_t)c, g, 0u, TAG_SEL, seed);
    const uint64_t xa = ((uint64_t)r.x << 32) | r.y, xb = ((uint64_t)r.z << 32) | r.w;
    const uint64_t W = cum[P - 1];
    int64_t pa, pb;
    if (W == 0) {
        pa = (int64_t)mulhi64(xa, (uint64_t)P);
        pb = (int64_t)mulhi64(xb, (uint64_t)P);
    } else {
        pa = upper_bound_u64(cum, P, mulhi64(xa, W));
        pb = upper_bound_u64(cum, P, mulhi64(xb, W));
    }
    // mobile occupations in sublattice order: ch (child), rf (path walk), bb (parent
    // B); then the row walk's bit rows
    const int Mr = (int)round_up(M, 16);
    uint8_t* ch = lds;
    uint8_t* rf = lds + Mr;
    uint8_t* bb = lds + 2 * Mr;
    uint64_t* rows = reinterpret_cast<uint64_t*>(lds + round_up(3 * (int64_t)Mr, 16));
    const uint8_t* A = pop_in + pa * n;
    const uint8_t* B = pop_in + pb * n;
    // eight positions per lane per round, their loads in flight together
    for (int x0 = lane; x0 < M; x0 += 8 * 64) {
        int st[8];
        uint8_t av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) st[u] = x0 + 64 * u < M ? ssite[x0 + 64 * u] : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            av[u] = A[st[u]];
            bv[u] = B[st[u]];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int x = x0 + 64 * u;
            if (x < M) {
                ch[x] = av[u];
                rf[x] = av[u];
                bb[x] = bv[u];
            }
        }
    }
    wave_lds_order();
    for (int s = 0; s < S; ++s) {
        const int base = suboff[s], len = subsize[s];
        uint8_t* rs = rf + base;
        uint8_t* cs = ch + base;
        const uint8_t* bs = bb + base;
        if (len <= kByteMaxLen) {
            if (len <= 256) crossover_bytes<1>(cs, bs, len, spos + base, (uint32_t)c, g, seed, lane);
            else if (len <= 512) crossover_bytes<2>(cs, bs, len, spos + base, (uint32_t)c, g, seed, lane);
            else crossover_bytes<4>(cs, bs, len, spos + base, (uint32_t)c, g, seed, lane);
            continue;
        }
        if ((int64_t)(E + 2) * ((len + 63) / 64) <= rows_words) {
            crossover_rows(rs, cs, bs, len, spos + base, E, rows, (uint32_t)c, g, seed, lane);
            continue;
        }
        // scan walk: the next disagreeing position and its partner, 64 positions at a
        // time; lane 0 swaps the path copy and, on a set coin, the child
        int p = 0;
        for (;;) {
            p = wave_find(p, len, [&](int x) { return rs[x] != bs[x]; });
            if (p >= len) break;
            const uint8_t want = bs[p];
            const int q = wave_find(p + 1, len, [&](int x) { return rs[x] == want && rs[x] != bs[x]; });
            if (q >= len) break;  // cannot happen: ref and B share the composition
            if (lane == 0) {
                const uint8_t t = rs[p]; rs[p] = rs[q]; rs[q] = t;
                const u32x4 rx = philox((uint32_t)spos[base + p], (uint32_t)c, g, TAG_X, seed);
                if (rx.x >> 31) { const uint8_t t2 = cs[p]; cs[p] = cs[q]; cs[q] = t2; }
            }
            wave_lds_order();
            ++p;
        }
    }
    // mutation: one valid swap with probability p_mut
    const u32x4 rm = philox((uint32_t)c, g, 1u, TAG_MUT, seed);
    if (M > 0 && unit_open(rm.z, rm.w) < p_mut) {
        const int im = (int)mulshift(rm.x, (uint32_t)M);
        const int s = msub[im];
        const int base = suboff[s];
        const int px = spos_inv[im] - base;
        const uint8_t a = ch[base + px];
        const int na = a < E ? cnt[s * E + a] : 0;
        const int cn = subsize[s] - na;
        if (a < E && cn > 0) {
            const int k = (int)mulshift(rm.y, (uint32_t)cn);
            const int idx = k < offs[s * E + a] ? k : k + na;
            int e = 0;
            while (!(idx < offs[s * E + e] + cnt[s * E + e])) ++e;
            int rank = idx - offs[s * E + e];
            // rank-th position of species e, ascending
            int pos = -1;
            const int len = subsize[s];
            for (int b0 = 0; b0 < len && pos < 0; b0 += 64) {
                const int x = b0 + lane;
                const bool hit = x < len && ch[base + x] == e;
                const uint64_t m = __ballot(hit);
                const int pc = __popcll(m);
                if (rank < pc) {
                    uint64_t mm = m;
                    for (int z = 0; z < rank; ++z) mm &= mm - 1;
                    pos = b0 + (int)__ffsll((long long)mm) - 1;
                } else {
                    rank -= pc;
                }
            }
            if (lane == 0 && pos >= 0) {
                const uint8_t t = ch[base + px]; ch[base + px] = ch[base + pos]; ch[base + pos] = t;
            }
            wave_lds_order();
        }
    }
    for (int x0 = lane; x0 < M; x0 += 8 * 64) {
        int st[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) st[u] = x0 + 64 * u < M ? ssite[x0 + 64 * u] : -1;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (st[u] >= 0) out[st[u]] = ch[x0 + 64 * u];
    }
    for (int f = lane; f < n_fixed; f += 64) out[fixed_idx[f]] = ref_occ[fixed_idx[f]];
}

// LDS of a child: its occupation, the path copy and parent B (bytes), then the row
// walk's bit rows for the longest sublattice above the byte walk's range: (E + 2)
// words per 64 positions, left out when they would not fit (those sublattices then
// take the scan walk)
static int64_t ga_rows_words(const goac_problem* pb) {
    int maxlen = 0;
    for (int s = 0; s < pb->d.S; ++s) maxlen = std::max(maxlen, (int)pb->tab_host[2 + s]);
    if (maxlen <= kByteMaxLen) return 0;
    const int64_t words = (int64_t)(pb->d.E + 2) * ((maxlen + 63) / 64);
    const int64_t base = round_up(3 * round_up(pb->d.M, 16), 16);
    return base + 8 * words <= 160 * 1024 ? words : 0;
}

size_t ga_child_lds(const goac_problem* pb) {
    return round_up(3 * round_up(pb->d.M, 16), 16) + 8 * ga_rows_words(pb);
}

goac_status ga_children(goac_problem* pb, int64_t P, const uint8_t* pop_in, const uint64_t* cum, const int32_t* elite,
                        int32_t n_elite, const goac_ga_params* prm, uint8_t* pop_out, const uint32_t* g_dev) {
    goac_ctx* ctx = pb->ctx;
    const ProblemDev& d = pb->d;
    const size_t lds = ga_child_lds(pb);
    if (lds > 64 * 1024)
        GOAC_HIP(ctx, hipFuncSetAttribute((const void*)k_ga_child, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_ga_child, dim3((unsigned)P), dim3(64), lds, ctx->stream, d.n, d.M, d.S, d.E, d.tab, pb->spos,
                       pb->spos_inv, d.msub, pb->ssite, pb->fixed_idx, pb->n_fixed, d.ref_occ, P, pop_in, cum, elite,
                       n_elite, prm->seed, prm->generation, g_dev, prm->p_mut, (int32_t)ga_rows_words(pb), pop_out);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

// ------------------------------------------------------------------ ranking
// rank(p) = #{q : (E_q, q) < (E_p, p)} (a strict total order, so ranks are
// distinct); the k smallest ranks are the k lowest configurations. A workgroup
// counts, for its 256 p, the q of one 64-wide segment staged in LDS and adds the
// count to rank(p) with an integer atomic (exact, so the order of the additions
// does not matter).
constexpr int RK_SEG = 64;

__global__ __launch_bounds__(256) void k_rank_count(int64_t P, const double* __restrict__ E,
                                                    int32_t* __restrict__ cnt) {
    __shared__ double tile[RK_SEG];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double ep = p < P ? E[p] : 0.0;
    int c = 0;
    for (int64_t b0 = (int64_t)blockIdx.y * RK_SEG; b0 < P; b0 += (int64_t)gridDim.y * RK_SEG) {
        const int len = (int)(P - b0 < RK_SEG ? P - b0 : RK_SEG);
        __syncthreads();
        if (threadIdx.x < len) tile[threadIdx.x] = E[b0 + threadIdx.x];
        __syncthreads();
        for (int x = 0; x < len; ++x) {
            const double eq = tile[x];
            c += (eq < ep || (eq == ep && b0 + x < p)) ? 1 : 0;
        }
    }
    if (p < P && c) atomicAdd(cnt + p, c);
}

// idx[rank] = p (int64 or int32 output) and Eout[rank] = E_p for rank < k
__global__ void k_rank_finish(int64_t P, int32_t k, const double* __restrict__ E, const int32_t* __restrict__ cnt,
                              int64_t* __restrict__ idx64, int32_t* __restrict__ idx32, double* __restrict__ Eout) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t r = cnt[p];
    if (r < k) {
        if (idx64) idx64[r] = p;
        if (idx32) idx32[r] = (int32_t)p;
        if (Eout) Eout[r] = E[p];
    }
}

__global__ void k_zero_rank(int64_t P, int32_t* __restrict__ cnt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) cnt[p] = 0;
}

// cnt_scratch: P int32
goac_status rank_select(goac_ctx* ctx, int64_t P, const double* E, int32_t k, int32_t* cnt_scratch,
                        int64_t* idx64, int32_t* idx32, double* Eout) {
    if (k <= 0 || P <= 0) return GOAC_OK;
    const unsigned pb = (unsigned)((P + 255) / 256);
    hipLaunchKernelGGL(k_zero_rank, dim3(pb), dim3(256), 0, ctx->stream, P, cnt_scratch);
    dim3 g1(pb, (unsigned)std::min<int64_t>((P + RK_SEG - 1) / RK_SEG, 65535));
    hipLaunchKernelGGL(k_rank_count, g1, dim3(256), 0, ctx->stream, P, E, cnt_scratch);
    hipLaunchKernelGGL(k_rank_finish, dim3(pb), dim3(256), 0, ctx->stream, P, k, E, cnt_scratch, idx64, idx32, Eout);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

}  // namespace goac
