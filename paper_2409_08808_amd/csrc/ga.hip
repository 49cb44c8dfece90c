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
// A wave's LDS operations complete in issue order, so ordering them across the
// lanes of one wave needs no wait, only that the compiler keeps their order.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// sublattices up to this length take the byte walk (crossover_bytes), longer ones
// the window walk (crossover_win) over kWinWords words of 64 positions
constexpr int kByteMaxLen = 1024;
constexpr int kWinWords = 3;

__device__ __forceinline__ uint32_t byte_of(uint32_t v, int k) { return (v >> (8 * k)) & 0xffu; }

// Crossover walk of a sublattice longer than the byte walk's range, through a
// window of K consecutive 64-position words held in registers. Slot k holds word
// w0 + k: lane l has the path copy's byte at position 64 (w0 + k) + l in rv[k]
// and parent B's and the child's bytes (B | child << 8) in bc[k]; the uniform
// masks cur[k] (the word's positions that still disagree with B and are not yet
// walked) and cw[k] (the word's coins) sit in scalar registers. Every position
// before the walk's p agrees with B, so p's partner q is the first position of
// cur holding B[p] in the path copy: one compare and ballot per slot finds it,
// and the swap is a few readlane / writelane with uniform lanes. A partner beyond
// the window is found with 64-position ballots over the bytes in LDS, where its
// update goes. When slot 0 has no position left, its child bytes return to LDS and
// the window moves on by one word. coin: LDS for one 64-bit word per 64 positions.
__device__ __forceinline__ uint32_t lane_get(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// the writelane intrinsic (v_writelane_b32), which this compiler has no builtin for
__device__ int amdgcn_writelane(int x, int l, int v) __asm("llvm.amdgcn.writelane.i32");

// v with lane l (uniform) replaced by x (uniform)
__device__ __forceinline__ uint32_t lane_put(uint32_t v, int l, uint32_t x) {
    return (uint32_t)amdgcn_writelane((int)x, l, (int)v);
}

template <int K>
struct WinWalk {
    uint32_t rv[K], bc[K];
    uint64_t cur[K], cw[K];
    uint8_t* rs;
    uint8_t* cs;
    const uint8_t* bs;
    const uint64_t* coin;
    int len, nw, lane;

    __device__ __forceinline__ void load(int k, int w) {
        const int x = w * 64 + lane;
        const bool in = x < len;   // false for every w >= nw
        const uint32_t r = in ? rs[x] : 0u, b = in ? bs[x] : 0u;
        rv[k] = r;
        bc[k] = b | ((in ? (uint32_t)cs[x] : 0u) << 8);
        cur[k] = __ballot(r != b);
        const uint64_t cwv = w < nw ? coin[w] : 0ull;
        cw[k] = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(cwv >> 32)) << 32) |
                (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)cwv);
    }

    // p (slot 0, lane po, path byte a, packed B | child vp) swaps with the first
    // holder of b = B[p] in slot k or later
    template <int k>
    __device__ __forceinline__ void swap(int po, uint32_t a, uint32_t vp, uint32_t take, int w0) {
        const uint32_t b = vp & 0xffu;
        if constexpr (k < K) {
            const uint64_t hv = __ballot(rv[k] == b) & cur[k];
            if (!hv) {
                swap<k + 1>(po, a, vp, take, w0);
                return;
            }
            const int qo = (int)__ffsll((long long)hv) - 1;
            const uint32_t vq = lane_get(bc[k], qo);
            rv[k] = lane_put(rv[k], qo, a);
            // q now agrees with B: it leaves cur (its bit is set, so xor clears it)
            cur[k] = (vq & 0xffu) == a ? cur[k] ^ (1ull << qo) : cur[k];
            if (take) {
                bc[0] = lane_put(bc[0], po, b | (vq & 0xff00u));
                bc[k] = lane_put(bc[k], qo, (vq & 0xffu) | (vp & 0xff00u));
            }
        } else {
            // the partner lies beyond the window
            for (int wb = w0 + K; wb < nw; ++wb) {
                const int x = wb * 64 + lane;
                const bool in = x < len;
                const uint32_t r = in ? rs[x] : 0xffu, bb = in ? bs[x] : 0xffu;
                const uint64_t m = __ballot(r == b && bb != b);
                if (m) {
                    const int l = (int)__ffsll((long long)m) - 1;
                    const uint32_t cq = lane_get(in ? (uint32_t)cs[x] : 0u, l);
                    if (lane == 0) {
                        rs[wb * 64 + l] = (uint8_t)a;
                        if (take) cs[wb * 64 + l] = (uint8_t)(vp >> 8);
                    }
                    if (take) bc[0] = lane_put(bc[0], po, b | (cq << 8));
                    wave_lds_order();
                    return;
                }
            }
            // (no partner cannot happen: the path copy and B share the composition)
        }
    }

    __device__ void run() {
#pragma unroll
        for (int k = 0; k < K; ++k) load(k, k);
        int w0 = 0;
        for (;;) {
            while (cur[0]) {
                const int po = (int)__ffsll((long long)cur[0]) - 1;
                cur[0] ^= 1ull << po;   // (bit po is set: it is the lowest)
                const uint32_t a = lane_get(rv[0], po);
                const uint32_t vp = lane_get(bc[0], po);
                const uint32_t take = (uint32_t)(cw[0] >> po) & 1u;   // the child takes this swap of the path
                swap<0>(po, a, vp, take, w0);
            }
            if (w0 * 64 + lane < len) cs[w0 * 64 + lane] = (uint8_t)(bc[0] >> 8);
            if (++w0 >= nw) break;
#pragma unroll
            for (int k = 0; k + 1 < K; ++k) {
                rv[k] = rv[k + 1];
                bc[k] = bc[k + 1];
                cur[k] = cur[k + 1];
                cw[k] = cw[k + 1];
            }
            load(K - 1, w0 + K - 1);
        }
        wave_lds_order();
    }
};

template <int K>
__device__ void crossover_win(uint8_t* rs, uint8_t* cs, const uint8_t* bs, int len, const int32_t* spos_s,
                              uint64_t* coin, uint32_t c, uint32_t g, uint64_t seed, int lane) {
    const int nw = (len + 63) >> 6;
    // the coin of every position, 64 per ballot, eight words' draws in flight together
    for (int w8 = 0; w8 < nw; w8 += 8) {
        uint32_t sp[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int x = (w8 + u) * 64 + lane;
            sp[u] = x < len ? (uint32_t)spos_s[x] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int x = (w8 + u) * 64 + lane;
            const uint64_t m = __ballot(x < len && (philox(sp[u], c, g, TAG_X, seed).x >> 31) != 0);
            if (lane == 0 && w8 + u < nw) coin[w8 + u] = m;
        }
    }
    wave_lds_order();
    WinWalk<K> ww;
    ww.rs = rs;
    ww.cs = cs;
    ww.bs = bs;
    ww.coin = coin;
    ww.len = len;
    ww.nw = nw;
    ww.lane = lane;
    ww.run();
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
// Sublattices of up to 1024 positions take the byte walk (crossover_bytes), longer
// ones the window walk (crossover_win).
__global__ __launch_bounds__(64) void k_ga_child(
    int64_t n, int32_t M, int32_t S, int32_t E, const int32_t* __restrict__ tab, const int32_t* __restrict__ spos,
    const int32_t* __restrict__ spos_inv, const uint8_t* __restrict__ msub, const int32_t* __restrict__ ssite,
    const int32_t* __restrict__ fixed_idx, int32_t n_fixed, const uint8_t* __restrict__ ref_occ, int64_t P,
    const uint8_t* __restrict__ pop_in, const uint64_t* __restrict__ cum, const int32_t* __restrict__ elite,
    int32_t n_elite, uint64_t seed, uint32_t g, const uint32_t* __restrict__ g_dev, double p_mut,
    uint8_t* __restrict__ pop_out) {
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
    // B); then the window walk's coin words
    const int Mr = (int)round_up(M, 16);
    uint8_t* ch = lds;
    uint8_t* rf = lds + Mr;
    uint8_t* bb = lds + 2 * Mr;
    uint64_t* coin = reinterpret_cast<uint64_t*>(lds + round_up(3 * (int64_t)Mr, 16));
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
        crossover_win<kWinWords>(rs, cs, bs, len, spos + base, coin, (uint32_t)c, g, seed, lane);
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

// LDS of a child: its occupation, the path copy and parent B (bytes), then the
// window walk's coin words (one per 64 positions of the longest sublattice above
// the byte walk's range)
size_t ga_child_lds(const goac_problem* pb) {
    int maxlen = 0;
    for (int s = 0; s < pb->d.S; ++s) maxlen = std::max(maxlen, (int)pb->tab_host[2 + s]);
    const int64_t words = maxlen > kByteMaxLen ? (maxlen + 63) / 64 : 0;
    return round_up(3 * round_up(pb->d.M, 16), 16) + 8 * words;
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
                       n_elite, prm->seed, prm->generation, g_dev, prm->p_mut, pop_out);
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
