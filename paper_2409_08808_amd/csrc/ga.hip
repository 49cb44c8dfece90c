// Genetic-algorithm generation, random starts and top-k selection on gfx950
// (SI, "Genetic Algorithm" and "Random"; Methodology: output of the n lowest
// configurations).
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

// Crossover walk of one sublattice held in registers (len <= 4096 positions,
// species ids < kRegSpecies). Lane l owns positions 64 l .. 64 l + 63: the bytes of
// ref (the path copy), of parent B and of the child in R, Bv, Cv (dword d holds
// positions 4 d .. 4 d + 3), one 64-bit word of each species' bit row (bit j: the
// position holds e in ref and disagrees with B), the word of disagreeing positions
// still to visit (mm), and, in lane e, the head of species e's row. A step reads
// and writes single bytes and words of given lanes with uniform register indices
// (no memory traffic); the coin bits of a chunk are drawn when the walk enters
// it. Returns false on a species id out of range or a broken composition.
constexpr int kRegSpecies = 16;
constexpr int kRegMaxLen = 64 * 64;
// sublattices up to this length take the byte walk (crossover_bytes), longer ones
// the register walk when it applies, else the scan walk
constexpr int kByteMaxLen = 1024;

__device__ __forceinline__ uint32_t byte_of(uint32_t v, int k) { return (v >> (8 * k)) & 0xffu; }

__device__ bool crossover_regs(uint8_t* rs, uint8_t* cs, const uint8_t* bs, int len, const int32_t* spos_s,
                               uint64_t* mk, uint32_t c, uint32_t g, uint64_t seed, int lane) {
    uint32_t R[16], Bv[16], Cv[16];
    const int x0 = lane * 64;
#pragma unroll
    for (int d = 0; d < 16; ++d) {
        uint32_t r = 0, b = 0, ch = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = x0 + 4 * d + k;
            if (x < len) {
                r |= (uint32_t)rs[x] << (8 * k);
                b |= (uint32_t)bs[x] << (8 * k);
                ch |= (uint32_t)cs[x] << (8 * k);
            }
        }
        R[d] = r;
        Bv[d] = b;
        Cv[d] = ch;
    }
    // species rows through LDS: lane l ors bit j into mk[e][l] for each of its
    // disagreeing positions (each lane touches only its own column)
    for (int e = 0; e < kRegSpecies; ++e) mk[e * 64 + lane] = 0;
    wave_lds_order();
    uint64_t mm = 0;
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 16; ++d)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t e = byte_of(R[d], k), b = byte_of(Bv[d], k);
            if (e != b) {
                if (e < kRegSpecies && b < kRegSpecies) {
                    const uint64_t bit = 1ull << (4 * d + k);
                    atomicOr(reinterpret_cast<unsigned long long*>(&mk[e * 64 + lane]), (unsigned long long)bit);
                    mm |= bit;
                } else {
                    ok = false;
                }
            }
        }
    if (__ballot(!ok)) return false;
    wave_lds_order();
    uint64_t rows[kRegSpecies];
#pragma unroll
    for (int e = 0; e < kRegSpecies; ++e) rows[e] = mk[e * 64 + lane];
    int hv = kInf;
#pragma unroll
    for (int e = 0; e < kRegSpecies; ++e) {
        const uint64_t m = __ballot(rows[e] != 0);
        if (m) {
            const int l = (int)__ffsll((long long)m) - 1;
            const uint64_t v = readlane64(rows[e], l);
            if (lane == e) hv = l * 64 + (int)__ffsll((long long)v) - 1;
        }
    }
    const int nw = (len + 63) >> 6;
    for (int w = 0; w < nw; ++w) {
        uint64_t cur = readlane64(mm, w);
        if (!cur) continue;
        // coins of the chunk: lane j draws position 64 w + j
        const int xj = w * 64 + lane;
        const bool coin = xj < len && (philox((uint32_t)spos_s[xj], c, g, TAG_X, seed).x >> 31) != 0;
        const uint64_t xm = __ballot(coin);
        while (cur) {
            const int po = (int)__ffsll((long long)cur) - 1;
            cur &= cur - 1;
            const int p = w * 64 + po;
            const int a = (int)byte_of((uint32_t)__builtin_amdgcn_readlane((int)R[po >> 2], w), po & 3);
            const int b = (int)byte_of((uint32_t)__builtin_amdgcn_readlane((int)Bv[po >> 2], w), po & 3);
            const int q = __builtin_amdgcn_readlane(hv, b);
            if (q >= len || q <= p) return false;
            const int qw = q >> 6, qo = q & 63;
            const int bq = (int)byte_of((uint32_t)__builtin_amdgcn_readlane((int)Bv[qo >> 2], qw), qo & 3);
            const bool carry = bq != a;   // q keeps disagreeing with B after taking a
            const uint64_t bitq = 1ull << qo, bitp = 1ull << po;
            // row of b loses q; its new head is the first set bit from lane qw on
            uint64_t rb = rows[b];
            rb = lane == qw ? rb & ~bitq : rb;
            rows[b] = rb;
            int hb = kInf;
            {
                const uint64_t m = __ballot(lane >= qw && rb != 0);
                if (m) {
                    const int l = (int)__ffsll((long long)m) - 1;
                    hb = l * 64 + (int)__ffsll((long long)readlane64(rb, l)) - 1;
                }
            }
            // row of a loses p and gains q when q keeps disagreeing
            uint64_t ra = rows[a];
            ra = lane == w ? ra & ~bitp : ra;
            if (carry) ra = lane == qw ? ra | bitq : ra;
            rows[a] = ra;
            int ha = kInf;
            {
                const uint64_t m = __ballot(lane >= w && ra != 0);
                if (m) {
                    const int l = (int)__ffsll((long long)m) - 1;
                    ha = l * 64 + (int)__ffsll((long long)readlane64(ra, l)) - 1;
                }
            }
            hv = lane == b ? hb : hv;
            hv = lane == a ? ha : hv;
            // ref[q] = a
            {
                const uint32_t sh = 8u * (uint32_t)(qo & 3);
                const uint32_t v = R[qo >> 2];
                const uint32_t nv = (v & ~(0xffu << sh)) | ((uint32_t)a << sh);
                R[qo >> 2] = lane == qw ? nv : v;
            }
            if (!carry) {
                if (qw == w) cur &= ~bitq;
                else mm = lane == qw ? mm & ~bitq : mm;
            }
            // the child takes this swap of the path with probability 1/2
            if ((xm >> po) & 1) {
                const uint32_t vp = Cv[po >> 2], vq = Cv[qo >> 2];
                const uint32_t cp = byte_of((uint32_t)__builtin_amdgcn_readlane((int)vp, w), po & 3);
                const uint32_t cq = byte_of((uint32_t)__builtin_amdgcn_readlane((int)vq, qw), qo & 3);
                const uint32_t shp = 8u * (uint32_t)(po & 3), shq = 8u * (uint32_t)(qo & 3);
                Cv[po >> 2] = lane == w ? (vp & ~(0xffu << shp)) | (cq << shp) : vp;
                const uint32_t vq2 = Cv[qo >> 2];
                Cv[qo >> 2] = lane == qw ? (vq2 & ~(0xffu << shq)) | (cp << shq) : vq2;
            }
        }
    }
    // child bytes back to LDS
#pragma unroll
    for (int d = 0; d < 16; ++d)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = x0 + 4 * d + k;
            if (x < len) cs[x] = (uint8_t)byte_of(Cv[d], k);
        }
    wave_lds_order();
    return true;
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
// Sublattices of up to 1024 positions take the byte walk (crossover_bytes); those
// of 1025..4096 positions with at most 16 species the species-row walk
// (crossover_regs, compiled in only when REG); others the scan walk, which finds p
// and q with 64-position ballots over the path copy in LDS.
template <bool REG>
__global__ __launch_bounds__(64) void k_ga_child(
    int64_t n, int32_t M, int32_t S, int32_t E, const int32_t* __restrict__ tab, const int32_t* __restrict__ spos,
    const int32_t* __restrict__ spos_inv, const uint8_t* __restrict__ msub, const int32_t* __restrict__ mob,
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
    // B); then the register walk's 16 x 64 words of species rows
    const int Mr = (int)round_up(M, 16);
    uint8_t* ch = lds;
    uint8_t* rf = lds + Mr;
    uint8_t* bb = lds + 2 * Mr;
    uint64_t* mk = reinterpret_cast<uint64_t*>(lds + round_up(3 * (int64_t)Mr, 16));
    const uint8_t* A = pop_in + pa * n;
    const uint8_t* B = pop_in + pb * n;
    for (int x = lane; x < M; x += 64) {
        const int site = mob[spos[x]];
        const uint8_t a = A[site];
        ch[x] = a;
        rf[x] = a;
        bb[x] = B[site];
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
        if (REG && len <= kRegMaxLen && E <= kRegSpecies) {
            crossover_regs(rs, cs, bs, len, spos + base, mk, (uint32_t)c, g, seed, lane);
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
    for (int x = lane; x < M; x += 64) out[mob[spos[x]]] = ch[x];
    for (int f = lane; f < n_fixed; f += 64) out[fixed_idx[f]] = ref_occ[fixed_idx[f]];
}

// The register walk's arrays take most of the register file (one wavefront per
// SIMD), so its variant runs only for problems with a sublattice it walks.
static bool ga_reg_walk(const goac_problem* pb) {
    bool reg = false;
    for (int s = 0; s < pb->d.S; ++s) {
        const int len = pb->tab_host[2 + s];
        reg = reg || (len > kByteMaxLen && len <= kRegMaxLen && pb->d.E <= kRegSpecies);
    }
    return reg;
}

// LDS of a child: its occupation, the path copy and parent B (bytes), then the
// register walk's 16 x 64 words of species rows
size_t ga_child_lds(const goac_problem* pb) {
    return round_up(3 * round_up(pb->d.M, 16), 16) + (ga_reg_walk(pb) ? 8 * kRegSpecies * 64 : 0);
}

goac_status ga_children(goac_problem* pb, int64_t P, const uint8_t* pop_in, const uint64_t* cum, const int32_t* elite,
                        int32_t n_elite, const goac_ga_params* prm, uint8_t* pop_out, const uint32_t* g_dev) {
    goac_ctx* ctx = pb->ctx;
    const ProblemDev& d = pb->d;
    const bool reg = ga_reg_walk(pb);
    const size_t lds = ga_child_lds(pb);
    const void* fn = reg ? (const void*)k_ga_child<true> : (const void*)k_ga_child<false>;
    if (lds > 64 * 1024) GOAC_HIP(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    auto launch = reg ? k_ga_child<true> : k_ga_child<false>;
    hipLaunchKernelGGL(launch, dim3((unsigned)P), dim3(64), lds, ctx->stream, d.n, d.M, d.S, d.E, d.tab, pb->spos,
                       pb->spos_inv, d.msub, d.mob, pb->fixed_idx, pb->n_fixed, d.ref_occ, P, pop_in, cum, elite,
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
