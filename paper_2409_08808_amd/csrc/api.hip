// C ABI entry points of the gfx950 library (declared in include/goac.h): argument
// checks, problem derivation, chain-set management and kernel dispatch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.h"

namespace goac {

goac_status build_ewald(goac_ctx*, const double*, int64_t, const double*, const goac_ewald_params*, double*);

__global__ void k_init(int64_t, int32_t, int32_t, const int32_t*, const int32_t*, const int32_t*, const int32_t*,
                       int32_t, const uint8_t*, uint64_t, uint32_t, uint32_t, uint8_t*);
__global__ void k_ga_prep(int64_t, const double*, uint64_t*, int32_t*);
size_t ga_child_lds(const goac_problem* pb);
goac_status ga_children(goac_problem* pb, int64_t P, const uint8_t* pop_in, const uint64_t* cum, const int32_t* elite,
                        int32_t n_elite, const goac_ga_params* prm, uint8_t* pop_out, const uint32_t* g_dev);
goac_status anchor_batched(goac_ctx*, goac_chains*, int, uint32_t);
// rows of every group from its slot permutation (hybrid.hip)
__global__ void k_rows_from_slot(int64_t n_groups, int32_t R, const int32_t* __restrict__ slot,
                                 ChainScalars* __restrict__ sc);
constexpr int kInlineAnchorMaxMp = 1024;

// Arenas of problems and chain sets come from the context's block cache
// (lifetime.h): a released block is reused only by work queued after everything
// that used it, since all work of a context runs on its one stream.
goac_status pool_get(goac_ctx* ctx, size_t* bytes, void** out) {
    if (!ctx->pool.get(ctx->dev, bytes, out)) return fail(ctx, GOAC_ENOMEM, "device allocation failed");
    return GOAC_OK;
}

void pool_put(goac_ctx* ctx, void* p, size_t bytes) { ctx->pool.put(ctx->dev, p, bytes); }

// A copy from pinned memory is queued at once; one from pageable memory makes the
// host wait. The ring's halves take turns: a half is written again only once the
// event recorded when the copies from it were queued has completed, which the
// stream has long passed unless a half's worth of uploads is still queued.
goac_status upload(goac_ctx* ctx, void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return GOAC_OK;
    if (ctx->capturing) return fail(ctx, GOAC_EINVAL, "host copy inside a stream capture");
    const size_t need = (size_t)round_up((int64_t)bytes, 256);
    if (need > ctx->stage_half) {
        if (ctx->stage) {
            // queued copies may still read the old ring
            GOAC_HIP(ctx, hipStreamSynchronize(ctx->stream));
            GOAC_HIP(ctx, hipHostFree(ctx->stage));
            ctx->stage = nullptr;
        }
        const size_t half = std::max<size_t>((size_t)round_up((int64_t)need, 1 << 20), (size_t)4 << 20);
        GOAC_HIP(ctx, hipHostMalloc((void**)&ctx->stage, 2 * half, hipHostMallocDefault));
        ctx->stage_half = half;
        ctx->stage_off = 0;
        ctx->stage_cur = 0;
        ctx->stage_pending[0] = ctx->stage_pending[1] = false;
        for (int h = 0; h < 2; ++h)
            if (!ctx->stage_ev[h]) GOAC_HIP(ctx, hipEventCreateWithFlags(&ctx->stage_ev[h], hipEventDisableTiming));
    }
    if (ctx->stage_off + need > ctx->stage_half) {
        GOAC_HIP(ctx, hipEventRecord(ctx->stage_ev[ctx->stage_cur], ctx->stream));
        ctx->stage_pending[ctx->stage_cur] = true;
        ctx->stage_cur ^= 1;
        ctx->stage_off = 0;
        if (ctx->stage_pending[ctx->stage_cur]) {
            GOAC_HIP(ctx, hipEventSynchronize(ctx->stage_ev[ctx->stage_cur]));
            ctx->stage_pending[ctx->stage_cur] = false;
        }
    }
    char* s = ctx->stage + (size_t)ctx->stage_cur * ctx->stage_half + ctx->stage_off;
    std::memcpy(s, src, bytes);
    GOAC_HIP(ctx, hipMemcpyAsync(dst, s, bytes, hipMemcpyHostToDevice, ctx->stream));
    ctx->stage_off += need;
    return GOAC_OK;
}

goac_status workspace(goac_ctx* ctx, int slot, size_t bytes, void** out) {
    if (slot < 0 || slot >= kWsSlots) return fail(ctx, GOAC_EINVAL, "workspace slot");
    if (bytes > ctx->ws_size[slot]) {
        if (ctx->ws[slot]) {
            // work already queued may still read the old buffer
            GOAC_HIP(ctx, hipStreamSynchronize(ctx->stream));
            GOAC_HIP(ctx, hipFree(ctx->ws[slot]));
            ctx->ws[slot] = nullptr;
            ctx->ws_size[slot] = 0;
        }
        const size_t sz = round_up((int64_t)bytes, 1 << 20);
        GOAC_HIP(ctx, hipMalloc(&ctx->ws[slot], sz));
        ctx->ws_size[slot] = sz;
    }
    *out = ctx->ws[slot];
    return GOAC_OK;
}

// ------------------------------------------------------------------ problem derivation kernels

// V64/V32 (M x Mp) of the mobile block and the bf16 split (Mq x Mq) of the
// population product's weighted matrix W, zero-padded: with k and l in 128-wide
// tiles, W_kl = V_kl when l's tile is before k's, V_kl / 2 when they are the same
// tile, 0 after (1/2 q^T V q = sum over tiles j and tiles i <= j of the W-weighted
// blocks; halving is exact in bf16, so hi and lo of W are those of V halved)
__global__ void k_extract(int64_t n, int32_t M, int32_t Mp, int32_t Mq, const double* __restrict__ V,
                          const int32_t* __restrict__ mob, double* __restrict__ V64, float* __restrict__ V32,
                          __hip_bfloat16* __restrict__ Vhi, __hip_bfloat16* __restrict__ Vlo) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)Mq * Mq) return;
    const int k = (int)(idx / Mq), l = (int)(idx - (int64_t)k * Mq);
    double v = 0.0;
    if (k < M && l < M) v = V[(int64_t)mob[k] * n + mob[l]];
    if (k < M && l < Mp) {
        V64[(int64_t)k * Mp + l] = v;
        V32[(int64_t)k * Mp + l] = (float)v;
    }
    const int tk = k >> 7, tl = l >> 7;
    const double w = tl < tk ? v : (tl == tk ? 0.5 * v : 0.0);
    const __hip_bfloat16 hi = __float2bfloat16((float)w);
    const double rest = w - (double)__bfloat162float(hi);
    Vhi[idx] = hi;
    Vlo[idx] = __float2bfloat16((float)rest);
}

__device__ inline double wsum64(double x) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ inline double wmax64(double x) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) x = fmax(x, __shfl_xor(x, o, 64));
    return x;
}

// one wavefront per mobile row k: diag, rowmax (rounded up), rowabs = sum_l |V_kl|,
// h_k = sum_f V[mob_k][f] q_f over the fixed sites, vc_k = sum_l V_kl c_l and the
// field of the reference occupation phiref_k = h_k + sum_l V_kl q_l (fixed-order
// butterfly sums)
__global__ __launch_bounds__(256) void k_rows(int64_t n, int32_t M, int32_t Mp, const double* __restrict__ V,
                                              const int32_t* __restrict__ mob, const int32_t* __restrict__ fixed_idx,
                                              const double* __restrict__ fixed_q, int32_t n_fixed,
                                              const double* __restrict__ V64, const double* __restrict__ cvec,
                                              const double* __restrict__ qref, double* __restrict__ diag,
                                              float* __restrict__ rowmax, double* __restrict__ rowabs,
                                              double* __restrict__ h, double* __restrict__ vc,
                                              double* __restrict__ phiref) {
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= Mp) return;
    if (k >= M) {
        if (lane == 0) {
            h[k] = 0.0;
            vc[k] = 0.0;
        }
        return;
    }
    const double* row = V + (int64_t)mob[k] * n;
    double hs = 0.0;
    for (int f = lane; f < n_fixed; f += 64) hs += row[fixed_idx[f]] * fixed_q[f];
    const double* r64 = V64 + (int64_t)k * Mp;
    double s1 = 0.0, s2 = 0.0, mx = 0.0, ab = 0.0;
    for (int l = lane; l < M; l += 64) {
        const double v = r64[l];
        s1 += v * cvec[l];
        s2 += v * qref[l];
        mx = fmax(mx, fabs(v));
        ab += fabs(v);
    }
    hs = wsum64(hs);
    s1 = wsum64(s1);
    s2 = wsum64(s2);
    mx = wmax64(mx);
    ab = wsum64(ab);
    if (lane == 0) {
        diag[k] = r64[k];
        float r = (float)mx;
        if ((double)r < mx) r = nextafterf(r, INFINITY);
        rowmax[k] = r;
        rowabs[k] = ab;
        h[k] = hs;
        vc[k] = s1;
        phiref[k] = hs + s2;
    }
}

// fixed-ion energy terms, one wavefront per fixed row: out[f] = q_f sum_g V[f][g] q_g
__global__ __launch_bounds__(256) void k_fixed_energy(int64_t n, const int32_t* __restrict__ fixed_idx,
                                                      const double* __restrict__ fixed_q, int32_t n_fixed,
                                                      const double* __restrict__ V, double* __restrict__ out) {
    const int f = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (f >= n_fixed) return;
    const double* row = V + (int64_t)fixed_idx[f] * n;
    double s = 0.0;
    for (int g = lane; g < n_fixed; g += 64) s += row[fixed_idx[g]] * fixed_q[g];
    s = wsum64(s);
    if (lane == 0) out[f] = fixed_q[f] * s;
}

// one workgroup, fixed-order sums (per-thread strided partials, then a tree):
//   out[0] = E_ff = 1/2 sum efix,  out[1] = E~ = E_ff + sum c_k h_k + 1/2 sum c_k vc_k,
//   phibar[s] = mean of phiref over sublattice s; ht_k = h_k + vc_k;
//   out[2] = 2^sc, out[3] = 2^-sc: the scale of the population product's 64-bit
//   fixed-point row sums, sc the largest integer with 2^sc B < 2^61 for the bound
//   B = dqmax^2 sum_k rowabs_k + dqmax sum_k |ht_k| + 1 on the absolute terms of a
//   row's linear and quadratic parts (dqmax = the largest |charge - shift|)
__global__ __launch_bounds__(256) void k_derive_scalars(int32_t M, int32_t n_fixed, int32_t S,
                                                        const double* __restrict__ efix,
                                                        const double* __restrict__ cvec,
                                                        const double* __restrict__ h,
                                                        const double* __restrict__ vc,
                                                        const double* __restrict__ phiref,
                                                        const uint8_t* __restrict__ msub,
                                                        const double* __restrict__ rowabs, double dqmax,
                                                        double* __restrict__ ht, double* __restrict__ phibar,
                                                        double* __restrict__ out) {
    __shared__ double red[5 + kMaxSub][256];
    __shared__ int cnt[kMaxSub][256];
    const int t = threadIdx.x;
    double e = 0.0, ch = 0.0, cvc = 0.0, rab = 0.0, hab = 0.0;
    double acc[kMaxSub];
    int nc[kMaxSub];
    for (int s = 0; s < kMaxSub; ++s) { acc[s] = 0.0; nc[s] = 0; }
    for (int f = t; f < n_fixed; f += 256) e += efix[f];
    for (int k = t; k < M; k += 256) {
        ch += cvec[k] * h[k];
        cvc += cvec[k] * vc[k];
        ht[k] = h[k] + vc[k];
        rab += rowabs[k];
        hab += fabs(ht[k]);
        const int s = msub[k];
        for (int q = 0; q < kMaxSub; ++q)
            if (q == s) { acc[q] += phiref[k]; nc[q] += 1; }
    }
    red[0][t] = e;
    red[1][t] = ch;
    red[2][t] = cvc;
    for (int s = 0; s < kMaxSub; ++s) { red[3 + s][t] = acc[s]; cnt[s][t] = nc[s]; }
    red[3 + kMaxSub][t] = rab;
    red[4 + kMaxSub][t] = hab;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            for (int r = 0; r < 5 + kMaxSub; ++r) red[r][t] += red[r][t + w];
            for (int s = 0; s < kMaxSub; ++s) cnt[s][t] += cnt[s][t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double Eff = 0.5 * red[0][0];
        out[0] = Eff;
        out[1] = Eff + red[1][0] + 0.5 * red[2][0];
        for (int s = 0; s < S; ++s) phibar[s] = cnt[s][0] ? red[3 + s][0] / cnt[s][0] : 0.0;
        const double B = dqmax * dqmax * red[3 + kMaxSub][0] + dqmax * red[4 + kMaxSub][0] + 1.0;
        int ex = 0;
        (void)frexp(B, &ex);   // B < 2^ex
        out[2] = ldexp(1.0, 61 - ex);
        out[3] = ldexp(1.0, ex - 61);
    }
}

// ------------------------------------------------------------------ chain kernels

// Composition check of row c (Eq. 2's occupancy constraints): err |= 1 when a
// mobile site holds a species id >= E or the species counts of a sublattice differ
// from the problem's. One workgroup per row; each thread takes 16 consecutive
// sites per step with 16-byte loads of the row and of the per-site class table.
// With at most 16 (class, species) pairs the counts stay in registers, eight bits
// per pair in two 64-bit words (moved to 32-bit counters every eight steps, before
// a field can reach 256), then are summed over the workgroup; more pairs count
// into an LDS histogram.
__global__ __launch_bounds__(256) void k_check_comp(int64_t n, int32_t S, int32_t E, const int32_t* __restrict__ tab,
                                                    const int8_t* __restrict__ site_sub,
                                                    const uint8_t* __restrict__ occ, int32_t* __restrict__ err) {
    __shared__ int hist[kMaxSub * kMaxSpecies];
    const int64_t c = blockIdx.x;
    const int tid = threadIdx.x;
    const int nb = S * E;
    for (int x = tid; x < nb; x += 256) hist[x] = 0;
    __syncthreads();
    const uint8_t* row = occ + c * n;
    const bool vec = (n & 15) == 0 && (((uintptr_t)row) & 15) == 0 && (((uintptr_t)site_sub) & 15) == 0;
    bool bad = false;
    uint32_t tot[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) tot[b] = 0;
    uint64_t lo = 0, hi = 0;
    int blk = 0;
    auto flush = [&]() {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            tot[b] += (uint32_t)((lo >> (8 * b)) & 0xffu);
            tot[b + 8] += (uint32_t)((hi >> (8 * b)) & 0xffu);
        }
        lo = hi = 0;
    };
    for (int64_t x0 = (int64_t)tid * 16; x0 < n; x0 += 256 * 16) {
        uint8_t e16[16];
        int8_t s16[16];
        if (vec) {
            *reinterpret_cast<uint4*>(e16) = *reinterpret_cast<const uint4*>(row + x0);
            *reinterpret_cast<uint4*>(s16) = *reinterpret_cast<const uint4*>(site_sub + x0);
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const bool in = x0 + k < n;
                e16[k] = in ? row[x0 + k] : 0;
                s16[k] = in ? site_sub[x0 + k] : (int8_t)-1;
            }
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int s = s16[k], e = e16[k];
            if (s < 0) continue;
            if (e >= E) {
                bad = true;
                continue;
            }
            const int b = s * E + e;
            if (nb <= 16) {
                lo += b < 8 ? 1ull << (8 * (b & 7)) : 0ull;
                hi += b >= 8 ? 1ull << (8 * (b & 7)) : 0ull;
            } else {
                atomicAdd(&hist[b], 1);
            }
        }
        if (nb <= 16 && ++blk == 8) {
            flush();
            blk = 0;
        }
    }
    if (nb <= 16) {
        flush();
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            if (b < nb) {
                uint32_t v = tot[b];
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
                if ((tid & 63) == 0) atomicAdd(&hist[b], (int)v);
            }
        }
    }
    __syncthreads();
    const int32_t* cnt = tab + 2 + 2 * S;
    for (int x = tid; x < nb; x += 256)
        if (hist[x] != cnt[x]) bad = true;
    if (bad) atomicOr(err, 1);
}

// mobile occupation, perm (positions of each sublattice sorted by (species,
// position)) and, unless best is NULL, the best copy of one chain, and, unless sc
// is NULL, its fresh scalars; one wavefront per chain. Within a
// 64-position chunk the rank of a position among equal (sublattice, species)
// keys is a popcount of a ballot; running counts carry across chunks.
__global__ __launch_bounds__(64) void k_chain_setup(int64_t n, int32_t M, int32_t Mp, int32_t S, int32_t E,
                                                    const int32_t* __restrict__ tab, const int32_t* __restrict__ mob,
                                                    const uint8_t* __restrict__ msub, const uint8_t* __restrict__ occ,
                                                    int64_t first, const int64_t* __restrict__ offs,
                                                    uint8_t* __restrict__ occ_m, uint16_t* __restrict__ perm,
                                                    uint8_t* __restrict__ best, ChainScalars* __restrict__ sc,
                                                    int32_t inst, uint32_t id_base) {
    __shared__ int next[kMaxSub * kMaxSpecies];
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t off = offs[first + c];
    if (sc && lane == 0) {
        // a new chain: counters zero, ids and offset set
        ChainScalars z{};
        z.inst = inst;
        z.chain_id = id_base + (uint32_t)c;
        z.off = off;
        sc[first + c] = z;
    }
    const uint8_t* row = occ + c * n;
    const int32_t* subsize = tab + 2;
    const int32_t* suboff = subsize + S;
    const int32_t* offs_se = suboff + S + S * E;
    for (int x = lane; x < S * E; x += 64) next[x] = suboff[x / E] + offs_se[x];
    __syncthreads();
    for (int k0 = 0; k0 < Mp; k0 += 64) {
        const int k = k0 + lane;
        const bool mobile = k < M;
        const int e = mobile ? row[mob[k]] : 0;
        const int s = mobile ? msub[k] : 0;
        const int key = (mobile && e < E) ? s * E + e : -1;
        occ_m[off + k] = (uint8_t)e;
        if (best) best[off + k] = (uint8_t)e;
        if (!mobile) perm[off + k] = 0;
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        // each distinct key of the chunk in turn (uniform loop)
        uint64_t todo = __ballot(key >= 0);
        while (todo) {
            const int leader = (int)__ffsll((long long)todo) - 1;
            const int kk = __shfl(key, leader, 64);
            const uint64_t m = __ballot(key == kk);
            if (key == kk) {
                const int at = next[kk] + __popcll(m & below);
                if (at < suboff[s] + subsize[s]) perm[off + at] = (uint16_t)k;
            }
            __syncthreads();
            if (lane == 0) next[kk] += __popcll(m);
            __syncthreads();
            todo &= ~m;
        }
    }
}

// field and energy of every chain of one instance from Phi = Q V_mm (FP64):
// phi = Phi + h; E = E_ff + 1/2 sum q (phi + h); MIXED stores phi - phibar_s in
// FP32 with its error bound. A start sets the best energy; a reload keeps the
// best (energy and occupation) unless the new occupation is strictly lower.
template <bool MIXED>
__global__ __launch_bounds__(256) void k_chain_field(int32_t M, int32_t Mp, const double* __restrict__ Q,
                                                     const double* __restrict__ Phi, const double* __restrict__ h,
                                                     const double* __restrict__ rowabs, double qmax,
                                                     const uint8_t* __restrict__ msub,
                                                     const double* __restrict__ phibar, const double* __restrict__ Ed,
                                                     int64_t first,
                                                     ChainScalars* __restrict__ sc, void* __restrict__ phi,
                                                     int reload, const uint8_t* __restrict__ occ_m,
                                                     uint8_t* __restrict__ best) {
    __shared__ double s_a[256], s_b[256], s_c[256];
    __shared__ int s_copy;
    const int64_t c = blockIdx.x;
    ChainScalars* S = sc + first + c;
    const int64_t off = S->off;
    double es = 0.0, pm = 0.0, am = 0.0;
    for (int k = threadIdx.x; k < Mp; k += 256) {
        const double q = Q[c * Mp + k];
        const double p = k < M ? Phi[c * Mp + k] + h[k] : 0.0;
        if (k < M) es += q * (p + h[k]);
        if (MIXED) {
            const float v = k < M ? (float)(p - phibar[msub[k]]) : 0.0f;
            reinterpret_cast<float*>(phi)[off + k] = v;
            pm = fmax(pm, fabs((double)v));
            if (k < M) am = fmax(am, fabs(h[k]) + qmax * rowabs[k]);
        } else {
            reinterpret_cast<double*>(phi)[off + k] = p;
        }
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
        const double E = Ed[0] + 0.5 * s_a[0];
        S->E = E;
        // a start sets the best; a reload replaces it only when strictly lower
        const bool better = !reload || E < S->best_E;
        if (better) S->best_E = E;
        s_copy = reload && better;
        S->since_anchor = 0;
        S->status = 0;
        if (MIXED) {
            const double gM = (double)(M + 2) * 0x1p-53 * 1.01;
            S->eps = 0x1p-24 * s_b[0] * 1.0001 + gM * s_c[0] * 2.0;
            float pb = 1.0f;
            while ((double)pb < 2.0 * s_b[0]) pb *= 2.0f;
            S->phibound = pb;
        } else {
            S->eps = 0.0;
            S->phibound = 0.0f;
        }
    }
    __syncthreads();
    if (s_copy)
        for (int k = threadIdx.x; k < Mp; k += 256) best[off + k] = occ_m[off + k];
}

__global__ void k_export(int64_t n, int32_t M, const int32_t* __restrict__ mob, const int32_t* __restrict__ fixed_idx,
                         int32_t n_fixed, const uint8_t* __restrict__ ref_occ, int64_t first,
                         const ChainScalars* __restrict__ sc, const uint8_t* __restrict__ occ_m,
                         const uint8_t* __restrict__ best_m, uint8_t* __restrict__ occ_out,
                         uint8_t* __restrict__ best_out, goac_chain_stats* __restrict__ stats) {
    const int64_t c = blockIdx.x;
    const ChainScalars& S = sc[first + c];
    const int64_t g = first + c;
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        if (occ_out) occ_out[g * n + mob[k]] = occ_m[S.off + k];
        if (best_out) best_out[g * n + mob[k]] = best_m[S.off + k];
    }
    for (int f = threadIdx.x; f < n_fixed; f += blockDim.x) {
        if (occ_out) occ_out[g * n + fixed_idx[f]] = ref_occ[fixed_idx[f]];
        if (best_out) best_out[g * n + fixed_idx[f]] = ref_occ[fixed_idx[f]];
    }
    if (threadIdx.x == 0 && stats) {
        goac_chain_stats o;
        o.t = S.t;
        o.accepts = S.accepts;
        o.updates = S.updates;
        o.hash = S.hash;
        o.fallbacks = S.fallbacks;
        o.anchors = S.anchors;
        o.E = S.E;
        o.best_E = S.best_E;
        o.status = S.status;
        o.row = S.row;
        stats[g] = o;
    }
}

// replica exchange: one workgroup per group of R consecutive chains. The slots
// are checked to be a permutation of 0..R-1 (an LDS bit per value); the pairs of
// the step are disjoint, so each is decided by its own thread and the outcome is
// that of deciding them in order. x_dev, when given, holds the step index (a
// captured round reads it); the last workgroup to finish then advances it and
// clears the sweep's work counter for the next round.
__global__ void k_remc(int32_t R, const double* __restrict__ kT, uint64_t x, uint64_t* x_dev, uint64_t seed,
                       ChainScalars* __restrict__ sc, int32_t* __restrict__ slot, uint8_t* __restrict__ acc,
                       uint32_t* ticket, int32_t* queue) {
    extern __shared__ uint32_t seen[];
    __shared__ int s_bad;
    __shared__ uint64_t s_x;
    const int tid = threadIdx.x, bs = blockDim.x;
    const int64_t g = blockIdx.x;
    int32_t* sl = slot + g * R;
    ChainScalars* gs = sc + g * R;
    for (int w = tid; w < (R + 31) / 32; w += bs) seen[w] = 0;
    if (tid == 0) {
        s_bad = 0;
        s_x = x_dev ? *x_dev : x;   // read once, before this workgroup takes its ticket
    }
    __syncthreads();
    x = s_x;
    for (int k = tid; k < R; k += bs) {
        const int32_t v = sl[k];
        if (acc) acc[g * R + k] = 0;
        if ((uint32_t)v >= (uint32_t)R) {
            s_bad = 1;
        } else {
            const uint32_t bit = 1u << (v & 31);
            if (atomicOr(&seen[v >> 5], bit) & bit) s_bad = 1;
        }
    }
    __syncthreads();
    if (!s_bad) {   // otherwise the group is left unchanged
        const int par = (int)(x & 1u);
        for (int k = par + 2 * tid; k + 1 < R; k += 2 * bs) {
            const int32_t a = sl[k], b = sl[k + 1];
            const u32x4 r = philox((uint32_t)k, (uint32_t)x, (uint32_t)(x >> 32), ((uint32_t)g << 8) | TAG_REMC, seed);
            const double u = unit_open(r.x, r.y);
            const double arg = (gs[a].E - gs[b].E) * (1.0 / kT[k] - 1.0 / kT[k + 1]);
            const bool ok = (arg >= 0.0) || (u < exp(arg));
            if (acc) acc[g * R + k] = ok ? 1 : 0;
            if (ok) {
                sl[k] = b;
                sl[k + 1] = a;
            }
            gs[ok ? b : a].row = k;
            gs[ok ? a : b].row = k + 1;
        }
        // the positions outside every pair keep their chains
        if (tid == 0) {
            if (par) gs[sl[0]].row = 0;
            if ((R - par) & 1) gs[sl[R - 1]].row = R - 1;
        }
    }
    if (ticket) {
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            if (atomicAdd(ticket, 1u) == gridDim.x - 1) {
                __threadfence();
                *ticket = 0;
                *queue = 0;
                *x_dev = x + 1;
                __threadfence();
            }
        }
    }
}

__global__ void k_set_rows(int64_t C, const int32_t* __restrict__ rows, ChainScalars* __restrict__ sc) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C) sc[c].row = rows[c];
}

// step index, ticket and work counter of a captured replica-exchange round
__global__ void k_remc_init(uint64_t* x_dev, uint64_t x0, uint32_t* ticket, int32_t* queue) {
    *x_dev = x0;
    *ticket = 0;
    *queue = 0;
}

__global__ void k_zero_i32(int32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// *flag |= 1 when a chain's FP32 field has left its error bound
__global__ void k_drift_flag(int64_t C, const ChainScalars* __restrict__ sc, int32_t* __restrict__ flag) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C && sc[c].status) atomicOr(flag, 1);
}

// the verdict word, its pinned host copy and the event after the copy
static goac_status check_buffers(goac_ctx* ctx) {
    if (!ctx->chk_dev) GOAC_HIP(ctx, hipMalloc((void**)&ctx->chk_dev, 256));
    if (!ctx->chk_host) GOAC_HIP(ctx, hipHostMalloc((void**)&ctx->chk_host, 256, hipHostMallocDefault));
    if (!ctx->chk_ev) GOAC_HIP(ctx, hipEventCreateWithFlags(&ctx->chk_ev, hipEventDisableTiming));
    return GOAC_OK;
}

// queue the copy of the verdict to the host and the event after it
static goac_status check_publish(goac_ctx* ctx) {
    GOAC_HIP(ctx, hipMemcpyAsync(ctx->chk_host, ctx->chk_dev, 4, hipMemcpyDeviceToHost, ctx->stream));
    GOAC_HIP(ctx, hipEventRecord(ctx->chk_ev, ctx->stream));
    return GOAC_OK;
}

goac_status rows_check_launch(goac_problem* pb, int64_t P, const uint8_t* occ, int32_t* flag) {
    goac_ctx* ctx = pb->ctx;
    if (P < 0 || P > ((int64_t)1 << 30) || (P > 0 && !occ)) return fail(ctx, GOAC_EINVAL, "row check: bad rows");
    const ProblemDev& d = pb->d;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, flag, 1);
    if (P > 0)
        hipLaunchKernelGGL(k_check_comp, dim3((unsigned)P), dim3(256), 0, ctx->stream, d.n, d.S, d.E, d.tab,
                           d.site_sub, occ, flag);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

goac_status rows_check_enqueue(goac_problem* pb, int64_t P, const uint8_t* occ) {
    goac_ctx* ctx = pb->ctx;
    if (ctx->capturing) return fail(ctx, GOAC_EINVAL, "row check inside a stream capture");
    GOAC_TRY(check_buffers(ctx));
    GOAC_TRY(rows_check_launch(pb, P, occ, ctx->chk_dev));
    return check_publish(ctx);
}

goac_status rows_check_wait(goac_ctx* ctx, const char* who) {
    // the check is short: poll its event for up to 2 ms, so the host answers at
    // once and the next call's kernels follow without a gap, then block
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t q = hipEventQuery(ctx->chk_ev);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) GOAC_HIP(ctx, q);
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
            GOAC_HIP(ctx, hipEventSynchronize(ctx->chk_ev));
            break;
        }
    }
    if (*ctx->chk_host)
        return fail(ctx, GOAC_EINVAL,
                    std::string(who) + ": an occupation holds an unknown species or breaks the problem's composition");
    return GOAC_OK;
}

}  // namespace goac

using namespace goac;

// ------------------------------------------------------------------ helpers
namespace {

struct DevAllocs {
    std::vector<void*> ptrs;
    ~DevAllocs() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    void release() { ptrs.clear(); }
};

template <typename T>
goac_status dalloc(goac_ctx* ctx, T** p, size_t count, DevAllocs* track = nullptr) {
    void* q = nullptr;
    GOAC_HIP(ctx, hipMalloc(&q, std::max<size_t>(count * sizeof(T), 16)));
    *p = (T*)q;
    if (track) track->ptrs.push_back(q);
    return GOAC_OK;
}

// Byte offsets of the sub-arrays of one device arena (256-byte aligned).
struct ArenaPlan {
    size_t end = 0;
    size_t take(size_t bytes) {
        const size_t o = (size_t)round_up((int64_t)end, 256);
        end = o + std::max<size_t>(bytes, 1);
        return o;
    }
};

void problem_free(goac_problem* pb) {
    if (pb->arena) pool_put(pb->ctx, pb->arena, pb->arena_bytes);
    pb->arena = nullptr;
}

}  // namespace

// ------------------------------------------------------------------ context
extern "C" goac_status goac_ctx_create(int device, void* hip_stream, goac_ctx** out) {
    if (!out) return GOAC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GOAC_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return GOAC_EHIP;
    goac_ctx* ctx = new goac_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->dev.stream = ctx->stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
    // the device address of the allocation-free entry point's scratch array
    if (noalloc_setup(device) != hipSuccess) {
        delete ctx;
        return GOAC_EHIP;
    }
    *out = ctx;
    return GOAC_OK;
}

// The context is freed once the caller has released it and no problem or chain
// set made on it is left, in whichever order the two happen (lifetime.h).
static void ctx_free(goac_ctx* ctx) {
    (void)hipStreamSynchronize(ctx->stream);
    for (int q = 0; q < kWsSlots; ++q)
        if (ctx->ws[q]) (void)hipFree(ctx->ws[q]);
    ctx->pool.clear(ctx->dev);
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    for (int h = 0; h < 2; ++h)
        if (ctx->stage_ev[h]) (void)hipEventDestroy(ctx->stage_ev[h]);
    if (ctx->chk_dev) (void)hipFree(ctx->chk_dev);
    if (ctx->chk_host) (void)hipHostFree(ctx->chk_host);
    if (ctx->chk_ev) (void)hipEventDestroy(ctx->chk_ev);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    delete ctx;
}

extern "C" void goac_ctx_destroy(goac_ctx* ctx) { release_context(ctx, ctx_free); }

extern "C" const char* goac_last_error(const goac_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" goac_status goac_ctx_synchronize(goac_ctx* ctx) {
    if (!ctx) return GOAC_EINVAL;
    GOAC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GOAC_OK;
}

// ------------------------------------------------------------------ Ewald
extern "C" goac_status goac_build_ewald(goac_ctx* ctx, const double lattice[9], int64_t n, const double* pos,
                                        const goac_ewald_params* params, double* V) {
    if (!ctx) return GOAC_EINVAL;
    if (!lattice || !pos || !V || n <= 0 || n > 65536)
        return fail(ctx, GOAC_EINVAL, "build_ewald: null pointer or n outside [1, 65536]");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    return goac::build_ewald(ctx, lattice, n, pos, params, V);
}

// ------------------------------------------------------------------ problem
extern "C" goac_status goac_problem_create(goac_ctx* ctx, const double* V, int64_t n, const int32_t* sub,
                                           const uint8_t* species, int32_t n_species, const double* charge,
                                           goac_problem** out) {
    if (!ctx) return GOAC_EINVAL;
    if (!out || !V || !sub || !species || !charge || n <= 0)
        return fail(ctx, GOAC_EINVAL, "problem_create: null pointer or n <= 0");
    *out = nullptr;
    if (n_species <= 0 || n_species > kMaxSpecies)
        return fail(ctx, GOAC_EINVAL, "problem_create: n_species outside [1, 32]");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    int S = 0;
    std::vector<int32_t> mob, fixed;
    std::vector<double> fq;
    double qsum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (species[i] >= n_species) return fail(ctx, GOAC_EINVAL, "problem_create: species id >= n_species");
        if (sub[i] >= kMaxSub) return fail(ctx, GOAC_EINVAL, "problem_create: sublattice id >= 16");
        qsum += charge[species[i]];
        if (sub[i] >= 0) {
            mob.push_back((int32_t)i);
            S = std::max(S, sub[i] + 1);
        } else {
            fixed.push_back((int32_t)i);
            fq.push_back(charge[species[i]]);
        }
    }
    if (!(std::fabs(qsum) <= 1e-9)) return fail(ctx, GOAC_ENOTNEUTRAL, "problem_create: total charge is not zero");
    const int32_t M = (int32_t)mob.size();
    if (M == 0 || M > 65535) return fail(ctx, GOAC_EINVAL, "problem_create: need 1..65535 mobile positions");
    const int32_t E = n_species;
    const int32_t Mp = (int32_t)round_up(M, kPad);
    const int32_t Mq = (int32_t)round_up(M, 128);
    std::vector<uint8_t> msub(Mp, 0);
    std::vector<int32_t> tab(tab_words(S, E), 0);
    tab[0] = S;
    tab[1] = E;
    int32_t* subsize = tab.data() + 2;
    int32_t* suboff = subsize + S;
    int32_t* cnt = suboff + S;
    int32_t* offs = cnt + S * E;
    for (int32_t k = 0; k < M; ++k) {
        msub[k] = (uint8_t)sub[mob[k]];
        subsize[msub[k]]++;
        cnt[msub[k] * E + species[mob[k]]]++;
    }
    for (int s = 0, acc = 0; s < S; ++s) {
        if (subsize[s] == 0) return fail(ctx, GOAC_EINVAL, "problem_create: sublattice ids must be dense 0..S-1");
        suboff[s] = acc;
        acc += subsize[s];
        for (int e = 0, o = 0; e < E; ++e) {
            offs[s * E + e] = o;
            o += cnt[s * E + e];
        }
    }
    // positions of each sublattice in ascending order, and the inverse map
    std::vector<int32_t> spos(M), spos_inv(M);
    {
        std::vector<int32_t> nxt(suboff, suboff + S);
        for (int32_t k = 0; k < M; ++k) {
            spos[nxt[msub[k]]] = k;
            spos_inv[k] = nxt[msub[k]]++;
        }
    }
    // integer shift per sublattice: nearest integer to the mean charge
    std::vector<double> shift(S, 0.0), dq(S * E, 0.0), cvec(Mp, 0.0), qref(Mp, 0.0);
    int exact = 1;
    for (int s = 0; s < S; ++s) {
        double tot = 0.0;
        for (int e = 0; e < E; ++e) tot += cnt[s * E + e] * charge[e];
        shift[s] = std::nearbyint(tot / subsize[s]);
        for (int e = 0; e < E; ++e) {
            const double v = charge[e] - shift[s];
            dq[s * E + e] = v;
            if (cnt[s * E + e] > 0) {
                const float f = (float)v;
                const double back = (double)__bfloat162float(__float2bfloat16(f));
                if (back != v) exact = 0;
            }
        }
    }
    for (int32_t k = 0; k < M; ++k) {
        cvec[k] = shift[msub[k]];
        qref[k] = charge[species[mob[k]]];
    }

    goac_problem* pb = new goac_problem();
    pb->ctx = ctx;
    ProblemDev& d = pb->d;
    d.n = n;
    d.M = M;
    d.Mp = Mp;
    d.Mq = Mq;
    d.S = S;
    d.E = E;
    d.mixed_exact = exact;
    d.qmax = 0.0;
    for (int e = 0; e < E; ++e) d.qmax = std::max(d.qmax, std::fabs(charge[e]));
    pb->tab_host = tab;
    pb->mob_host = mob;
    pb->charge_host.assign(charge, charge + E);
    pb->shift_host = shift;
    pb->n_fixed = (int32_t)fixed.size();
    auto bail = [&](goac_status s) {
        problem_free(pb);
        delete pb;
        return s;
    };
    // one arena: the uploaded tables (one copy from a packed host image), then the
    // derived device-only arrays
    const int32_t nf = (int32_t)fixed.size();
    ArenaPlan ap;
    const size_t o_mob = ap.take(M * 4), o_msub = ap.take(Mp), o_ref = ap.take(n), o_ssub = ap.take(n),
                 o_chg = ap.take(E * 8),
                 o_dq = ap.take(S * E * 8), o_tab = ap.take(tab.size() * 4), o_spos = ap.take(M * 4),
                 o_sinv = ap.take(M * 4), o_site = ap.take(M * 4), o_fix = ap.take((nf + 1) * 4),
                 o_fq = ap.take((nf + 1) * 8),
                 o_c = ap.take(Mp * 8), o_q = ap.take(Mp * 8);
    const size_t up_end = ap.end;
    const size_t o_V64 = ap.take((size_t)M * Mp * 8), o_V32 = ap.take((size_t)M * Mp * 4),
                 o_hi = ap.take((size_t)Mq * Mq * 2), o_lo = ap.take((size_t)Mq * Mq * 2), o_diag = ap.take(M * 8),
                 o_rmax = ap.take(M * 4), o_rabs = ap.take(M * 8), o_h = ap.take(Mp * 8), o_ht = ap.take(Mp * 8),
                 o_pbar = ap.take(kMaxSub * 8), o_efix = ap.take((nf + 1) * 8), o_vc = ap.take(Mp * 8),
                 o_phi = ap.take(Mp * 8), o_out = ap.take(64);
    pb->arena_bytes = ap.end;
    if (pool_get(ctx, &pb->arena_bytes, &pb->arena) != GOAC_OK) {
        ctx->err = "problem_create: device allocation failed";
        return bail(GOAC_ENOMEM);
    }
    char* base = (char*)pb->arena;
    d.mob = (int32_t*)(base + o_mob);
    d.msub = (uint8_t*)(base + o_msub);
    d.ref_occ = (uint8_t*)(base + o_ref);
    d.site_sub = (int8_t*)(base + o_ssub);
    d.charge = (double*)(base + o_chg);
    d.dq = (double*)(base + o_dq);
    d.tab = (int32_t*)(base + o_tab);
    pb->spos = (int32_t*)(base + o_spos);
    pb->spos_inv = (int32_t*)(base + o_sinv);
    pb->ssite = (int32_t*)(base + o_site);
    pb->fixed_idx = (int32_t*)(base + o_fix);
    double* w_fq = (double*)(base + o_fq);
    double* w_c = (double*)(base + o_c);
    double* w_q = (double*)(base + o_q);
    d.V64 = (double*)(base + o_V64);
    d.V32 = (float*)(base + o_V32);
    d.Vhi = (__hip_bfloat16*)(base + o_hi);
    d.Vlo = (__hip_bfloat16*)(base + o_lo);
    d.diag = (double*)(base + o_diag);
    d.rowmax = (float*)(base + o_rmax);
    d.rowabs = (double*)(base + o_rabs);
    d.h = (double*)(base + o_h);
    d.ht = (double*)(base + o_ht);
    d.phibar = (double*)(base + o_pbar);
    double* w_efix = (double*)(base + o_efix);
    double* w_vc = (double*)(base + o_vc);
    double* w_phi = (double*)(base + o_phi);
    double* w_out = (double*)(base + o_out);
    std::vector<char> img(up_end, 0);
    std::memcpy(img.data() + o_mob, mob.data(), M * 4);
    std::memcpy(img.data() + o_msub, msub.data(), Mp);
    std::memcpy(img.data() + o_ref, species, n);
    for (int64_t x = 0; x < n; ++x) reinterpret_cast<int8_t*>(img.data() + o_ssub)[x] = (int8_t)(sub[x] < 0 ? -1 : sub[x]);
    std::memcpy(img.data() + o_chg, charge, E * 8);
    std::memcpy(img.data() + o_dq, dq.data(), S * E * 8);
    std::memcpy(img.data() + o_tab, tab.data(), tab.size() * 4);
    std::memcpy(img.data() + o_spos, spos.data(), M * 4);
    std::memcpy(img.data() + o_sinv, spos_inv.data(), M * 4);
    for (int32_t x = 0; x < M; ++x) reinterpret_cast<int32_t*>(img.data() + o_site)[x] = mob[spos[x]];
    if (nf) std::memcpy(img.data() + o_fix, fixed.data(), nf * 4);
    if (nf) std::memcpy(img.data() + o_fq, fq.data(), nf * 8);
    std::memcpy(img.data() + o_c, cvec.data(), Mp * 8);
    std::memcpy(img.data() + o_q, qref.data(), Mp * 8);
    hipStream_t sm = ctx->stream;
    if (upload(ctx, base, img.data(), up_end) != GOAC_OK) return bail(GOAC_EHIP);
    {
        const int64_t tot = (int64_t)Mq * Mq;
        hipLaunchKernelGGL(k_extract, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, sm, n, M, Mp, Mq, V, d.mob,
                           d.V64, d.V32, d.Vhi, d.Vlo);
        hipLaunchKernelGGL(k_rows, dim3((unsigned)((Mp + 3) / 4)), dim3(256), 0, sm, n, M, Mp, V, d.mob,
                           pb->fixed_idx, w_fq, nf, d.V64, w_c, w_q, d.diag, d.rowmax, d.rowabs, d.h, w_vc, w_phi);
        if (nf)
            hipLaunchKernelGGL(k_fixed_energy, dim3((unsigned)((nf + 3) / 4)), dim3(256), 0, sm, n, pb->fixed_idx,
                               w_fq, nf, V, w_efix);
        double dqmax = 0.0;
        for (double x : dq) dqmax = std::max(dqmax, std::fabs(x));
        hipLaunchKernelGGL(k_derive_scalars, dim3(1), dim3(256), 0, sm, M, nf, S, w_efix, w_c, d.h, w_vc, w_phi,
                           d.msub, d.rowabs, dqmax, d.ht, d.phibar, w_out);
        if (hipGetLastError() != hipSuccess) {
            ctx->err = "problem_create: launch failed";
            return bail(GOAC_EHIP);
        }
        // E_ff and E_t stay on the device; kernels read them there
        d.Ed = w_out;
    }
    // ht beyond M is zero
    if (Mp > M && hipMemsetAsync(d.ht + M, 0, (Mp - M) * 8, sm) != hipSuccess) return bail(GOAC_EHIP);
    ctx->holders.attach();
    *out = pb;
    return GOAC_OK;
}

// Destruction does not wait for the stream: the arena returns to the context's
// cache, whose blocks only work queued later on the same stream reuses.
extern "C" void goac_problem_destroy(goac_problem* pb) {
    if (!pb) return;
    destroy_dependent(pb->ctx, pb, problem_free, ctx_free);
}

extern "C" goac_status goac_problem_get_info(const goac_problem* pb, goac_problem_info* out) {
    if (!pb || !out) return GOAC_EINVAL;
    out->n = pb->d.n;
    out->M = pb->d.M;
    out->n_sublattices = pb->d.S;
    out->n_species = pb->d.E;
    if (!pb->e_host) {
        double e[2];
        if (hipSetDevice(pb->ctx->device) != hipSuccess ||
            hipMemcpyAsync(e, pb->d.Ed, 16, hipMemcpyDeviceToHost, pb->ctx->stream) != hipSuccess ||
            hipStreamSynchronize(pb->ctx->stream) != hipSuccess)
            return fail(pb->ctx, GOAC_EHIP, "problem_get_info: reading the fixed-ion energy failed");
        pb->E_ff = e[0];
        pb->E_t = e[1];
        pb->e_host = true;
    }
    out->E_fixed = pb->E_ff;
    out->mixed_exact = pb->d.mixed_exact;
    out->reserved = 0;
    return GOAC_OK;
}

extern "C" goac_status goac_init_occupations(goac_problem* pb, int64_t C, uint64_t seed, uint32_t chain_base,
                                             uint32_t instance, uint8_t* occ) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (C < 0 || (C > 0 && !occ)) return fail(ctx, GOAC_EINVAL, "init_occupations: bad arguments");
    if (C == 0) return GOAC_OK;
    if (instance >= (1u << 24)) return fail(ctx, GOAC_EINVAL, "init_occupations: instance id >= 2^24");
    const ProblemDev& d = pb->d;
    int maxP = 0;
    for (int s = 0; s < d.S; ++s) maxP = std::max(maxP, pb->tab_host[2 + s]);
    const size_t lds = round_up(maxP, 16) + 2 * (size_t)maxP + 16;
    if (lds > 160 * 1024) return fail(ctx, GOAC_EINVAL, "init_occupations: sublattice too large");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    if (lds > 64 * 1024)
        GOAC_HIP(ctx, hipFuncSetAttribute((const void*)k_init, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_init, dim3((unsigned)(C * d.S)), dim3(128), lds, ctx->stream, d.n, d.S, d.E, d.tab, pb->spos,
                       d.mob, pb->fixed_idx, pb->n_fixed, d.ref_occ, seed, chain_base, instance, occ);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

// ------------------------------------------------------------------ energies, top-k
extern "C" goac_status goac_energies(goac_problem* pb, int64_t P, const uint8_t* occ, goac_precision prec,
                                     double* E) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (P < 0 || P > ((int64_t)1 << 30) || (P > 0 && (!occ || !E)))
        return fail(ctx, GOAC_EINVAL, "energies: bad arguments");
    if (prec != GOAC_FP64 && prec != GOAC_MIXED) return fail(ctx, GOAC_EINVAL, "energies: unknown precision");
    if (prec == GOAC_MIXED && !pb->d.mixed_exact)
        return fail(ctx, GOAC_EINEXACT, "energies: a shifted charge is not bf16-exact");
    if (P == 0) return GOAC_OK;
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    // The rows are checked first (the mixed path's row kernel checks them as it
    // reads them). The energy kernels are queued right behind the check and skip
    // their work when it failed, so the host waits for the check alone while the
    // device goes on without a gap; a rejected call leaves E as it was.
    if (prec == GOAC_MIXED) {
        if (ctx->capturing) return fail(ctx, GOAC_EINVAL, "energies: row check inside a stream capture");
        GOAC_TRY(check_buffers(ctx));
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, ctx->chk_dev, 1);
        GOAC_CHECK_LAUNCH(ctx);
        GOAC_TRY(energies_mixed(pb, P, occ, E, 0, ctx->chk_dev, nullptr, ctx->chk_host, ctx->chk_ev));
    } else {
        GOAC_TRY(rows_check_enqueue(pb, P, occ));
        GOAC_TRY(energies_fp64(pb, P, occ, E, ctx->chk_dev));
    }
    return rows_check_wait(ctx, "energies");
}

// tiles of the mixed population product: 1, 2, 4 or 8 n-tiles of 128 positions per
// K block, no more than the problem has (one always works)
static bool valid_pop_kt(const goac_problem* pb, int32_t kt) {
    const int32_t nt = (pb->d.Mp + 127) / 128;
    return (kt == 1 || kt == 2 || kt == 4 || kt == 8) && (kt == 1 || kt <= nt);
}

extern "C" goac_status goac_energies_tile(goac_problem* pb, int64_t P, int32_t kt) {
    if (!pb) return GOAC_EINVAL;
    if (P <= 0) return fail(pb->ctx, GOAC_EINVAL, "energies_tile: P must be positive");
    if (kt == 0) {
        pb->pop_kt.erase(P);
        return GOAC_OK;
    }
    if (!valid_pop_kt(pb, kt)) return fail(pb->ctx, GOAC_EINVAL, "energies_tile: tile not 1, 2, 4 or 8 n-tiles within the problem");
    pb->pop_kt[P] = kt;
    return GOAC_OK;
}

// Times the mixed energies of the given population with each tile (one warm-up
// and the best of three timed calls, HIP events on the context's stream) and keeps
// the fastest for later calls with the same population size.
extern "C" goac_status goac_energies_autotune(goac_problem* pb, int64_t P, const uint8_t* occ, int32_t* kt_out) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (P <= 0 || !occ) return fail(ctx, GOAC_EINVAL, "energies_autotune: bad arguments");
    if (!pb->d.mixed_exact) return fail(ctx, GOAC_EINEXACT, "energies_autotune: a shifted charge is not bf16-exact");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    GOAC_TRY(rows_check(pb, P, occ, "energies_autotune"));
    size_t bytes = (size_t)P * 8;
    void* buf = nullptr;
    GOAC_TRY(pool_get(ctx, &bytes, &buf));
    double* E = (double*)buf;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t ec = hipEventCreate(&e0);
    if (ec == hipSuccess) ec = hipEventCreate(&e1);
    goac_status st = GOAC_OK;
    int32_t best = 0;
    float best_ms = 0.0f;
    for (int32_t kt = 1; kt <= 8 && st == GOAC_OK && ec == hipSuccess; kt *= 2) {
        if (!valid_pop_kt(pb, kt)) continue;
        st = energies_mixed(pb, P, occ, E, kt);
        float t_min = -1.0f;
        for (int rep = 0; rep < 3 && st == GOAC_OK && ec == hipSuccess; ++rep) {
            ec = hipEventRecord(e0, ctx->stream);
            if (ec == hipSuccess) st = energies_mixed(pb, P, occ, E, kt);
            if (ec == hipSuccess && st == GOAC_OK) ec = hipEventRecord(e1, ctx->stream);
            if (ec == hipSuccess && st == GOAC_OK) ec = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (ec == hipSuccess && st == GOAC_OK) ec = hipEventElapsedTime(&ms, e0, e1);
            if (ec == hipSuccess && st == GOAC_OK && (t_min < 0.0f || ms < t_min)) t_min = ms;
        }
        if (st == GOAC_OK && ec == hipSuccess && (best == 0 || t_min < best_ms)) {
            best = kt;
            best_ms = t_min;
        }
    }
    (void)hipStreamSynchronize(ctx->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    pool_put(ctx, buf, bytes);
    if (st != GOAC_OK) return st;
    if (ec != hipSuccess) return fail(ctx, GOAC_EHIP, std::string("energies_autotune: ") + hipGetErrorString(ec));
    pb->pop_kt[P] = best;
    if (kt_out) *kt_out = best;
    return GOAC_OK;
}

extern "C" goac_status goac_topk_fp64(goac_problem* pb, int64_t P, const uint8_t* occ, int32_t k, int64_t* idx,
                                      double* Eout) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (P <= 0 || k <= 0 || k > P || !occ || !idx || !Eout) return fail(ctx, GOAC_EINVAL, "topk: bad arguments");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    GOAC_TRY(rows_check(pb, P, occ, "topk"));
    const size_t bE = round_up(P * 8, 256), bC = round_up(P * 4, 256);
    void* sel = nullptr;
    GOAC_TRY(workspace(ctx, 2, bE + bC, &sel));
    double* E = (double*)sel;
    int32_t* cnt = (int32_t*)((char*)sel + bE);
    GOAC_TRY(energies_fp64(pb, P, occ, E));
    return rank_select(ctx, P, E, k, cnt, idx, nullptr, Eout);
}

// ------------------------------------------------------------------ GA
namespace goac {

// one generation queued on the context's stream; a roulette-weight failure is
// or-ed into *err_out (cleared first when zero_err), which the caller reads, or,
// with check_first, reported (after a wait for the weights alone) before any
// child is formed
goac_status ga_generation_enqueue(goac_problem* pb, int64_t P, const uint8_t* pop_in, const double* E_in,
                                  const goac_ga_params* prm, uint8_t* pop_out, bool zero_err, int32_t** err_out,
                                  const uint32_t* g_dev, bool check_first) {
    goac_ctx* ctx = pb->ctx;
    if (P <= 0 || !pop_in || !E_in || !prm || !pop_out || pop_in == pop_out || !(prm->p_mut >= 0.0))
        return fail(ctx, GOAC_EINVAL, "ga_generation: bad arguments");
    if (P > (int64_t)1 << 30) return fail(ctx, GOAC_EINVAL, "ga_generation: population too large");
    if (ga_child_lds(pb) > 160 * 1024) return fail(ctx, GOAC_EINVAL, "ga_generation: too many mobile positions");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    const int32_t ne = (int32_t)std::min<int64_t>(std::max(prm->n_elite, 0), P);
    void* ws = nullptr;
    const size_t b_cum = round_up(P * 8, 256), b_el = round_up((ne + 1) * 4, 256);
    const size_t b_cnt = round_up(P * 4, 256);
    GOAC_TRY(workspace(ctx, 2, b_cum + b_el + b_cnt + 256, &ws));
    uint64_t* cum = (uint64_t*)ws;
    int32_t* elite = (int32_t*)((char*)ws + b_cum);
    int32_t* cnt = (int32_t*)((char*)ws + b_cum + b_el);
    int32_t* err = (int32_t*)((char*)ws + b_cum + b_el + b_cnt);
    if (zero_err) hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, err, 1);
    hipLaunchKernelGGL(k_ga_prep, dim3(1), dim3(1024), 0, ctx->stream, P, E_in, cum, err);
    GOAC_CHECK_LAUNCH(ctx);
    if (check_first) GOAC_TRY(ga_check_err(ctx, err));
    GOAC_TRY(rank_select(ctx, P, E_in, ne, cnt, nullptr, elite, nullptr));
    GOAC_TRY(ga_children(pb, P, pop_in, cum, elite, ne, prm, pop_out, g_dev));
    *err_out = err;
    return GOAC_OK;
}

goac_status ga_check_err(goac_ctx* ctx, const int32_t* err) {
    int32_t herr = 0;
    GOAC_HIP(ctx, hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, ctx->stream));
    GOAC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (herr) return fail(ctx, GOAC_EINVAL, "ga_generation: energy spread too large for the roulette weights");
    return GOAC_OK;
}

}  // namespace goac

extern "C" goac_status goac_ga_generation(goac_problem* pb, int64_t P, const uint8_t* pop_in, const double* E_in,
                                          const goac_ga_params* prm, uint8_t* pop_out) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (P <= 0 || !pop_in) return fail(ctx, GOAC_EINVAL, "ga_generation: bad arguments");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    GOAC_TRY(rows_check(pb, P, pop_in, "ga_generation"));
    int32_t* err = nullptr;
    return ga_generation_enqueue(pb, P, pop_in, E_in, prm, pop_out, true, &err, nullptr, true);
}

namespace {
__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }
__global__ void k_add_u32(uint32_t* p, uint32_t v) { *p += v; }
}  // namespace

// Many generations, each followed by the children's energies. The first runs on
// the stream (it sizes the workspaces); then kGaGraphGens generations at a time
// are captured once as a graph and replayed, the generation index read from a
// device counter that the graph's last node advances; the rest run on the stream.
// The roulette flag of all generations is read once at the end.
constexpr int32_t kGaGraphGens = 8;   // even, so each replay starts on the same buffer

extern "C" goac_status goac_ga_run(goac_problem* pb, int64_t P, uint8_t* pop, double* E, const goac_ga_params* prm,
                                   int32_t generations, int32_t precision) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (!prm || !pop || !E || P <= 0 || generations < 0 || (precision != GOAC_FP64 && precision != GOAC_MIXED))
        return fail(ctx, GOAC_EINVAL, "ga_run: bad arguments");
    if (generations == 0) return GOAC_OK;
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    // the caller's population is checked once; its children keep the composition
    GOAC_TRY(rows_check(pb, P, pop, "ga_run"));
    hipStream_t sm = ctx->stream;
    if (!ctx->cap) GOAC_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    // the second population and the generation counter
    const size_t b_pop = round_up(P * pb->d.n, 256);
    size_t bytes = b_pop + 256;
    void* buf = nullptr;
    GOAC_TRY(pool_get(ctx, &bytes, &buf));
    uint8_t* bufs[2] = {pop, (uint8_t*)buf};
    uint32_t* g_dev = (uint32_t*)((char*)buf + b_pop);
    int32_t* err = nullptr;
    const goac_precision pr = (goac_precision)precision;
    // generation k reads bufs[k & 1] and writes bufs[(k + 1) & 1]
    auto gen = [&](int32_t k, const uint32_t* gd, uint32_t g) -> goac_status {
        goac_ga_params gp = *prm;
        gp.generation = g;
        GOAC_TRY(ga_generation_enqueue(pb, P, bufs[k & 1], E, &gp, bufs[(k + 1) & 1], k == 0, &err, gd));
        return energies_enqueue(pb, P, bufs[(k + 1) & 1], pr, E);
    };
    goac_status st = gen(0, nullptr, prm->generation);
    int32_t k = 1;
    hipError_t ec = hipSuccess;
    // the graph lives until the stream has finished its launches
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (st == GOAC_OK && generations - 1 >= 2 * kGaGraphGens) {
        hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, sm, g_dev, prm->generation + 1u);
        ctx->stream = ctx->cap;
        ctx->capturing = true;
        ec = hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal);
        if (ec == hipSuccess) {
            for (int32_t q = 0; q < kGaGraphGens && st == GOAC_OK; ++q) st = gen(k + q, g_dev, (uint32_t)q);
            if (st == GOAC_OK) hipLaunchKernelGGL(k_add_u32, dim3(1), dim3(1), 0, ctx->cap, g_dev, (uint32_t)kGaGraphGens);
            const hipError_t ee = hipStreamEndCapture(ctx->cap, &graph);
            if (ec == hipSuccess) ec = ee;
        }
        ctx->stream = sm;
        ctx->capturing = false;
        if (st == GOAC_OK && ec == hipSuccess) ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        for (; st == GOAC_OK && ec == hipSuccess && k + kGaGraphGens <= generations; k += kGaGraphGens)
            ec = hipGraphLaunch(exec, sm);
    }
    for (; st == GOAC_OK && ec == hipSuccess && k < generations; ++k) st = gen(k, nullptr, prm->generation + (uint32_t)k);
    if (st == GOAC_OK && ec == hipSuccess && (generations & 1))
        ec = hipMemcpyAsync(pop, bufs[1], (size_t)(P * pb->d.n), hipMemcpyDeviceToDevice, sm);
    if (st == GOAC_OK && ec == hipSuccess) st = ga_check_err(ctx, err);   // synchronises
    if (exec) {
        (void)hipStreamSynchronize(sm);   // also after an error: no launch of it may be pending
        (void)hipGraphExecDestroy(exec);
    }
    if (graph) (void)hipGraphDestroy(graph);
    pool_put(ctx, buf, bytes);
    if (st != GOAC_OK) return st;
    if (ec != hipSuccess) return fail(ctx, GOAC_EHIP, std::string("ga_run: graph: ") + hipGetErrorString(ec));
    return GOAC_OK;
}

// ------------------------------------------------------------------ chains
static goac_status chains_fill(goac_chains* ch, const uint8_t* occ, bool reload);

static goac_status chains_build(goac_chains* ch, const uint8_t* occ) {
    goac_ctx* ctx = ch->ctx;
    const int n_inst = (int)ch->pbs.size();
    const bool mixed = ch->prec == GOAC_MIXED;
    const int64_t C = ch->C;
    // per-chain offsets
    ch->offs.resize(C);
    int64_t tot = 0;
    for (int64_t c = 0; c < C; ++c) {
        ch->offs[c] = tot;
        tot += ch->pbs[ch->inst_of[c]]->d.Mp;
    }
    ch->total = tot;
    // one arena: the uploaded tables first (one copy), then the device-only state
    // (the chain scalars are set by the setup kernel; one instance needs no order)
    ArenaPlan ap;
    const size_t o_in = ap.take(n_inst * sizeof(McInst));
    const size_t o_of = ap.take(C * sizeof(int64_t));
    const size_t o_or = ap.take(n_inst > 1 ? C * sizeof(int32_t) : 0);
    const size_t up_end = ap.end;
    const size_t o_q = ap.take(64 * sizeof(int32_t));
    const size_t o_sc = ap.take(C * sizeof(ChainScalars));
    const size_t o_occ = ap.take(tot);
    const size_t o_perm = ap.take(tot * sizeof(uint16_t));
    const size_t o_best = ap.take(tot);
    const size_t o_phi = ap.take(tot * (mixed ? 4 : 8));
    ch->arena_bytes = ap.end;
    GOAC_TRY(pool_get(ctx, &ch->arena_bytes, &ch->arena));
    char* base = (char*)ch->arena;
    ch->sc = (ChainScalars*)(base + o_sc);
    ch->insts = (McInst*)(base + o_in);
    ch->d_offs = (int64_t*)(base + o_of);
    ch->order = n_inst > 1 ? (int32_t*)(base + o_or) : nullptr;
    ch->queue = (int32_t*)(base + o_q);
    ch->occ = (uint8_t*)(base + o_occ);
    ch->perm = (uint16_t*)(base + o_perm);
    ch->best = (uint8_t*)(base + o_best);
    ch->phi = base + o_phi;
    std::vector<char> host(up_end, 0);
    McInst* insts = (McInst*)(host.data() + o_in);
    for (int i = 0; i < n_inst; ++i) {
        const ProblemDev& d = ch->pbs[i]->d;
        McInst& I = insts[i];
        I.V64 = d.V64; I.V32 = d.V32; I.diag = d.diag; I.rowmax = d.rowmax; I.h = d.h; I.phibar = d.phibar;
        I.msub = d.msub; I.tab = d.tab; I.charge = d.charge; I.Ed = d.Ed;
        I.M = d.M; I.Mp = d.Mp; I.S = d.S; I.E = d.E;
        I.instance = ch->inst_id[i];
        I.pad_ = 0;
        ch->max_Mp = std::max(ch->max_Mp, d.Mp);
        ch->max_S = std::max(ch->max_S, d.S);
        ch->max_E = std::max(ch->max_E, d.E);
        ch->max_tab = std::max(ch->max_tab, tab_words(d.S, d.E));
    }
    std::memcpy(host.data() + o_of, ch->offs.data(), C * 8);
    if (n_inst > 1) {
        // longest chains first (Mp as the cost), stable
        int32_t* order = (int32_t*)(host.data() + o_or);
        std::iota(order, order + C, 0);
        std::stable_sort(order, order + C, [&](int32_t a, int32_t b) {
            return ch->pbs[ch->inst_of[a]]->d.Mp > ch->pbs[ch->inst_of[b]]->d.Mp;
        });
    }
    GOAC_TRY(upload(ctx, base, host.data(), up_end));
    return chains_fill(ch, occ, false);
}

// composition check, setup (mobile occupation, position lists, best copy) and
// FP64 field of every chain from occupations occ (instance after instance); a
// reload keeps counters, rows and the best unless beaten. Synchronises to report
// a broken composition.
static goac_status chains_fill(goac_chains* ch, const uint8_t* occ, bool reload) {
    goac_ctx* ctx = ch->ctx;
    const int n_inst = (int)ch->pbs.size();
    hipStream_t sm = ctx->stream;
    const bool mixed = ch->prec == GOAC_MIXED;
    void* sel = nullptr;
    GOAC_TRY(workspace(ctx, 2, 256, &sel));
    int32_t* err = (int32_t*)sel;
    // the composition check first: the host waits for nothing queued after it, and
    // the chains are left untouched when an occupation breaks the composition
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, sm, err, 1);
    for (int i = 0; i < n_inst; ++i) {
        const ProblemDev& d = ch->pbs[i]->d;
        const int64_t Ci = ch->count[i];
        if (Ci == 0) continue;
        hipLaunchKernelGGL(k_check_comp, dim3((unsigned)Ci), dim3(256), 0, sm, d.n, d.S, d.E, d.tab, d.site_sub,
                           occ + ch->occ_row_off[i], err);
    }
    GOAC_CHECK_LAUNCH(ctx);
    int32_t herr = 0;
    GOAC_HIP(ctx, hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, sm));
    GOAC_HIP(ctx, hipStreamSynchronize(sm));
    if (herr) return fail(ctx, GOAC_EINVAL, "chains: an occupation breaks the problem's composition");
    for (int i = 0; i < n_inst; ++i) {
        goac_problem* pb = ch->pbs[i];
        const ProblemDev& d = pb->d;
        const int64_t Ci = ch->count[i];
        if (Ci == 0) continue;
        const uint8_t* occ_i = occ + ch->occ_row_off[i];
        hipLaunchKernelGGL(k_chain_setup, dim3((unsigned)Ci), dim3(64), 0, sm, d.n, d.M, d.Mp, d.S, d.E, d.tab, d.mob,
                           d.msub, occ_i, ch->first_chain[i], ch->d_offs, ch->occ, ch->perm,
                           reload ? nullptr : ch->best, reload ? nullptr : ch->sc, i,
                           ch->chain_id[ch->first_chain[i]]);
        const size_t qb = (size_t)round_up((int64_t)Ci * d.Mp * 8, 256);
        void* ws = nullptr;
        GOAC_TRY(workspace(ctx, 0, 2 * qb, &ws));
        double* Q = (double*)ws;
        double* Phi = (double*)((char*)ws + qb);
        GOAC_TRY(build_q64(ctx, Ci, d.n, d.M, d.Mp, d.E, occ_i, d.mob, d.charge, Q));
        GOAC_TRY(dgemm_nt(ctx, Ci, d.M, d.Mp, Q, d.Mp, d.V64, d.Mp, Phi, d.Mp, 1.0, 0.0, nullptr));
        if (mixed)
            hipLaunchKernelGGL(k_chain_field<true>, dim3((unsigned)Ci), dim3(256), 0, sm, d.M, d.Mp, Q, Phi, d.h,
                               d.rowabs, d.qmax, d.msub, d.phibar, d.Ed, ch->first_chain[i], ch->sc, ch->phi,
                               reload ? 1 : 0, ch->occ, ch->best);
        else
            hipLaunchKernelGGL(k_chain_field<false>, dim3((unsigned)Ci), dim3(256), 0, sm, d.M, d.Mp, Q, Phi, d.h,
                               d.rowabs, d.qmax, d.msub, d.phibar, d.Ed, ch->first_chain[i], ch->sc, ch->phi,
                               reload ? 1 : 0, ch->occ, ch->best);
        GOAC_CHECK_LAUNCH(ctx);
    }
    return GOAC_OK;
}

static void chains_free(goac_chains* ch) {
    for (hipEvent_t e : ch->tev) (void)hipEventDestroy(e);
    ch->tev.clear();
    if (ch->arena) pool_put(ch->ctx, ch->arena, ch->arena_bytes);
    ch->arena = nullptr;
    pool_put(ch->ctx, ch->kT, ch->kT_cap * 8);
    pool_put(ch->ctx, ch->scratch, ch->scratch_size);
    pool_put(ch->ctx, ch->ladder, ch->ladder_cap * 8);
    ch->kT = nullptr;
    ch->scratch = nullptr;
    ch->ladder = nullptr;
}

extern "C" goac_status goac_chains_load(goac_chains* ch, const uint8_t* occ_dev) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    if (!occ_dev) return fail(ctx, GOAC_EINVAL, "chains_load: bad arguments");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    return chains_fill(ch, occ_dev, true);
}

extern "C" goac_status goac_chains_create(goac_problem* pb, int64_t C, const uint8_t* occ, goac_precision prec,
                                          uint32_t chain_base, uint32_t instance, goac_chains** out) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (!out || C <= 0 || !occ || C > (1 << 30)) return fail(ctx, GOAC_EINVAL, "chains_create: bad arguments");
    if (prec != GOAC_FP64 && prec != GOAC_MIXED) return fail(ctx, GOAC_EINVAL, "chains_create: unknown precision");
    if (instance >= (1u << 24)) return fail(ctx, GOAC_EINVAL, "chains_create: instance id >= 2^24");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    goac_chains* ch = new goac_chains();
    ch->ctx = ctx;
    ch->prec = prec;
    ch->C = C;
    ch->pbs = {pb};
    ch->inst_id = {instance};
    ch->count = {C};
    ch->first_chain = {0};
    ch->occ_row_off = {0};
    ch->inst_of.assign(C, 0);
    ch->chain_id.resize(C);
    for (int64_t c = 0; c < C; ++c) ch->chain_id[c] = chain_base + (uint32_t)c;
    goac_status st = chains_build(ch, occ);
    if (st != GOAC_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        chains_free(ch);
        delete ch;
        return st;
    }
    ctx->holders.attach();
    *out = ch;
    return GOAC_OK;
}

extern "C" goac_status goac_chains_create_batch(goac_problem* const* pbs, int32_t n_inst, const int64_t* cpi,
                                                const uint8_t* occ, goac_precision prec, goac_chains** out) {
    if (!pbs || n_inst <= 0 || !pbs[0]) return GOAC_EINVAL;
    goac_ctx* ctx = pbs[0]->ctx;
    if (!out || !cpi || !occ) return fail(ctx, GOAC_EINVAL, "chains_create_batch: bad arguments");
    if (prec != GOAC_FP64 && prec != GOAC_MIXED) return fail(ctx, GOAC_EINVAL, "chains_create_batch: precision");
    goac_chains* ch = new goac_chains();
    ch->ctx = ctx;
    ch->prec = prec;
    int64_t C = 0, rowoff = 0;
    for (int i = 0; i < n_inst; ++i) {
        if (!pbs[i] || cpi[i] < 0) {
            delete ch;
            return fail(ctx, GOAC_EINVAL, "chains_create_batch: bad instance");
        }
        if (pbs[i]->ctx != ctx) {
            delete ch;
            return fail(ctx, GOAC_ESTATE, "chains_create_batch: problems of different contexts");
        }
        ch->pbs.push_back(pbs[i]);
        ch->inst_id.push_back((uint32_t)i);
        ch->count.push_back(cpi[i]);
        ch->first_chain.push_back(C);
        ch->occ_row_off.push_back(rowoff);
        for (int64_t c = 0; c < cpi[i]; ++c) {
            ch->inst_of.push_back(i);
            ch->chain_id.push_back((uint32_t)c);
        }
        C += cpi[i];
        rowoff += cpi[i] * pbs[i]->d.n;
    }
    if (C <= 0 || C > (1 << 30)) {
        delete ch;
        return fail(ctx, GOAC_EINVAL, "chains_create_batch: no chains");
    }
    ch->C = C;
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    goac_status st = chains_build(ch, occ);
    if (st != GOAC_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        chains_free(ch);
        delete ch;
        return st;
    }
    ctx->holders.attach();
    *out = ch;
    return GOAC_OK;
}

extern "C" void goac_chains_destroy(goac_chains* ch) {
    if (!ch) return;
    destroy_dependent(ch->ctx, ch, chains_free, ctx_free);
}

extern "C" goac_status goac_chains_set_rows(goac_chains* ch, const int32_t* rows) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    if (!rows) return fail(ctx, GOAC_EINVAL, "chains_set_rows: null rows");
    for (int64_t c = 0; c < ch->C; ++c)
        if (rows[c] < 0) return fail(ctx, GOAC_EINVAL, "chains_set_rows: negative row");
    void* ws = nullptr;
    GOAC_TRY(workspace(ctx, 0, (size_t)ch->C * 4, &ws));
    int32_t* d = (int32_t*)ws;
    GOAC_TRY(upload(ctx, d, rows, ch->C * 4));
    hipLaunchKernelGGL(k_set_rows, dim3((unsigned)((ch->C + 255) / 256)), dim3(256), 0, ctx->stream, ch->C, d, ch->sc);
    GOAC_CHECK_LAUNCH(ctx);
    ch->max_row = 0;
    for (int64_t c = 0; c < ch->C; ++c) ch->max_row = std::max(ch->max_row, rows[c]);
    return GOAC_OK;
}

// ------------------------------------------------------------------ sweep planning
// The launch configuration of a sweep: threads per chain (wg), chains resident per
// compute unit (per_cu, bounded by the LDS a chain needs) and the grid.
struct SweepPlan {
    int wg = 64;
    int per_cu = 1;
    int grid = 1;
    size_t lds = 0;
    McArgs a{};
};

static goac_status sweep_plan(goac_chains* ch, const goac_mc_params* prm, int wg_req, int per_cu_req,
                              SweepPlan* out) {
    goac_ctx* ctx = ch->ctx;
    const bool mixed = ch->prec == GOAC_MIXED;
    int wg = wg_req == 64 || wg_req == 256 ? wg_req : (ch->max_Mp >= 2048 ? 256 : 64);
    // one-wave chains gather V_mm entries through 32-bit byte offsets
    if ((uint64_t)ch->max_Mp * (uint64_t)ch->max_Mp * 8u >= ((uint64_t)1 << 32)) wg = 256;
    const size_t phi_bytes = (size_t)round_up(ch->max_Mp * (mixed ? 4 : 8), 16);
    // occupation, site class (only with several classes), perm and where per
    // position; one-wave chains add the FP64 diagonal, multi-wave chains the log
    // of swaps since the last best-occupation copy
    const bool msub_lds = ch->max_S > 1;
    const size_t lds_base = phi_bytes + (size_t)ch->max_Mp * (1 + (msub_lds ? 1 : 0) + 2 + 2) +
                            round_up(ch->max_tab * 4, 16) + kMaxSpecies * 8;
    if (wg == 64 && lds_base + (size_t)ch->max_Mp * 8 > 160 * 1024) wg = 256;   // no room for it
    const size_t lds = lds_base + (wg == 64 ? (size_t)ch->max_Mp * 8 : (size_t)kBestLog * 4);
    if (lds > 160 * 1024) return fail(ctx, GOAC_EINVAL, "mc_sweep: the chain state does not fit in LDS");
    const int cap = std::max<int>(1, std::min<int>(wg == 64 ? 16 : 4, (int)((160 * 1024) / lds)));
    const int per_cu = per_cu_req > 0 ? std::min(per_cu_req, cap) : cap;
    SweepPlan& P = *out;
    P.wg = wg;
    P.per_cu = per_cu;
    P.lds = lds;
    P.grid = (int)std::min<int64_t>(ch->C, (int64_t)ctx->num_cus * per_cu);
    McArgs& a = P.a;
    a.insts = ch->insts;
    a.sc = ch->sc;
    a.phi = ch->phi;
    a.occ = ch->occ;
    a.perm = ch->perm;
    a.best = ch->best;
    a.order = ch->order;
    a.queue = ch->queue;
    a.n_items = (int32_t)ch->C;
    a.n_blocks = prm->n_blocks;
    a.kT = ch->kT;
    a.block_len = prm->block_len;
    a.n_trials = prm->n_trials;
    a.seed = prm->seed;
    a.reanchor_every = prm->reanchor_every;
    a.lds_phi_bytes = (int32_t)phi_bytes;
    a.Mp_max = ch->max_Mp;
    a.tab_max = (int32_t)round_up(ch->max_tab, 4);
    // MIXED: small cells re-anchor inside the kernel; large cells run in chunks of
    // 8 x reanchor_every trials with a batched FP64 anchor of the due chains after each
    a.inline_anchor = (mixed && ch->max_Mp > kInlineAnchorMaxMp) ? 0 : 1;
    a.msub_lds = msub_lds ? 1 : 0;
    return GOAC_OK;
}

// device kT table of a sweep (rows x blocks), copied from the host unless it equals
// the table uploaded last (a copy from pageable host memory waits for the stream)
static goac_status sweep_upload_kT(goac_chains* ch, const double* kT_host, size_t nkT) {
    goac_ctx* ctx = ch->ctx;
    if (ch->kT && ch->kT_last.size() == nkT && std::equal(ch->kT_last.begin(), ch->kT_last.end(), kT_host))
        return GOAC_OK;
    ch->kT_last.assign(kT_host, kT_host + nkT);
    if (nkT > ch->kT_cap) {
        pool_put(ctx, ch->kT, ch->kT_cap * 8);
        ch->kT = nullptr;
        ch->kT_cap = 0;
        size_t bytes = nkT * 8;
        void* p = nullptr;
        GOAC_TRY(pool_get(ctx, &bytes, &p));
        ch->kT = (double*)p;
        ch->kT_cap = bytes / 8;
    }
    GOAC_TRY(upload(ctx, ch->kT, kT_host, nkT * 8));
    return GOAC_OK;
}

// the launches of a sweep: kernels only (no host copies), so a stream capture may
// record them. The persistent grid pulls chains from a counter reset before each
// launch.
// zero_queue false: the caller has cleared the work counter (one launch only)
// a timing mark: records the next event of a pair (GOAC_MC_TIMING)
static goac_status timing_mark(goac_chains* ch, uint8_t kind) {
    goac_ctx* ctx = ch->ctx;
    if (ch->tev_used == ch->tev.size()) {
        hipEvent_t e = nullptr;
        GOAC_HIP(ctx, hipEventCreate(&e));
        ch->tev.push_back(e);
        ch->tev_kind.push_back(kind);
    }
    ch->tev_kind[ch->tev_used] = kind;
    GOAC_HIP(ctx, hipEventRecord(ch->tev[ch->tev_used++], ctx->stream));
    return GOAC_OK;
}

static goac_status sweep_enqueue(goac_chains* ch, SweepPlan P, bool trace, uint64_t n_trials,
                                 int32_t reanchor_every, bool zero_queue = true, bool timing = false) {
    goac_ctx* ctx = ch->ctx;
    const bool mixed = ch->prec == GOAC_MIXED;
    P.a.kT = ch->kT;
    if (P.a.inline_anchor) {
        P.a.n_trials = n_trials;
        if (zero_queue) hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, ch->queue, 1);
        if (timing) GOAC_TRY(timing_mark(ch, 0));
        GOAC_TRY(mc_launch(ctx, P.a, mixed, trace, P.wg, P.lds, P.grid));
        if (timing) GOAC_TRY(timing_mark(ch, 0));
        return GOAC_OK;
    }
    const uint64_t chunk = (uint64_t)reanchor_every * 8;
    for (uint64_t done = 0; done < n_trials; done += chunk) {
        P.a.n_trials = std::min<uint64_t>(chunk, n_trials - done);
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, ch->queue, 1);
        if (timing) GOAC_TRY(timing_mark(ch, 0));
        GOAC_TRY(mc_launch(ctx, P.a, mixed, trace, P.wg, P.lds, P.grid));
        if (timing) GOAC_TRY(timing_mark(ch, 0));
        if (timing) GOAC_TRY(timing_mark(ch, 1));
        for (size_t i = 0; i < ch->pbs.size(); ++i)
            GOAC_TRY(anchor_batched(ctx, ch, (int)i, (uint32_t)reanchor_every));
        if (timing) GOAC_TRY(timing_mark(ch, 1));
    }
    return GOAC_OK;
}

static goac_status sweep_check(goac_chains* ch, const goac_mc_params* prm) {
    goac_ctx* ctx = ch->ctx;
    if (!prm || !prm->kT_host || prm->n_rows <= 0 || prm->n_blocks <= 0 || prm->block_len == 0)
        return fail(ctx, GOAC_EINVAL, "mc_sweep: bad parameters");
    if (prm->n_rows <= ch->max_row) return fail(ctx, GOAC_EINVAL, "mc_sweep: a chain's temperature row is beyond n_rows");
    const size_t nkT = (size_t)prm->n_rows * prm->n_blocks;
    for (size_t x = 0; x < nkT; ++x)
        if (!(prm->kT_host[x] > 0.0)) return fail(ctx, GOAC_EINVAL, "mc_sweep: kT must be positive");
    if (ch->prec == GOAC_MIXED && prm->reanchor_every <= 0)
        return fail(ctx, GOAC_EINVAL, "mc_sweep: reanchor_every must be positive");
    if (prm->variant != 0 && prm->variant != 64 && prm->variant != 256)
        return fail(ctx, GOAC_EINVAL, "mc_sweep: variant must be 0, 64 or 256");
    return GOAC_OK;
}

extern "C" goac_status goac_mc_sweep(goac_chains* ch, const goac_mc_params* prm) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    GOAC_TRY(sweep_check(ch, prm));
    if (prm->n_trials == 0) return GOAC_OK;
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    GOAC_TRY(sweep_upload_kT(ch, prm->kT_host, (size_t)prm->n_rows * prm->n_blocks));
    SweepPlan P;
    // an explicit variant wins; otherwise the tuned configuration, else the size rule
    const int wg = prm->variant != 0 ? prm->variant : ch->tuned_wg;
    const int per_cu = prm->variant != 0 ? 0 : ch->tuned_per_cu;
    GOAC_TRY(sweep_plan(ch, prm, wg, per_cu, &P));
    return sweep_enqueue(ch, P, (prm->flags & GOAC_MC_TRACE_HASH) != 0, prm->n_trials, prm->reanchor_every, true,
                         (prm->flags & GOAC_MC_TIMING) != 0);
}

extern "C" goac_status goac_chains_timing(goac_chains* ch, double* mc_seconds, double* anchor_seconds,
                                          int64_t* mc_launches) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    double t[2] = {0.0, 0.0};
    int64_t launches = 0;
    if (ch->tev_used > 0) GOAC_HIP(ctx, hipEventSynchronize(ch->tev[ch->tev_used - 1]));
    for (size_t e = 0; e + 1 < ch->tev_used; e += 2) {
        float ms = 0.0f;
        GOAC_HIP(ctx, hipEventElapsedTime(&ms, ch->tev[e], ch->tev[e + 1]));
        t[ch->tev_kind[e]] += 1e-3 * (double)ms;
        if (ch->tev_kind[e] == 0) ++launches;
    }
    ch->tev_used = 0;
    if (mc_seconds) *mc_seconds = t[0];
    if (anchor_seconds) *anchor_seconds = t[1];
    if (mc_launches) *mc_launches = launches;
    return GOAC_OK;
}

// ------------------------------------------------------------------ autotuning
// Times short probe sweeps of each launch configuration on the chains themselves
// and keeps the fastest for later sweeps that request no variant. The chain state
// (scalars, field, occupations, position lists, best copies) is saved before and
// restored after every probe, so the chains are left exactly as they were.
extern "C" goac_status goac_chains_autotune(goac_chains* ch, uint64_t probe_trials, double kT, int32_t* wg_out,
                                            int32_t* per_cu_out) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    if (probe_trials == 0 || !(kT > 0.0)) return fail(ctx, GOAC_EINVAL, "chains_autotune: bad arguments");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = ctx->stream;
    const bool mixed = ch->prec == GOAC_MIXED;
    const size_t b_sc = ch->C * sizeof(ChainScalars), b_phi = ch->total * (mixed ? 4 : 8);
    const size_t b_occ = ch->total, b_perm = ch->total * 2, b_best = ch->total;
    const size_t parts[5] = {b_sc, b_phi, b_occ, b_perm, b_best};
    void* const srcs[5] = {ch->sc, ch->phi, ch->occ, ch->perm, ch->best};
    size_t offs[5], tot = 0;
    for (int q = 0; q < 5; ++q) { offs[q] = tot; tot += round_up(parts[q], 256); }
    char* save = nullptr;
    GOAC_HIP(ctx, hipMalloc((void**)&save, tot));
    auto copy_all = [&](bool to_save) -> goac_status {
        for (int q = 0; q < 5; ++q) {
            char* s = to_save ? (char*)srcs[q] : save + offs[q];
            char* d = to_save ? save + offs[q] : (char*)srcs[q];
            GOAC_HIP(ctx, hipMemcpyAsync(d, s, parts[q], hipMemcpyDeviceToDevice, sm));
        }
        return GOAC_OK;
    };
    goac_status st = copy_all(true);
    std::vector<double> table((size_t)ch->max_row + 1, kT);
    goac_mc_params prm{};
    prm.seed = 0x5eed;
    prm.n_trials = probe_trials;
    prm.kT_host = table.data();
    prm.n_rows = (int32_t)table.size();
    prm.n_blocks = 1;
    prm.block_len = probe_trials;
    prm.reanchor_every = 1024;
    if (st == GOAC_OK) st = sweep_upload_kT(ch, table.data(), table.size());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == GOAC_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(ctx, GOAC_EHIP, "chains_autotune: event creation failed");
    float best_ms = INFINITY;
    int best_wg = 0, best_pc = 0;
    for (int wg : {64, 256}) {
        if (st != GOAC_OK) break;
        SweepPlan P0;
        if ((st = sweep_plan(ch, &prm, wg, 0, &P0)) != GOAC_OK) break;
        const int cap = P0.per_cu;
        std::vector<int> cands = {cap};
        if (cap / 2 >= 1) cands.push_back(cap / 2);
        for (int pc : cands) {
            SweepPlan P;
            if ((st = sweep_plan(ch, &prm, wg, pc, &P)) != GOAC_OK) break;
            float ms = 0.0f;
            for (int rep = 0; rep < 2 && st == GOAC_OK; ++rep) {   // the first run warms the caches
                if ((st = copy_all(false)) != GOAC_OK) break;
                if (hipEventRecord(e0, sm) != hipSuccess) { st = fail(ctx, GOAC_EHIP, "event"); break; }
                if ((st = sweep_enqueue(ch, P, false, probe_trials, prm.reanchor_every)) != GOAC_OK) break;
                if (hipEventRecord(e1, sm) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                    st = fail(ctx, GOAC_EHIP, "chains_autotune: timing failed");
            }
            if (st == GOAC_OK && ms < best_ms) { best_ms = ms; best_wg = wg; best_pc = pc; }
        }
    }
    if (st == GOAC_OK) st = copy_all(false);
    (void)hipStreamSynchronize(sm);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(save);
    if (st != GOAC_OK) return st;
    ch->tuned_wg = best_wg;
    ch->tuned_per_cu = best_pc;
    if (wg_out) *wg_out = best_wg;
    if (per_cu_out) *per_cu_out = best_pc;
    return GOAC_OK;
}

namespace goac {
goac_status chains_export_enqueue(goac_chains* ch, uint8_t* occ, uint8_t* best, goac_chain_stats* stats) {
    goac_ctx* ctx = ch->ctx;
    for (size_t i = 0; i < ch->pbs.size(); ++i) {
        goac_problem* pb = ch->pbs[i];
        const ProblemDev& d = pb->d;
        const int64_t Ci = ch->count[i];
        if (Ci == 0) continue;
        // rows of instance i start at occ_row_off; k_export indexes rows by global chain
        // id, so shift the base pointers to make row g land at occ_row_off + (g - first) n
        const int64_t first = ch->first_chain[i];
        uint8_t* o = occ ? occ + ch->occ_row_off[i] - first * d.n : nullptr;
        uint8_t* b = best ? best + ch->occ_row_off[i] - first * d.n : nullptr;
        hipLaunchKernelGGL(k_export, dim3((unsigned)Ci), dim3(256), 0, ctx->stream, d.n, d.M, d.mob, pb->fixed_idx,
                           pb->n_fixed, d.ref_occ, first, ch->sc, ch->occ, ch->best, o, b, stats);
        GOAC_CHECK_LAUNCH(ctx);
    }
    return GOAC_OK;
}
}  // namespace goac

// The copies, then the chains' drift flags; the host waits for the flags (and so
// for the copies, which precede them on the stream).
extern "C" goac_status goac_chains_export(goac_chains* ch, uint8_t* occ, uint8_t* best, goac_chain_stats* stats) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    if (ctx->capturing) return fail(ctx, GOAC_EINVAL, "chains_export inside a stream capture");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    GOAC_TRY(chains_export_enqueue(ch, occ, best, stats));
    GOAC_TRY(check_buffers(ctx));
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, ctx->chk_dev, 1);
    hipLaunchKernelGGL(k_drift_flag, dim3((unsigned)((ch->C + 255) / 256)), dim3(256), 0, ctx->stream, ch->C, ch->sc,
                       ctx->chk_dev);
    GOAC_CHECK_LAUNCH(ctx);
    GOAC_TRY(check_publish(ctx));
    GOAC_HIP(ctx, hipEventSynchronize(ctx->chk_ev));
    if (*ctx->chk_host)
        return fail(ctx, GOAC_EDRIFT, "chains_export: a chain's FP32 field left its error bound");
    return GOAC_OK;
}

// replicas per group: the permutation check keeps one LDS bit per slot value
constexpr int32_t kRemcMaxR = 1 << 19;
// rounds per captured graph of goac_remc_run
constexpr uint64_t kRemcGraphRounds = 8;

static void remc_launch(hipStream_t s, int64_t ng, int32_t R, const double* kT, uint64_t x, uint64_t* x_dev,
                        uint64_t seed, ChainScalars* sc, int32_t* slot, uint8_t* acc, uint32_t* ticket,
                        int32_t* queue) {
    const size_t lds = (size_t)((R + 31) / 32) * 4;
    hipLaunchKernelGGL(k_remc, dim3((unsigned)ng), dim3(R <= 128 ? 64 : 256), lds, s, R, kT, x, x_dev, seed, sc,
                       slot, acc, ticket, queue);
}

extern "C" goac_status goac_remc_exchange(goac_chains* ch, int32_t R, const double* kT_host, uint64_t x,
                                          uint64_t seed, int32_t* slot, uint8_t* acc) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    if (R < 2 || R > kRemcMaxR || !kT_host || !slot || ch->C % R != 0)
        return fail(ctx, GOAC_EINVAL, "remc_exchange: R must be in [2, 2^19] and divide the chain count");
    for (int k = 0; k < R; ++k)
        if (!(kT_host[k] > 0.0)) return fail(ctx, GOAC_EINVAL, "remc_exchange: kT must be positive");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    // the ladder lives with the chains; copied only when it changed
    if (!ch->ladder || ch->ladder_last.size() != (size_t)R ||
        !std::equal(ch->ladder_last.begin(), ch->ladder_last.end(), kT_host)) {
        if ((size_t)R > ch->ladder_cap) {
            pool_put(ctx, ch->ladder, ch->ladder_cap * 8);
            ch->ladder = nullptr;
            ch->ladder_cap = 0;
            size_t bytes = (size_t)R * 8;
            void* p = nullptr;
            GOAC_TRY(pool_get(ctx, &bytes, &p));
            ch->ladder = (double*)p;
            ch->ladder_cap = bytes / 8;
        }
        ch->ladder_last.assign(kT_host, kT_host + R);
        GOAC_TRY(upload(ctx, ch->ladder, kT_host, R * 8));
    }
    const double* d = ch->ladder;
    const int64_t ng = ch->C / R;
    remc_launch(ctx->stream, ng, R, d, x, nullptr, seed, ch->sc, slot, acc, nullptr, nullptr);
    GOAC_CHECK_LAUNCH(ctx);
    ch->max_row = std::max(ch->max_row, R - 1);
    return GOAC_OK;
}


// Many replica-exchange rounds (each a sweep and its exchange step), launched on
// the stream round after round. With GOAC_REMC_GRAPH, up to kRemcGraphRounds
// rounds are captured once as a graph and replayed instead, the step index x0 + r
// read from device memory and advanced by each exchange; the last rounds that do
// not fill a graph launch the same kernels on the stream. Cells whose MIXED field
// re-anchors between sweep chunks (workspace sized on the host) run without
// capture.
extern "C" goac_status goac_remc_run(goac_chains* ch, int32_t R, const double* kT_host, uint64_t trials,
                                     uint64_t rounds, uint64_t x0, uint64_t seed, uint32_t flags,
                                     int32_t reanchor_every, int32_t* slot) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    if (R < 2 || R > kRemcMaxR || !kT_host || !slot || ch->C % R != 0 || trials == 0 ||
        (flags & ~(GOAC_MC_TRACE_HASH | GOAC_REMC_GRAPH)))
        return fail(ctx, GOAC_EINVAL, "remc_run: bad arguments");
    for (int k = 0; k < R; ++k)
        if (!(kT_host[k] > 0.0)) return fail(ctx, GOAC_EINVAL, "remc_run: kT must be positive");
    if (ch->prec == GOAC_MIXED && reanchor_every <= 0) return fail(ctx, GOAC_EINVAL, "remc_run: reanchor_every");
    if (rounds == 0) return GOAC_OK;
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = ctx->stream;
    const int64_t ng = ch->C / R;
    goac_mc_params prm{};
    prm.seed = seed;
    prm.n_trials = trials;
    prm.kT_host = kT_host;
    prm.n_rows = R;
    prm.n_blocks = 1;
    prm.block_len = trials;
    prm.reanchor_every = reanchor_every > 0 ? reanchor_every : 1024;
    prm.flags = flags & GOAC_MC_TRACE_HASH;
    // the ladder is the sweep's table (R rows x 1 block) and the exchange's
    GOAC_TRY(sweep_upload_kT(ch, kT_host, (size_t)R));
    SweepPlan P;
    GOAC_TRY(sweep_plan(ch, &prm, ch->tuned_wg, ch->tuned_per_cu, &P));
    const bool trace = (flags & GOAC_MC_TRACE_HASH) != 0;
    ch->max_row = std::max(ch->max_row, R - 1);
    hipLaunchKernelGGL(k_rows_from_slot, dim3((unsigned)ng), dim3(R <= 128 ? 64 : 256), (size_t)((R + 31) / 32) * 4, sm,
                       ng, R, slot, ch->sc);
    GOAC_CHECK_LAUNCH(ctx);
    if (!P.a.inline_anchor || !(flags & GOAC_REMC_GRAPH)) {
        for (uint64_t r = 0; r < rounds; ++r) {
            GOAC_TRY(sweep_enqueue(ch, P, trace, trials, prm.reanchor_every));
            remc_launch(sm, ng, R, ch->kT, x0 + r, nullptr, seed, ch->sc, slot, nullptr, nullptr, nullptr);
            GOAC_CHECK_LAUNCH(ctx);
        }
        return GOAC_OK;
    }
    void* xs = nullptr;
    GOAC_TRY(workspace(ctx, 2, 256, &xs));
    uint64_t* xdev = (uint64_t*)xs;
    uint32_t* ticket = (uint32_t*)(xdev + 1);
    // the first round's work counter is cleared here, later ones by the exchange
    hipLaunchKernelGGL(k_remc_init, dim3(1), dim3(1), 0, sm, xdev, x0, ticket, ch->queue);
    GOAC_CHECK_LAUNCH(ctx);
    // capture on a private stream (the context's may be the null stream, which
    // cannot be captured); the graph then runs on the context's stream
    if (!ctx->cap) GOAC_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    hipStream_t cap = ctx->cap;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ctx->stream = cap;
    ctx->capturing = true;
    goac_status st = GOAC_OK;
    // a graph holds K rounds: consecutive launches of one graph are separated by a
    // gap of several microseconds, the kernels inside it are not
    const uint64_t K = std::min<uint64_t>(rounds, kRemcGraphRounds);
    hipError_t ec = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (ec == hipSuccess) {
        for (uint64_t q = 0; q < K && st == GOAC_OK; ++q) {
            st = sweep_enqueue(ch, P, trace, trials, prm.reanchor_every, false);
            if (st == GOAC_OK)
                remc_launch(cap, ng, R, ch->kT, 0, xdev, seed, ch->sc, slot, nullptr, ticket, ch->queue);
        }
        ec = hipStreamEndCapture(cap, &graph);
    }
    ctx->stream = sm;
    ctx->capturing = false;
    if (st == GOAC_OK && ec == hipSuccess) ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    uint64_t r = 0;
    for (; st == GOAC_OK && ec == hipSuccess && r + K <= rounds; r += K) ec = hipGraphLaunch(exec, sm);
    // the last rounds % K rounds: the same kernels launched on the stream
    for (; st == GOAC_OK && ec == hipSuccess && r < rounds; ++r) {
        st = sweep_enqueue(ch, P, trace, trials, prm.reanchor_every, false);
        if (st == GOAC_OK) {
            remc_launch(sm, ng, R, ch->kT, 0, xdev, seed, ch->sc, slot, nullptr, ticket, ch->queue);
            ec = hipGetLastError();
        }
    }
    if (st == GOAC_OK && ec == hipSuccess) ec = hipStreamSynchronize(sm);
    if (exec) {
        (void)hipStreamSynchronize(sm);   // also after an error: no launch of it may be pending
        (void)hipGraphExecDestroy(exec);
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (st != GOAC_OK) return st;
    if (ec != hipSuccess) return fail(ctx, GOAC_EHIP, std::string("remc_run: graph: ") + hipGetErrorString(ec));
    return GOAC_OK;
}
