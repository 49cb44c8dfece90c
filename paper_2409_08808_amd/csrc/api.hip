// C ABI entry points of the gfx950 library (declared in include/goac.h): argument
// checks, problem derivation, chain-set management and kernel dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.h"

namespace goac {

goac_status build_ewald(goac_ctx*, const double*, int64_t, const double*, const goac_ewald_params*, double*);
goac_status energies_mixed(goac_problem*, int64_t, const uint8_t*, double*);
goac_status energies_fp64(goac_problem*, int64_t, const uint8_t*, double*);

__global__ void k_init(int64_t, int32_t, int32_t, const int32_t*, const int32_t*, const int32_t*, const int32_t*,
                       int32_t, const uint8_t*, uint64_t, uint32_t, uint32_t, uint8_t*);
__global__ void k_ga_prep(int64_t, const double*, int32_t, uint64_t*, int32_t*, int32_t*);
__global__ void k_ga_child(int64_t, int32_t, int32_t, int32_t, const int32_t*, const int32_t*, const int32_t*,
                           const uint8_t*, const int32_t*, const int32_t*, int32_t, const uint8_t*, int64_t,
                           const uint8_t*, const uint64_t*, const int32_t*, int32_t, uint64_t, uint32_t, double,
                           uint8_t*);
__global__ void k_topk_select(int64_t, int32_t, const double*, int64_t*, double*);

goac_status workspace(goac_ctx* ctx, size_t bytes, void** out) {
    if (bytes > ctx->ws_size) {
        if (ctx->ws) {
            GOAC_HIP(ctx, hipStreamSynchronize(ctx->stream));
            GOAC_HIP(ctx, hipFree(ctx->ws));
            ctx->ws = nullptr;
            ctx->ws_size = 0;
        }
        const size_t sz = round_up((int64_t)bytes, 1 << 20);
        GOAC_HIP(ctx, hipMalloc(&ctx->ws, sz));
        ctx->ws_size = sz;
    }
    *out = ctx->ws;
    return GOAC_OK;
}

// ------------------------------------------------------------------ problem derivation kernels

// V64/V32 (M x Mp) and the bf16 split (Mp x Mp) of the mobile block, zero-padded
__global__ void k_extract(int64_t n, int32_t M, int32_t Mp, const double* __restrict__ V,
                          const int32_t* __restrict__ mob, double* __restrict__ V64, float* __restrict__ V32,
                          __hip_bfloat16* __restrict__ Vhi, __hip_bfloat16* __restrict__ Vlo) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)Mp * Mp) return;
    const int k = (int)(idx / Mp), l = (int)(idx - (int64_t)k * Mp);
    double v = 0.0;
    if (k < M && l < M) v = V[(int64_t)mob[k] * n + mob[l]];
    if (k < M) {
        V64[(int64_t)k * Mp + l] = v;
        V32[(int64_t)k * Mp + l] = (float)v;
    }
    const __hip_bfloat16 hi = __float2bfloat16((float)v);
    const double rest = v - (double)__bfloat162float(hi);
    Vhi[idx] = hi;
    Vlo[idx] = __float2bfloat16((float)rest);
}

// per mobile row k: diag, rowmax (rounded up), h_k = sum_f V[f][mob_k] q_f over
// the fixed sites (V symmetric), vc_k = sum_l V64[l][k] c_l and the field of the
// reference occupation phi_k = h_k + sum_l V64[l][k] q_l
__global__ void k_rows(int64_t n, int32_t M, int32_t Mp, const double* __restrict__ V, const int32_t* __restrict__ mob,
                       const int32_t* __restrict__ fixed_idx, const double* __restrict__ fixed_q, int32_t n_fixed,
                       const double* __restrict__ V64, const double* __restrict__ cvec, const double* __restrict__ qref,
                       double* __restrict__ diag, float* __restrict__ rowmax, double* __restrict__ rowabs,
                       double* __restrict__ h, double* __restrict__ vc, double* __restrict__ phiref) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Mp) return;
    if (k >= M) {
        h[k] = 0.0;
        vc[k] = 0.0;
        return;
    }
    const int64_t mk = mob[k];
    double hs = 0.0;
    for (int f = 0; f < n_fixed; ++f) hs += V[(int64_t)fixed_idx[f] * n + mk] * fixed_q[f];
    double s1 = 0.0, s2 = 0.0, mx = 0.0, ab = 0.0;
    for (int l = 0; l < M; ++l) {
        const double v = V64[(int64_t)l * Mp + k];
        s1 += v * cvec[l];
        s2 += v * qref[l];
        mx = fmax(mx, fabs(v));
        ab += fabs(v);
    }
    rowabs[k] = ab;
    diag[k] = V64[(int64_t)k * Mp + k];
    float r = (float)mx;
    if ((double)r < mx) r = nextafterf(r, INFINITY);
    rowmax[k] = r;
    h[k] = hs;
    vc[k] = s1;
    phiref[k] = hs + s2;
}

// fixed-ion energy terms: out[f] = q_f sum_f' V[f][f'] q_f'
__global__ void k_fixed_energy(int64_t n, const int32_t* __restrict__ fixed_idx, const double* __restrict__ fixed_q,
                               int32_t n_fixed, const double* __restrict__ V, double* __restrict__ out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_fixed) return;
    const int64_t a = fixed_idx[f];
    double s = 0.0;
    for (int g = 0; g < n_fixed; ++g) s += V[(int64_t)fixed_idx[g] * n + a] * fixed_q[g];
    out[f] = fixed_q[f] * s;
}

// single-thread sums in index order (deterministic):
//   out[0] = E_ff = 1/2 sum efix,  out[1] = E~ = E_ff + sum c_k h_k + 1/2 sum c_k vc_k,
//   out[2 + s] = mean of phiref over sublattice s; ht_k = h_k + vc_k
__global__ void k_derive_scalars(int32_t M, int32_t n_fixed, int32_t S, const double* __restrict__ efix,
                                 const double* __restrict__ cvec, const double* __restrict__ h,
                                 const double* __restrict__ vc, const double* __restrict__ phiref,
                                 const uint8_t* __restrict__ msub, double* __restrict__ ht,
                                 double* __restrict__ phibar, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double e = 0.0;
    for (int f = 0; f < n_fixed; ++f) e += efix[f];
    const double Eff = 0.5 * e;
    double ch = 0.0, cvc = 0.0;
    for (int k = 0; k < M; ++k) {
        ch += cvec[k] * h[k];
        cvc += cvec[k] * vc[k];
        ht[k] = h[k] + vc[k];
    }
    out[0] = Eff;
    out[1] = Eff + ch + 0.5 * cvc;
    double acc[kMaxSub];
    int cnt[kMaxSub];
    for (int s = 0; s < S; ++s) { acc[s] = 0.0; cnt[s] = 0; }
    for (int k = 0; k < M; ++k) { acc[msub[k]] += phiref[k]; cnt[msub[k]] += 1; }
    for (int s = 0; s < S; ++s) phibar[s] = cnt[s] ? acc[s] / cnt[s] : 0.0;
}

// ------------------------------------------------------------------ chain kernels

// composition check: err |= 1 when a chain's species counts per sublattice differ
__global__ void k_check_comp(int64_t n, int32_t M, int32_t S, int32_t E, const int32_t* __restrict__ tab,
                             const int32_t* __restrict__ mob, const uint8_t* __restrict__ msub,
                             const uint8_t* __restrict__ occ, int32_t* __restrict__ err) {
    __shared__ int hist[kMaxSub * kMaxSpecies];
    const int64_t c = blockIdx.x;
    for (int x = threadIdx.x; x < S * E; x += blockDim.x) hist[x] = 0;
    __syncthreads();
    bool bad = false;
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        const int e = occ[c * n + mob[k]];
        if (e >= E) bad = true;
        else atomicAdd(&hist[msub[k] * E + e], 1);
    }
    __syncthreads();
    const int32_t* cnt = tab + 2 + 2 * S;
    for (int x = threadIdx.x; x < S * E; x += blockDim.x)
        if (hist[x] != cnt[x]) bad = true;
    if (bad) atomicOr(err, 1);
}

// mobile occupation, perm (positions of each sublattice sorted by (species,
// position)) and the best copy of one chain
__global__ void k_chain_setup(int64_t n, int32_t M, int32_t Mp, int32_t S, int32_t E, const int32_t* __restrict__ tab,
                              const int32_t* __restrict__ mob, const uint8_t* __restrict__ msub,
                              const uint8_t* __restrict__ occ, int64_t first, const int64_t* __restrict__ offs,
                              uint8_t* __restrict__ occ_m, uint16_t* __restrict__ perm, uint8_t* __restrict__ best) {
    __shared__ int next[kMaxSub * kMaxSpecies];
    const int64_t c = blockIdx.x;
    const int64_t off = offs[first + c];
    const uint8_t* row = occ + c * n;
    for (int k = threadIdx.x; k < Mp; k += blockDim.x) {
        const uint8_t e = k < M ? row[mob[k]] : 0;
        occ_m[off + k] = e;
        best[off + k] = e;
        if (k >= M) perm[off + k] = 0;
    }
    const int32_t* subsize = tab + 2;
    const int32_t* suboff = subsize + S;
    const int32_t* offs_se = suboff + S + S * E;
    for (int x = threadIdx.x; x < S * E; x += blockDim.x) next[x] = suboff[x / E] + offs_se[x];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < M; ++k) {
            const int e = row[mob[k]];
            const int s = msub[k];
            if (e >= E) continue;                      // rejected by the composition check
            const int at = next[s * E + e]++;
            if (at < suboff[s] + subsize[s]) perm[off + at] = (uint16_t)k;
        }
}

// field and energy of every chain of one instance from Phi = Q V_mm (FP64):
// phi = Phi + h; E = E_ff + 1/2 sum q (phi + h); MIXED stores phi - phibar_s in
// FP32 with its error bound
template <bool MIXED>
__global__ __launch_bounds__(256) void k_chain_field(int32_t M, int32_t Mp, const double* __restrict__ Q,
                                                     const double* __restrict__ Phi, const double* __restrict__ h,
                                                     const double* __restrict__ rowabs, double qmax,
                                                     const uint8_t* __restrict__ msub,
                                                     const double* __restrict__ phibar, double E_ff, int64_t first,
                                                     ChainScalars* __restrict__ sc, void* __restrict__ phi) {
    __shared__ double s_a[256], s_b[256], s_c[256];
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
        const double E = E_ff + 0.5 * s_a[0];
        S->E = E;
        S->best_E = E;
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

// replica exchange: one thread per group of R consecutive chains
__global__ void k_remc(int64_t n_groups, int32_t R, const double* __restrict__ kT, uint64_t x, uint64_t seed,
                       ChainScalars* __restrict__ sc, int32_t* __restrict__ slot, uint8_t* __restrict__ acc) {
    const int64_t gidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gidx >= n_groups) return;
    int32_t* sl = slot + gidx * R;
    for (int k = 0; k < R; ++k)
        if ((uint32_t)sl[k] >= (uint32_t)R) return;    // not a permutation: left unchanged
    for (int k = (int)(x & 1u); k + 1 < R; k += 2) {
        const u32x4 r = philox((uint32_t)k, (uint32_t)x, (uint32_t)(x >> 32), ((uint32_t)gidx << 8) | TAG_REMC, seed);
        const double u = unit_open(r.x, r.y);
        const double Ea = sc[gidx * R + sl[k]].E, Eb = sc[gidx * R + sl[k + 1]].E;
        const double arg = (Ea - Eb) * (1.0 / kT[k] - 1.0 / kT[k + 1]);
        const bool ok = (arg >= 0.0) || (u < exp(arg));
        if (acc) acc[gidx * R + k] = ok ? 1 : 0;
        if (ok) {
            const int32_t t = sl[k];
            sl[k] = sl[k + 1];
            sl[k + 1] = t;
        }
    }
    for (int k = 0; k < R; ++k) sc[gidx * R + sl[k]].row = k;
}

__global__ void k_set_rows(int64_t C, const int32_t* __restrict__ rows, ChainScalars* __restrict__ sc) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C) sc[c].row = rows[c];
}

__global__ void k_zero_i32(int32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
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

#define GOAC_TRY(expr)                        \
    do {                                      \
        goac_status s_ = (expr);              \
        if (s_ != GOAC_OK) return s_;         \
    } while (0)

void problem_free(goac_problem* pb) {
    ProblemDev& d = pb->d;
    void* ptrs[] = {d.mob, d.msub, d.ref_occ, d.V64, d.V32, d.Vhi, d.Vlo, d.diag, d.rowmax, d.rowabs, d.h, d.ht, d.phibar,
                    d.charge, d.dq, d.tab, pb->spos, pb->spos_inv, pb->fixed_idx};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
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
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
    *out = ctx;
    return GOAC_OK;
}

extern "C" void goac_ctx_destroy(goac_ctx* ctx) {
    if (!ctx) return;
    if (ctx->ws) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->ws);
    }
    delete ctx;
}

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
    goac_status st = GOAC_OK;
    auto bail = [&](goac_status s) {
        problem_free(pb);
        delete pb;
        return s;
    };
#define PB_ALLOC(ptr, count)                                   \
    if ((st = dalloc(ctx, &(ptr), (count))) != GOAC_OK) return bail(st);
    PB_ALLOC(d.mob, M);
    PB_ALLOC(d.msub, Mp);
    PB_ALLOC(d.ref_occ, n);
    PB_ALLOC(d.V64, (size_t)M * Mp);
    PB_ALLOC(d.V32, (size_t)M * Mp);
    PB_ALLOC(d.Vhi, (size_t)Mp * Mp);
    PB_ALLOC(d.Vlo, (size_t)Mp * Mp);
    PB_ALLOC(d.diag, M);
    PB_ALLOC(d.rowmax, M);
    PB_ALLOC(d.rowabs, M);
    PB_ALLOC(d.h, Mp);
    PB_ALLOC(d.ht, Mp);
    PB_ALLOC(d.phibar, kMaxSub);
    PB_ALLOC(d.charge, E);
    PB_ALLOC(d.dq, S * E);
    PB_ALLOC(d.tab, tab.size());
    PB_ALLOC(pb->spos, M);
    PB_ALLOC(pb->spos_inv, M);
    PB_ALLOC(pb->fixed_idx, fixed.size() + 1);
#undef PB_ALLOC
    hipStream_t sm = ctx->stream;
#define PB_COPY(dst, src, bytes)                                                                     \
    if (hipMemcpyAsync((dst), (src), (bytes), hipMemcpyHostToDevice, sm) != hipSuccess) {            \
        ctx->err = "problem_create: upload failed";                                                 \
        return bail(GOAC_EHIP);                                                                     \
    }
    PB_COPY(d.mob, mob.data(), M * 4);
    PB_COPY(d.msub, msub.data(), Mp);
    PB_COPY(d.ref_occ, species, n);
    PB_COPY(d.charge, charge, E * 8);
    PB_COPY(d.dq, dq.data(), S * E * 8);
    PB_COPY(d.tab, tab.data(), tab.size() * 4);
    PB_COPY(pb->spos, spos.data(), M * 4);
    PB_COPY(pb->spos_inv, spos_inv.data(), M * 4);
    if (!fixed.empty()) PB_COPY(pb->fixed_idx, fixed.data(), fixed.size() * 4);
    // scratch for the derivation: fixed q, cvec, qref, efix, vc, phiref, scalars
    const int32_t nf = (int32_t)fixed.size();
    const size_t b_fq = round_up((nf + 1) * 8, 256), b_m = round_up(Mp * 8, 256);
    void* ws = nullptr;
    if ((st = workspace(ctx, b_fq * 2 + b_m * 4 + 256, &ws)) != GOAC_OK) return bail(st);
    char* p = (char*)ws;
    double* w_fq = (double*)p; p += b_fq;
    double* w_efix = (double*)p; p += b_fq;
    double* w_c = (double*)p; p += b_m;
    double* w_q = (double*)p; p += b_m;
    double* w_vc = (double*)p; p += b_m;
    double* w_phi = (double*)p; p += b_m;
    double* w_out = (double*)p;
    if (nf) PB_COPY(w_fq, fq.data(), nf * 8);
    PB_COPY(w_c, cvec.data(), Mp * 8);
    PB_COPY(w_q, qref.data(), Mp * 8);
#undef PB_COPY
    {
        const int64_t tot = (int64_t)Mp * Mp;
        hipLaunchKernelGGL(k_extract, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, sm, n, M, Mp, V, d.mob, d.V64,
                           d.V32, d.Vhi, d.Vlo);
        hipLaunchKernelGGL(k_rows, dim3((unsigned)((Mp + 127) / 128)), dim3(128), 0, sm, n, M, Mp, V, d.mob,
                           pb->fixed_idx, w_fq, nf, d.V64, w_c, w_q, d.diag, d.rowmax, d.rowabs, d.h, w_vc, w_phi);
        if (nf)
            hipLaunchKernelGGL(k_fixed_energy, dim3((unsigned)((nf + 127) / 128)), dim3(128), 0, sm, n, pb->fixed_idx,
                               w_fq, nf, V, w_efix);
        hipLaunchKernelGGL(k_derive_scalars, dim3(1), dim3(1), 0, sm, M, nf, S, w_efix, w_c, d.h, w_vc, w_phi,
                           d.msub, d.ht, d.phibar, w_out);
        if (hipGetLastError() != hipSuccess) {
            ctx->err = "problem_create: launch failed";
            return bail(GOAC_EHIP);
        }
        double sc[2];
        if (hipMemcpyAsync(sc, w_out, 16, hipMemcpyDeviceToHost, sm) != hipSuccess ||
            hipStreamSynchronize(sm) != hipSuccess) {
            ctx->err = "problem_create: derivation failed";
            return bail(GOAC_EHIP);
        }
        d.E_ff = sc[0];
        d.E_t = sc[1];
    }
    // ht beyond M is zero
    if (Mp > M && hipMemsetAsync(d.ht + M, 0, (Mp - M) * 8, sm) != hipSuccess) return bail(GOAC_EHIP);
    *out = pb;
    return GOAC_OK;
}

extern "C" void goac_problem_destroy(goac_problem* pb) {
    if (!pb) return;
    (void)hipStreamSynchronize(pb->ctx->stream);
    problem_free(pb);
    delete pb;
}

extern "C" goac_status goac_problem_get_info(const goac_problem* pb, goac_problem_info* out) {
    if (!pb || !out) return GOAC_EINVAL;
    out->n = pb->d.n;
    out->M = pb->d.M;
    out->n_sublattices = pb->d.S;
    out->n_species = pb->d.E;
    out->E_fixed = pb->d.E_ff;
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
    hipLaunchKernelGGL(k_init, dim3((unsigned)(C * d.S)), dim3(256), lds, ctx->stream, d.n, d.S, d.E, d.tab, pb->spos,
                       d.mob, pb->fixed_idx, pb->n_fixed, d.ref_occ, seed, chain_base, instance, occ);
    GOAC_CHECK_LAUNCH(ctx);
    return GOAC_OK;
}

// ------------------------------------------------------------------ energies, top-k
extern "C" goac_status goac_energies(goac_problem* pb, int64_t P, const uint8_t* occ, goac_precision prec,
                                     double* E) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (P < 0 || (P > 0 && (!occ || !E))) return fail(ctx, GOAC_EINVAL, "energies: bad arguments");
    if (P == 0) return GOAC_OK;
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    if (prec == GOAC_MIXED) {
        if (!pb->d.mixed_exact) return fail(ctx, GOAC_EINEXACT, "energies: a shifted charge is not bf16-exact");
        return energies_mixed(pb, P, occ, E);
    }
    if (prec != GOAC_FP64) return fail(ctx, GOAC_EINVAL, "energies: unknown precision");
    return energies_fp64(pb, P, occ, E);
}

extern "C" goac_status goac_topk_fp64(goac_problem* pb, int64_t P, const uint8_t* occ, int32_t k, int64_t* idx,
                                      double* Eout) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (P <= 0 || k <= 0 || k > P || !occ || !idx || !Eout) return fail(ctx, GOAC_EINVAL, "topk: bad arguments");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    double* E = nullptr;
    GOAC_HIP(ctx, hipMallocAsync((void**)&E, P * 8, ctx->stream));
    goac_status st = energies_fp64(pb, P, occ, E);
    if (st == GOAC_OK) {
        hipLaunchKernelGGL(k_topk_select, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, ctx->stream, P, k, E, idx,
                           Eout);
        if (hipGetLastError() != hipSuccess) st = fail(ctx, GOAC_EHIP, "topk: launch failed");
    }
    (void)hipFreeAsync(E, ctx->stream);
    return st;
}

// ------------------------------------------------------------------ GA
extern "C" goac_status goac_ga_generation(goac_problem* pb, int64_t P, const uint8_t* pop_in, const double* E_in,
                                          const goac_ga_params* prm, uint8_t* pop_out) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (P <= 0 || !pop_in || !E_in || !prm || !pop_out || pop_in == pop_out || !(prm->p_mut >= 0.0))
        return fail(ctx, GOAC_EINVAL, "ga_generation: bad arguments");
    if (P > (int64_t)1 << 30) return fail(ctx, GOAC_EINVAL, "ga_generation: population too large");
    const ProblemDev& d = pb->d;
    const size_t lds = 3 * round_up(d.M, 16);
    if (lds > 160 * 1024) return fail(ctx, GOAC_EINVAL, "ga_generation: too many mobile positions");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    const int32_t ne = (int32_t)std::min<int64_t>(std::max(prm->n_elite, 0), P);
    void* ws = nullptr;
    const size_t b_cum = round_up(P * 8, 256), b_el = round_up((ne + 1) * 4, 256);
    GOAC_TRY(workspace(ctx, b_cum + b_el + 256, &ws));
    uint64_t* cum = (uint64_t*)ws;
    int32_t* elite = (int32_t*)((char*)ws + b_cum);
    int32_t* err = (int32_t*)((char*)ws + b_cum + b_el);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, err, 1);
    hipLaunchKernelGGL(k_ga_prep, dim3(1), dim3(1024), 0, ctx->stream, P, E_in, ne, cum, elite, err);
    GOAC_CHECK_LAUNCH(ctx);
    if (lds > 64 * 1024)
        GOAC_HIP(ctx, hipFuncSetAttribute((const void*)k_ga_child, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_ga_child, dim3((unsigned)P), dim3(64), lds, ctx->stream, d.n, d.M, d.S, d.E, d.tab, pb->spos,
                       pb->spos_inv, d.msub, d.mob, pb->fixed_idx, pb->n_fixed, d.ref_occ, P, pop_in, cum, elite, ne,
                       prm->seed, prm->generation, prm->p_mut, pop_out);
    GOAC_CHECK_LAUNCH(ctx);
    int32_t herr = 0;
    GOAC_HIP(ctx, hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, ctx->stream));
    GOAC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (herr) return fail(ctx, GOAC_EINVAL, "ga_generation: energy spread too large for the roulette weights");
    return GOAC_OK;
}

// ------------------------------------------------------------------ chains
static goac_status chains_build(goac_chains* ch, const uint8_t* occ) {
    goac_ctx* ctx = ch->ctx;
    const int n_inst = (int)ch->pbs.size();
    hipStream_t sm = ctx->stream;
    const bool mixed = ch->prec == GOAC_MIXED;
    // per-chain offsets
    ch->offs.resize(ch->C);
    int64_t tot = 0;
    for (int64_t c = 0; c < ch->C; ++c) {
        ch->offs[c] = tot;
        tot += ch->pbs[ch->inst_of[c]]->d.Mp;
    }
    ch->total = tot;
    GOAC_TRY(dalloc(ctx, &ch->sc, ch->C));
    GOAC_TRY(dalloc(ctx, &ch->insts, n_inst));
    GOAC_TRY(dalloc(ctx, &ch->occ, tot));
    GOAC_TRY(dalloc(ctx, &ch->perm, tot));
    GOAC_TRY(dalloc(ctx, &ch->best, tot));
    GOAC_TRY(dalloc(ctx, &ch->order, ch->C));
    GOAC_TRY(dalloc(ctx, &ch->queue, 64));
    GOAC_TRY(dalloc(ctx, &ch->d_offs, ch->C));
    void* phi = nullptr;
    GOAC_HIP(ctx, hipMalloc(&phi, (size_t)tot * (mixed ? 4 : 8) + 16));
    ch->phi = phi;
    // instance table
    std::vector<McInst> insts(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const ProblemDev& d = ch->pbs[i]->d;
        McInst& I = insts[i];
        I.V64 = d.V64; I.V32 = d.V32; I.diag = d.diag; I.rowmax = d.rowmax; I.h = d.h; I.phibar = d.phibar;
        I.msub = d.msub; I.tab = d.tab; I.charge = d.charge; I.E_ff = d.E_ff;
        I.M = d.M; I.Mp = d.Mp; I.S = d.S; I.E = d.E;
        I.instance = ch->inst_id[i];
        I.pad_ = 0;
        ch->max_Mp = std::max(ch->max_Mp, d.Mp);
        ch->max_S = std::max(ch->max_S, d.S);
        ch->max_E = std::max(ch->max_E, d.E);
        ch->max_tab = std::max(ch->max_tab, tab_words(d.S, d.E));
    }
    GOAC_HIP(ctx, hipMemcpyAsync(ch->insts, insts.data(), n_inst * sizeof(McInst), hipMemcpyHostToDevice, sm));
    // scalars
    std::vector<ChainScalars> sc(ch->C);
    for (int64_t c = 0; c < ch->C; ++c) {
        ChainScalars& s = sc[c];
        std::memset(&s, 0, sizeof(s));
        s.inst = ch->inst_of[c];
        s.chain_id = ch->chain_id[c];
        s.off = ch->offs[c];
    }
    GOAC_HIP(ctx, hipMemcpyAsync(ch->sc, sc.data(), ch->C * sizeof(ChainScalars), hipMemcpyHostToDevice, sm));
    GOAC_HIP(ctx, hipMemcpyAsync(ch->d_offs, ch->offs.data(), ch->C * 8, hipMemcpyHostToDevice, sm));
    // longest chains first (Mp as the cost), stable
    std::vector<int32_t> order(ch->C);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return ch->pbs[ch->inst_of[a]]->d.Mp > ch->pbs[ch->inst_of[b]]->d.Mp;
    });
    GOAC_HIP(ctx, hipMemcpyAsync(ch->order, order.data(), ch->C * 4, hipMemcpyHostToDevice, sm));
    // composition check, setup and FP64 field, per instance
    int32_t* err = nullptr;
    GOAC_TRY(dalloc(ctx, &err, 1));
    DevAllocs tmp;
    tmp.ptrs.push_back(err);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, sm, err, 1);
    for (int i = 0; i < n_inst; ++i) {
        goac_problem* pb = ch->pbs[i];
        const ProblemDev& d = pb->d;
        const int64_t Ci = ch->count[i];
        if (Ci == 0) continue;
        const uint8_t* occ_i = occ + ch->occ_row_off[i];
        hipLaunchKernelGGL(k_check_comp, dim3((unsigned)Ci), dim3(256), 0, sm, d.n, d.M, d.S, d.E, d.tab, d.mob,
                           d.msub, occ_i, err);
        hipLaunchKernelGGL(k_chain_setup, dim3((unsigned)Ci), dim3(64), 0, sm, d.n, d.M, d.Mp, d.S, d.E, d.tab, d.mob,
                           d.msub, occ_i, ch->first_chain[i], ch->d_offs, ch->occ, ch->perm, ch->best);
        double *Q = nullptr, *Phi = nullptr;
        GOAC_HIP(ctx, hipMallocAsync((void**)&Q, (size_t)Ci * d.Mp * 8, sm));
        GOAC_HIP(ctx, hipMallocAsync((void**)&Phi, (size_t)Ci * d.Mp * 8, sm));
        GOAC_TRY(build_q64(ctx, Ci, d.n, d.M, d.Mp, d.E, occ_i, d.mob, d.charge, Q));
        GOAC_TRY(dgemm_nt(ctx, Ci, d.M, d.Mp, Q, d.Mp, d.V64, d.Mp, Phi, d.Mp, 1.0, 0.0, nullptr));
        if (mixed)
            hipLaunchKernelGGL(k_chain_field<true>, dim3((unsigned)Ci), dim3(256), 0, sm, d.M, d.Mp, Q, Phi, d.h,
                               d.rowabs, d.qmax, d.msub, d.phibar, d.E_ff, ch->first_chain[i], ch->sc, ch->phi);
        else
            hipLaunchKernelGGL(k_chain_field<false>, dim3((unsigned)Ci), dim3(256), 0, sm, d.M, d.Mp, Q, Phi, d.h,
                               d.rowabs, d.qmax, d.msub, d.phibar, d.E_ff, ch->first_chain[i], ch->sc, ch->phi);
        GOAC_CHECK_LAUNCH(ctx);
        GOAC_HIP(ctx, hipFreeAsync(Q, sm));
        GOAC_HIP(ctx, hipFreeAsync(Phi, sm));
    }
    int32_t herr = 0;
    GOAC_HIP(ctx, hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, sm));
    GOAC_HIP(ctx, hipStreamSynchronize(sm));
    if (herr) return fail(ctx, GOAC_EINVAL, "chains_create: an occupation breaks the problem's composition");
    return GOAC_OK;
}

static void chains_free(goac_chains* ch) {
    void* ptrs[] = {ch->sc, ch->insts, ch->phi, ch->occ, ch->perm, ch->best, ch->order, ch->queue, ch->kT, ch->d_offs};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
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
        if (!pbs[i] || pbs[i]->ctx != ctx || cpi[i] < 0) {
            delete ch;
            return fail(ctx, GOAC_EINVAL, "chains_create_batch: bad instance");
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
    *out = ch;
    return GOAC_OK;
}

extern "C" void goac_chains_destroy(goac_chains* ch) {
    if (!ch) return;
    (void)hipStreamSynchronize(ch->ctx->stream);
    chains_free(ch);
    delete ch;
}

extern "C" goac_status goac_chains_set_rows(goac_chains* ch, const int32_t* rows) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    if (!rows) return fail(ctx, GOAC_EINVAL, "chains_set_rows: null rows");
    for (int64_t c = 0; c < ch->C; ++c)
        if (rows[c] < 0) return fail(ctx, GOAC_EINVAL, "chains_set_rows: negative row");
    int32_t* d = nullptr;
    GOAC_HIP(ctx, hipMallocAsync((void**)&d, ch->C * 4, ctx->stream));
    GOAC_HIP(ctx, hipMemcpyAsync(d, rows, ch->C * 4, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_set_rows, dim3((unsigned)((ch->C + 255) / 256)), dim3(256), 0, ctx->stream, ch->C, d, ch->sc);
    GOAC_CHECK_LAUNCH(ctx);
    GOAC_HIP(ctx, hipFreeAsync(d, ctx->stream));
    GOAC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ch->max_row = 0;
    for (int64_t c = 0; c < ch->C; ++c) ch->max_row = std::max(ch->max_row, rows[c]);
    return GOAC_OK;
}

extern "C" goac_status goac_mc_sweep(goac_chains* ch, const goac_mc_params* prm) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    if (!prm || !prm->kT_host || prm->n_rows <= 0 || prm->n_blocks <= 0 || prm->block_len == 0)
        return fail(ctx, GOAC_EINVAL, "mc_sweep: bad parameters");
    if (prm->n_rows <= ch->max_row) return fail(ctx, GOAC_EINVAL, "mc_sweep: a chain's temperature row is beyond n_rows");
    const size_t nkT = (size_t)prm->n_rows * prm->n_blocks;
    for (size_t x = 0; x < nkT; ++x)
        if (!(prm->kT_host[x] > 0.0)) return fail(ctx, GOAC_EINVAL, "mc_sweep: kT must be positive");
    const bool mixed = ch->prec == GOAC_MIXED;
    if (mixed && prm->reanchor_every <= 0) return fail(ctx, GOAC_EINVAL, "mc_sweep: reanchor_every must be positive");
    if (prm->n_trials == 0) return GOAC_OK;
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    if (nkT > ch->kT_cap) {
        if (ch->kT) {
            GOAC_HIP(ctx, hipStreamSynchronize(ctx->stream));
            GOAC_HIP(ctx, hipFree(ch->kT));
            ch->kT = nullptr;
        }
        GOAC_TRY(dalloc(ctx, &ch->kT, nkT));
        ch->kT_cap = nkT;
    }
    GOAC_HIP(ctx, hipMemcpyAsync(ch->kT, prm->kT_host, nkT * 8, hipMemcpyHostToDevice, ctx->stream));
    // the persistent grid pulls chains from a counter that starts at zero
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, ch->queue, 1);
    const int wg = prm->variant == 64 || prm->variant == 256 ? prm->variant : (ch->max_Mp >= 2048 ? 256 : 64);
    if (prm->variant != 0 && prm->variant != 64 && prm->variant != 256)
        return fail(ctx, GOAC_EINVAL, "mc_sweep: variant must be 0, 64 or 256");
    const size_t phi_bytes = (size_t)round_up(ch->max_Mp * (mixed ? 4 : 8), 16);
    const size_t lds = phi_bytes + (size_t)ch->max_Mp * (1 + 1 + 2 + 2) + round_up(ch->max_tab * 4, 16) +
                       kMaxSpecies * 8;
    if (lds > 160 * 1024) return fail(ctx, GOAC_EINVAL, "mc_sweep: the chain state does not fit in LDS");
    const int per_cu = std::max<int>(1, std::min<int>(wg == 64 ? 16 : 4, (int)((160 * 1024) / lds)));
    int grid = std::min<int64_t>(ch->C, (int64_t)ctx->num_cus * per_cu);
    McArgs a;
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
    return mc_launch(ctx, a, mixed, (prm->flags & GOAC_MC_TRACE_HASH) != 0, wg, lds, grid);
}

extern "C" goac_status goac_chains_export(goac_chains* ch, uint8_t* occ, uint8_t* best, goac_chain_stats* stats) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
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

extern "C" goac_status goac_remc_exchange(goac_chains* ch, int32_t R, const double* kT_host, uint64_t x,
                                          uint64_t seed, int32_t* slot, uint8_t* acc) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    if (R < 2 || !kT_host || !slot || ch->C % R != 0)
        return fail(ctx, GOAC_EINVAL, "remc_exchange: R must be >= 2 and divide the chain count");
    for (int k = 0; k < R; ++k)
        if (!(kT_host[k] > 0.0)) return fail(ctx, GOAC_EINVAL, "remc_exchange: kT must be positive");
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    double* d = nullptr;
    GOAC_HIP(ctx, hipMallocAsync((void**)&d, R * 8, ctx->stream));
    GOAC_HIP(ctx, hipMemcpyAsync(d, kT_host, R * 8, hipMemcpyHostToDevice, ctx->stream));
    const int64_t ng = ch->C / R;
    hipLaunchKernelGGL(k_remc, dim3((unsigned)((ng + 63) / 64)), dim3(64), 0, ctx->stream, ng, R, d, x, seed, ch->sc,
                       slot, acc);
    GOAC_CHECK_LAUNCH(ctx);
    GOAC_HIP(ctx, hipFreeAsync(d, ctx->stream));
    ch->max_row = std::max(ch->max_row, R - 1);
    return GOAC_OK;
}
