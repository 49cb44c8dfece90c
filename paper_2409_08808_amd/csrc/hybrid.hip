// One round of the replica-exchange + genetic-algorithm hybrid (SI, "Hybrid
// Methods": the two heuristics run alternately and hand their best solutions to
// each other), composed from the library's own kernels:
//   1. REMC phase: `exchanges` times, every chain runs `trials` trials at the
//      temperature of its slot, then one exchange step x = round exchanges + e in
//      every group of R consecutive chains;
//   2. REMC -> GA: the population becomes the P lowest, by (FP64 energy, index),
//      of the population followed by the chains' best occupations;
//   3. GA phase: `generations` generations g = round generations + k, each
//      followed by the children's energies (the requested precision);
//   4. GA -> REMC: the coldest replica of group k takes the individual of rank
//      k mod min(inject, P) (order (E, index)) when that individual is strictly
//      lower than the replica's current energy; all chains continue from their
//      occupations (counters and rows kept, the best replaced only when beaten).
#include <algorithm>

#include "common.h"

namespace goac {

// rows of every group from its slot permutation: one workgroup per group checks
// that the slots are a permutation of 0..R-1 (an LDS bit per value, as the
// exchange step does) and leaves a group that is not one unchanged
__global__ void k_rows_from_slot(int64_t n_groups, int32_t R, const int32_t* __restrict__ slot,
                                 ChainScalars* __restrict__ sc) {
    extern __shared__ uint32_t seen[];
    __shared__ int s_bad;
    const int64_t g = blockIdx.x;
    if (g >= n_groups) return;
    const int32_t* sl = slot + g * R;
    for (int w = threadIdx.x; w < (R + 31) / 32; w += blockDim.x) seen[w] = 0;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < R; k += blockDim.x) {
        const int32_t v = sl[k];
        if ((uint32_t)v >= (uint32_t)R) {
            s_bad = 1;
        } else {
            const uint32_t bit = 1u << (v & 31);
            if (atomicOr(&seen[v >> 5], bit) & bit) s_bad = 1;
        }
    }
    __syncthreads();
    if (s_bad) return;
    for (int k = threadIdx.x; k < R; k += blockDim.x) sc[g * R + sl[k]].row = k;
}

// dst row r = src row idx[r]
__global__ void k_gather_rows(int64_t rows, int64_t n, const int64_t* __restrict__ idx,
                              const uint8_t* __restrict__ src, uint8_t* __restrict__ dst) {
    const int64_t r = blockIdx.x;
    if (r >= rows) return;
    const uint8_t* s = src + idx[r] * n;
    uint8_t* d = dst + r * n;
    for (int64_t x = threadIdx.x; x < n; x += blockDim.x) d[x] = s[x];
}

// group g's coldest replica takes individual order[g mod n_inj] when it is lower
__global__ void k_inject(int64_t n_groups, int32_t R, int32_t n_inj, int64_t n, const int32_t* __restrict__ slot,
                         const int64_t* __restrict__ order, const uint8_t* __restrict__ pop,
                         const double* __restrict__ E_pop, const ChainScalars* __restrict__ sc,
                         uint8_t* __restrict__ occ) {
    const int64_t g = blockIdx.x;
    if (g >= n_groups) return;
    const int32_t s0 = slot[g * R];
    if ((uint32_t)s0 >= (uint32_t)R) return;
    const int64_t c = g * R + s0;
    const int64_t i = order[g % n_inj];
    if (!(E_pop[i] < sc[c].E)) return;
    for (int64_t x = threadIdx.x; x < n; x += blockDim.x) occ[c * n + x] = pop[i * n + x];
}

static goac_status chains_scratch(goac_chains* ch, size_t bytes, void** out) {
    goac_ctx* ctx = ch->ctx;
    if (bytes > ch->scratch_size) {
        pool_put(ctx, ch->scratch, ch->scratch_size);
        ch->scratch = nullptr;
        ch->scratch_size = 0;
        size_t got = bytes;
        GOAC_TRY(pool_get(ctx, &got, &ch->scratch));
        ch->scratch_size = got;
    }
    *out = ch->scratch;
    return GOAC_OK;
}

}  // namespace goac

using namespace goac;


extern "C" goac_status goac_hybrid_round(goac_chains* ch, int32_t* slot_dev, int64_t P, uint8_t* pop_dev,
                                         double* E_dev, const goac_hybrid_params* prm) {
    if (!ch) return GOAC_EINVAL;
    goac_ctx* ctx = ch->ctx;
    if (!prm || !slot_dev || !pop_dev || !E_dev || P <= 0 || P > (1 << 30))
        return fail(ctx, GOAC_EINVAL, "hybrid_round: bad arguments");
    if (ch->pbs.size() != 1) return fail(ctx, GOAC_ESTATE, "hybrid_round: chains of one problem only");
    const int32_t R = prm->R;
    if (R < 2 || R > (1 << 19) || ch->C % R != 0 || !prm->kT_host || prm->exchanges < 0 || prm->generations < 0 ||
        prm->trials < 0 || !(prm->p_mut >= 0.0) || (prm->precision != GOAC_FP64 && prm->precision != GOAC_MIXED))
        return fail(ctx, GOAC_EINVAL, "hybrid_round: bad parameters");
    for (int k = 0; k < R; ++k)
        if (!(prm->kT_host[k] > 0.0)) return fail(ctx, GOAC_EINVAL, "hybrid_round: kT must be positive");
    goac_problem* pb = ch->pbs[0];
    const int64_t n = pb->d.n, C = ch->C, G = C / R, PC = P + C;
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    GOAC_TRY(rows_check(pb, P, pop_dev, "hybrid_round"));
    // scratch: candidates, their energies, ranks, second population, chain rows
    const size_t b_cand = round_up(PC * n, 256), b_E = round_up(PC * 8, 256), b_idx = round_up(PC * 8, 256);
    const size_t b_cnt = round_up(PC * 4, 256), b_pop = round_up(P * n, 256), b_occ = round_up(C * n, 256);
    void* base = nullptr;
    GOAC_TRY(chains_scratch(ch, b_cand + b_E + b_idx + b_cnt + b_pop + b_occ, &base));
    uint8_t* cand = (uint8_t*)base;
    double* Ecand = (double*)((char*)base + b_cand);
    int64_t* idx = (int64_t*)((char*)base + b_cand + b_E);
    int32_t* cnt = (int32_t*)((char*)base + b_cand + b_E + b_idx);
    uint8_t* pop2 = (uint8_t*)((char*)base + b_cand + b_E + b_idx + b_cnt);
    uint8_t* occ_buf = pop2 + b_pop;
    hipStream_t sm = ctx->stream;

    // 1. REMC phase
    hipLaunchKernelGGL(k_rows_from_slot, dim3((unsigned)G), dim3(R <= 128 ? 64 : 256), (size_t)((R + 31) / 32) * 4, sm,
                       G, R, slot_dev, ch->sc);
    GOAC_CHECK_LAUNCH(ctx);
    for (int32_t e = 0; e < prm->exchanges; ++e) {
        if (prm->trials > 0) {
            goac_mc_params mp{};
            mp.seed = prm->seed;
            mp.n_trials = (uint64_t)prm->trials;
            mp.kT_host = prm->kT_host;
            mp.n_rows = R;
            mp.n_blocks = 1;
            mp.block_len = (uint64_t)prm->trials;
            mp.reanchor_every = prm->reanchor_every > 0 ? prm->reanchor_every : 1024;
            GOAC_TRY(goac_mc_sweep(ch, &mp));
        }
        GOAC_TRY(goac_remc_exchange(ch, R, prm->kT_host, prm->round * (uint64_t)prm->exchanges + (uint64_t)e,
                                      prm->seed, slot_dev, nullptr));
    }
    // 2. REMC -> GA: the P lowest of the population and the chains' bests
    GOAC_HIP(ctx, hipMemcpyAsync(cand, pop_dev, (size_t)(P * n), hipMemcpyDeviceToDevice, sm));
    GOAC_TRY(chains_export_enqueue(ch, nullptr, cand + P * n, nullptr));
    GOAC_TRY(energies_fp64(pb, PC, cand, Ecand));
    GOAC_TRY(rank_select(ctx, PC, Ecand, (int32_t)P, cnt, idx, nullptr, E_dev));
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)P), dim3(256), 0, sm, P, n, idx, cand, pop_dev);
    GOAC_CHECK_LAUNCH(ctx);
    // 3. GA phase (double-buffered; the result ends in pop_dev)
    // (a failed roulette is reported once, after the last generation)
    uint8_t* cur = pop_dev;
    uint8_t* other = pop2;
    int32_t* ga_err = nullptr;
    for (int32_t k = 0; k < prm->generations; ++k) {
        goac_ga_params gp{};
        gp.seed = prm->seed;
        gp.generation = (uint32_t)(prm->round * (uint64_t)prm->generations + (uint64_t)k);
        gp.n_elite = prm->n_elite;
        gp.p_mut = prm->p_mut;
        GOAC_TRY(ga_generation_enqueue(pb, P, cur, E_dev, &gp, other, k == 0, &ga_err));
        GOAC_TRY(energies_enqueue(pb, P, other, (goac_precision)prm->precision, E_dev));
        std::swap(cur, other);
    }
    if (ga_err) GOAC_TRY(ga_check_err(ctx, ga_err));
    if (cur != pop_dev) GOAC_HIP(ctx, hipMemcpyAsync(pop_dev, cur, (size_t)(P * n), hipMemcpyDeviceToDevice, sm));
    // 4. GA -> REMC: the best individuals to the groups' coldest replicas
    const int32_t n_inj = (int32_t)std::max<int64_t>(1, std::min<int64_t>(prm->inject, P));
    GOAC_TRY(rank_select(ctx, P, E_dev, n_inj, cnt, idx, nullptr, nullptr));
    GOAC_TRY(chains_export_enqueue(ch, occ_buf, nullptr, nullptr));
    hipLaunchKernelGGL(k_inject, dim3((unsigned)G), dim3(256), 0, sm, G, R, n_inj, n, slot_dev, idx, pop_dev, E_dev,
                       ch->sc, occ_buf);
    GOAC_CHECK_LAUNCH(ctx);
    return goac_chains_load(ch, occ_buf);
}
