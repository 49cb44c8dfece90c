"""Benchmark of the Coulomb cluster-expansion hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic input, the
4x4x4 rock-salt supercell (N = 512; 256 O2- fixed; Li+ 128, Ni2+ 32, Co3+ 64,
Mn4+ 32 on 256 cation positions):
  1. FP64 Ewald pair matrix (real-space erfc + reciprocal sum on matrix cores)
  2. problem derivation (mobile block in FP64/FP32/bf16 hi+lo, fixed-ion field)
  3. 4096 random starts, 4096 chains
  4. 4096 chains x 1e5 swap trials, kT 0.5 -> 0.01 eV geometric over 100 blocks
     of 1000 trials; FP32 field with FP64 re-anchoring every 1024 field updates
  5. energies of the 4096 best occupations (bf16 hi+lo matrix-core product)
  6. one GA generation on them (8 elites, mutation rate 0.2)
  7. FP64 top-64 of the 4096 best occupations
value = swap trials per second over whole steps (inputs resident on the GPU).

Also measured: the same step with the FP64 field and FP64 energies ("plain
FP64"), and population energies per second of the GA workload (8x8x8 rock-salt,
N = 4096, P = 1024, 200 generations: bf16 hi+lo energies, GA generation).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MC swap-trials/s and config energies/s, mixed+batched vs plain FP64, 1 GPU"
CHAINS, TRIALS, BLOCKS, BLOCK_LEN = 4096, 100000, 100, 1000
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit or FP64 VALU lane operations per second
ALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
BF16_PEAK = 2.5e15
# HBM bytes of one k_mc<mixed, 64> launch of this step from FETCH_SIZE and WRITE_SIZE,
# each scaled by the same counter's reading for a 256 MiB copy (factors 2.0 and 1.0);
# valid only for the kernel sources they were taken on (profiles/k_mc_rocksalt4x4x4_traffic.md)
MC_TRAFFIC = {"bytes": 46128444.0,
              "sources": ("paper_2409_08808_amd/csrc/mc.hip", "paper_2409_08808_amd/csrc/common.h"),
              "sha256": "5d02a610c58232fd30f5d87930668adfcee22d9f121e06898af616cd51492ea1"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the plain-FP64 and GA-energies legs")
    ap.add_argument("--calibrate-copy", action="store_true", help="also run a copy kernel of known size")
    ap.add_argument("--ga-generations", type=int, default=200)
    ap.add_argument("--no-large", action="store_true", help="skip the 16384-site and 512-instance legs")
    ap.add_argument("--only", default="", help="comma list of legs to run alone: fp64, ga, cfg5, cfg4, nacl, "
                                                "gd, remc, hybrid (the step itself always runs)")
    return ap.parse_args()


def measured_traffic(entry):
    """The counter-based traffic figure, or None once its kernel sources changed."""
    import hashlib
    h = hashlib.sha256()
    for f in entry["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return entry["bytes"] if h.hexdigest() == entry["sha256"] else None


def algorithmic_ops(trials, updates, M):
    """VALU lane-operations a trial and a field update need at minimum:
    Philox4x32-10 80 (10 rounds of 2 mul-lo, 2 mul-hi, 4 xor), two index maps 4,
    the uniform 4, dE 10, the Metropolis test 20 (one logarithm); a field update
    2 fused multiply-adds per mobile position."""
    return trials * 118.0 + updates * 2.0 * M


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the hot path would shard chains, instances and "
              "populations without communication, but only a single MI355X is measured "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2409_08808_amd as G
    import supercells as S

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    ctx = G.Context(0, stream)
    cell = S.config2()
    kT = np.geomspace(0.5, 0.01, BLOCKS)

    def step(seed, prec, ev=None, host_stats=False):
        V = ctx.build_ewald(cell["lattice"], cell["pos"])
        pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
        occ0 = pb.init_occupations(CHAINS, seed=seed)
        ch = G.Chains(pb, occ0, prec)
        if ev is not None:
            ev[0].record(stream)
        ch.sweep(TRIALS, kT, BLOCK_LEN, seed=seed, reanchor_every=1024)
        if ev is not None:
            ev[1].record(stream)
        occ, best, stats = ch.export(host_stats=host_stats)
        best = best.view(CHAINS, -1)
        E = pb.energies(best, G.GOAC_MIXED if prec == G.GOAC_MIXED else G.GOAC_FP64)
        pb.ga_generation(best, E, seed=seed, generation=0, n_elite=8, p_mut=0.2)
        idx, Ek = pb.topk(best, 64)
        # no wait here: releases are stream-ordered, so the next step's host work
        # overlaps this step's last kernels
        ch.close()
        pb.close()
        return stats

    def timed(prec, steps, warmup):
        for w in range(warmup):
            step(1000 + w, prec)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        stats = None
        for k in range(steps):
            stats = step(k, prec, evs[k], host_stats=(k == steps - 1))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern = np.array([a.elapsed_time(b) for a, b in evs]) * 1e-3
        print("  [%s] %d steps in %.3f s; sweep %.2f ms avg" % ("mixed" if prec else "fp64", steps, wall,
                                                               1e3 * kern.mean()), file=sys.stderr, flush=True)
        return wall, kern, stats

    wall, kern, stats = timed(G.GOAC_MIXED, args.steps, args.warmup)
    total_trials = float(CHAINS) * TRIALS * args.steps
    value = total_trials / wall
    M = 256
    upd = float(stats["updates"].sum())
    ops = algorithmic_ops(float(CHAINS) * TRIALS, upd, M)
    achieved = ops / kern.mean()
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "swap-trials/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "rock-salt 4x4x4 (N=512, M=256; Li/Ni/Co/Mn 128/32/64/32), 4096 chains x 1e5 "
                               "trials, kT 0.5->0.01 eV over 100 blocks, FP32 field + FP64 re-anchor/1024, "
                               "then bf16 energies, GA generation and FP64 top-64 of the chain bests",
                   "chains": CHAINS, "trials_per_chain": TRIALS, "parallelism": "chains per workgroup"},
        "mc_sweep_ms": 1e3 * kern.mean(),
        "mc_trials_per_s_kernel": CHAINS * TRIALS / kern.mean(),
        "accept_rate": float(stats["accepts"].sum()) / (CHAINS * TRIALS),
        "field_updates_per_chain": upd / CHAINS,
        "fallbacks_per_chain": float(stats["fallbacks"].sum()) / CHAINS,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved / ALU_PEAK_OPS, "traffic": measured_traffic(MC_TRAFFIC),
                     "kernel": "k_mc<mixed>", "ops_per_launch": ops},
    }
    legs = set(args.only.split(",")) - {""}
    if not legs and not args.no_extras:
        legs = {"fp64", "ga", "nacl", "gd", "remc", "hybrid"} | (set() if args.no_large else {"cfg5", "cfg4"})
    if "fp64" in legs:
        w64, k64, s64 = timed(G.GOAC_FP64, max(2, args.steps // 2), 1)
        result["plain_fp64_trials_per_s"] = float(CHAINS) * TRIALS * max(2, args.steps // 2) / w64
        result["plain_fp64_sweep_ms"] = 1e3 * k64.mean()
        result["mixed_vs_fp64"] = result["value"] / result["plain_fp64_trials_per_s"]
    if "ga" in legs:
        result.update(ga_energies(ctx, G, S, torch, stream, args.ga_generations))
    if "cfg5" in legs:
        result.update(large_cell(ctx, G, S, torch, stream))
    if "cfg4" in legs:
        result.update(batched_instances(ctx, G, S, torch, stream))
    if "nacl" in legs:
        result.update(nacl_half(ctx, G, S, torch, stream))
    if "gd" in legs:
        result.update(gradient_descent(ctx, G, S, torch, stream))
    if "remc" in legs:
        result.update(replica_exchange(ctx, G, S, torch, stream))
    if "hybrid" in legs:
        result.update(hybrid(ctx, G, S, torch, stream))
    if args.calibrate_copy:
        x = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = 2 * x.numel()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(S)
    print(json.dumps(result), flush=True)


def ga_energies(ctx, G, S, torch, stream, generations):
    """GA workload: 8x8x8 rock-salt (N = 4096), P = 1024, `generations`
    generations; energies/s counts only the population-energy calls (mixed: with
    the tile the autotuner picked for this population size)."""
    cell = S.config3()
    V = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    del V
    out = {}
    for prec, name in ((G.GOAC_MIXED, "mixed"), (G.GOAC_FP64, "fp64")):
        pop = pb.init_occupations(1024, seed=0)
        E = torch.empty(1024, dtype=torch.float64, device=pop.device)
        if prec == G.GOAC_MIXED:
            out["ga_mixed_tile_autotuned"] = pb.energies_autotune(pop)
        pb.energies(pop, prec, out=E)                      # warm-up
        torch.cuda.synchronize()
        t_en = 0.0
        t0 = time.perf_counter()
        gens = generations if prec == G.GOAC_MIXED else max(10, generations // 10)
        for g in range(gens):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            pb.energies(pop, prec, out=E)
            b.record(stream)
            pop = pb.ga_generation(pop, E, seed=0, generation=g, n_elite=8, p_mut=0.2)
            b.synchronize()
            t_en += a.elapsed_time(b) * 1e-3
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out["ga_%s_energies_per_s" % name] = 1024 * gens / t_en
        out["ga_%s_energy_call_us" % name] = 1e6 * t_en / gens
        out["ga_%s_generation_ms" % name] = 1e3 * wall / gens
        if prec == G.GOAC_MIXED:
            # the symmetric product forms the upper triangle of the (k, n) plane, hi
            # and lo: 2 x 2 x P x M (M + 1) / 2 flops per call
            flops = 2 * 2.0 * 1024 * 2048 * 2049 / 2
            out["ga_mixed_mfma_frac"] = flops / (t_en / gens) / BF16_PEAK
            out["ga_run_mixed_generation_ms"] = 1e3 * ga_run_time(G, pb, torch, prec, 1024, gens)
    out["energies_per_s"] = out["ga_mixed_energies_per_s"]
    pb.close()
    # the same generation loop on the 4x4x4 cell (M = 256), where a generation is short
    # enough for the per-call work to show: generation by generation from Python
    # against goac_ga_run (graph replays)
    cell = S.config2()
    V = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    del V
    gens = 100
    pop = pb.init_occupations(1024, seed=0)
    E = pb.energies(pop, G.GOAC_MIXED)
    pb.ga_generation(pop, E, seed=0, generation=0)             # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(gens):
        pop = pb.ga_generation(pop, E, seed=0, generation=g, n_elite=8, p_mut=0.2)
        pb.energies(pop, G.GOAC_MIXED, out=E)
    torch.cuda.synchronize()
    out["ga_cfg2_loop_generation_ms"] = 1e3 * (time.perf_counter() - t0) / gens
    out["ga_cfg2_run_generation_ms"] = 1e3 * ga_run_time(G, pb, torch, G.GOAC_MIXED, 1024, gens)
    pb.close()
    return out


def ga_run_time(G, pb, torch, prec, P, gens):
    """Seconds per generation of goac_ga_run over `gens` generations (bf16 or FP64
    energies after each), after an untimed warm-up call."""
    pop = pb.init_occupations(P, seed=1)
    E = pb.energies(pop, prec)
    pb.ga_run(pop, E, seed=1, generation=0, generations=20, precision=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pb.ga_run(pop, E, seed=1, generation=20, generations=gens, precision=prec)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / gens


def large_cell(ctx, G, S, torch, stream):
    """16x16x8 rock-salt (N = 16384, M = 8192): 8192 chains x 1e5 trials, kT 0.5 ->
    0.01 eV over 100 blocks; mixed (FP32 field, batched FP64 anchors) against plain
    FP64. The field updates stream two rows of V_mm per update: HBM roofline."""
    cell = S.config5()
    V = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    del V
    torch.cuda.empty_cache()
    C, T, M = 8192, 100000, 8192
    occ0 = pb.init_occupations(C, seed=0)
    kT = np.geomspace(0.5, 0.01, 100)
    out = {}
    for prec, name in ((G.GOAC_MIXED, "mixed"), (G.GOAC_FP64, "fp64")):
        ch = G.Chains(pb, occ0, prec)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        ch.sweep(T, kT, T // 100, seed=0, reanchor_every=1024)
        b.record(stream)
        torch.cuda.synchronize()
        sec = a.elapsed_time(b) * 1e-3
        _, _, st = ch.export()
        upd = float(st["updates"].sum())
        row_bytes = upd * 2 * M * (4 if prec == G.GOAC_MIXED else 8)
        out["cfg5_%s_trials_per_s" % name] = C * T / sec
        out["cfg5_%s_sweep_s" % name] = sec
        out["cfg5_%s_field_update_GBs" % name] = row_bytes / sec / 1e9
        out["cfg5_%s_field_update_hbm_frac" % name] = row_bytes / sec / 1e9 / HBM_PEAK_GBS
        if prec == G.GOAC_MIXED:
            out["cfg5_accept_rate"] = float(st["accepts"].sum()) / (C * T)
            out["cfg5_field_updates_per_chain"] = upd / C
            out["cfg5_fallbacks_per_chain"] = float(st["fallbacks"].sum()) / C
            out["cfg5_anchors_per_chain"] = float(st["anchors"].sum()) / C
        ch.close()
        print("  [cfg5 %s] %.3f s" % (name, sec), file=sys.stderr, flush=True)
    out["cfg5_mixed_vs_fp64"] = out["cfg5_mixed_trials_per_s"] / out["cfg5_fp64_trials_per_s"]
    pb.close()
    return out


def batched_instances(ctx, G, S, torch, stream):
    """512 rock-salt/spinel instances (N log-uniform in [64, 2048]), 256 chains each,
    2e4 trials, kT 0.3 -> 0.01 eV over 20 blocks, one persistent launch whose
    workgroup size and chains per compute unit the autotuner picks (on a 2000-trial
    probe that leaves the chains unchanged, not timed)."""
    cells = S.config4()
    t0 = time.perf_counter()
    pbs = []
    for c in cells:
        V = ctx.build_ewald(c["lattice"], c["pos"])
        pbs.append(G.Problem(ctx, V, c["sublattice"], c["species"], c["charge"]))
    occs = [pb.init_occupations(256, seed=0, instance=i).reshape(-1) for i, pb in enumerate(pbs)]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    flat = torch.cat(occs)
    kT = np.geomspace(0.3, 0.01, 20)
    out = {}
    for prec, name in ((G.GOAC_MIXED, "mixed"), (G.GOAC_FP64, "fp64")):
        ch = G.Chains.batch(pbs, [256] * len(pbs), flat, prec)
        out["cfg4_%s_autotune" % name] = list(ch.autotune(2000, 0.3))
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        ch.sweep(20000, kT, 1000, seed=0, reanchor_every=1024)
        b.record(stream)
        torch.cuda.synchronize()
        sec = a.elapsed_time(b) * 1e-3
        out["cfg4_%s_trials_per_s" % name] = 512 * 256 * 20000 / sec
        out["cfg4_%s_sweep_s" % name] = sec
        ch.close()
        print("  [cfg4 %s] %.3f s" % (name, sec), file=sys.stderr, flush=True)
    out["cfg4_setup_s"] = t_setup
    for pb in pbs:
        pb.close()
    return out


K_E = 14.3996454784   # e / (4 pi eps0) in eV A (CODATA 2018)


def nacl_half(ctx, G, S, torch, stream):
    """Half-filled NaCl 3x3x3 (216 positions, 108 Na+ / 108 Cl- on one site class):
    4096 chains x 1e5 trials annealed kT 2 -> 0.02 eV (mixed). Reports the best
    Madelung constant found, M = -E r / ((N / 2) k_e) with r = 2.81 A, and the
    fraction of chains whose best energy is the rock-salt order's (FP64 energies)."""
    cell = S.nacl_half(3, 5.62)
    V = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    _, _, kind = S.rocksalt_conventional(3, 3, 3, 5.62)
    order = torch.from_numpy(np.where(kind == 0, 0, 1).astype(np.uint8)[None, :]).cuda()
    E_opt = float(pb.energies(order, G.GOAC_FP64).cpu()[0])
    C, T = 4096, 100000
    occ0 = pb.init_occupations(C, seed=0)
    ch = G.Chains(pb, occ0, G.GOAC_MIXED)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    ch.sweep(T, np.geomspace(2.0, 0.02, 100), T // 100, seed=0)
    b.record(stream)
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3
    _, best, st = ch.export()
    Eb = pb.energies(best, G.GOAC_FP64).cpu().numpy()
    n = len(cell["pos"])
    ch.close()
    pb.close()
    print("  [nacl] %.3f s" % sec, file=sys.stderr, flush=True)
    return {"nacl_trials_per_s": C * T / sec, "nacl_sweep_s": sec,
            "nacl_madelung_best": float(-Eb.min() * 2.81 / ((n / 2) * K_E)),
            "nacl_madelung_of_order": float(-E_opt * 2.81 / ((n / 2) * K_E)),
            "nacl_fraction_at_optimum": float(np.mean(np.abs(Eb - E_opt) <= 1e-6 * n))}


def gradient_descent(ctx, G, S, torch, stream):
    """Best-swap descent of 4096 random starts of the 4x4x4 rock-salt cell to local
    minima. A step scores all M (M - 1) / 2 pairs twice (lowest dE, then the first
    pair within the window), reading the upper triangle of the FP64 V_mm each time."""
    cell = S.config2()
    V = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    P, M = 4096, 256
    occ = pb.init_occupations(P, seed=0)
    pb.gd_run(occ.clone(), max_steps=2)                   # warm-up
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    occ, steps, E = pb.gd_run(occ)
    b.record(stream)
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3
    st = steps.cpu().numpy()
    pb.close()
    print("  [gd] %.3f s, %.1f swaps per start" % (sec, st.mean()), file=sys.stderr, flush=True)
    pairs = (st.sum() + P) * 2.0 * M * (M - 1) / 2      # the final, non-improving step scores once
    return {"gd_configs_per_s": P / sec, "gd_time_s": sec, "gd_swaps_per_start": float(st.mean()),
            "gd_swaps_per_s": float(st.sum()) / sec, "gd_pair_evals_per_s": pairs / sec}


def replica_exchange(ctx, G, S, torch, stream):
    """Replica-exchange MC on the 4x4x4 rock-salt cell: 256 groups of 16 replicas on
    a geometric ladder 0.02 -> 0.5 eV, 50 rounds of 2000 trials then one exchange
    step (mixed field). Timed three times from the same start: goac_remc_run
    launching the rounds on the stream and replaying them from a captured HIP graph
    (both after autotuning the launch), and the same rounds launched one call at a
    time from Python; all after an untimed warm-up round."""
    cell = S.config2()
    V = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    R, groups, rounds, per = 16, 256, 50, 2000
    C = R * groups
    ladder = np.geomspace(0.02, 0.5, R)
    occ0 = pb.init_occupations(C, seed=0)
    out = {}
    # untimed warm-up of both modes on a scratch chain set (first launches load code)
    w = G.Chains(pb, occ0, G.GOAC_MIXED)
    ws = torch.tensor(np.tile(np.arange(R, dtype=np.int32), groups), device=occ0.device)
    wa = torch.zeros(C, dtype=torch.uint8, device=occ0.device)
    wsum = torch.zeros(C, dtype=torch.int64, device=occ0.device)
    w.remc_run(R, ladder, per, 1, 0, 1, ws, graph=True)
    w.remc_run(R, ladder, per, 1, 1, 1, ws)
    w.sweep(per, ladder[:, None], per, seed=1)
    w.remc_exchange(R, ladder, 1, 1, ws, wa)
    wsum += wa
    float(wsum.sum().item())
    w.close()
    for mode in ("run", "graph", "eager"):
        ch = G.Chains(pb, occ0, G.GOAC_MIXED)
        ch.set_rows(np.tile(np.arange(R), groups))
        slot = torch.tensor(np.tile(np.arange(R, dtype=np.int32), groups), device=occ0.device)
        acc = torch.zeros(C, dtype=torch.uint8, device=occ0.device)
        acc_sum = torch.zeros(C, dtype=torch.int64, device=occ0.device)
        if mode != "eager":
            out["remc_autotune"] = list(ch.autotune(per, float(ladder[0])))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode != "eager":
            ch.remc_run(R, ladder, per, rounds, 0, 1, slot, graph=(mode == "graph"))
        else:
            for x in range(rounds):
                ch.sweep(per, ladder[:, None], per, seed=1)
                ch.remc_exchange(R, ladder, x, 1, slot, acc)
                acc_sum += acc
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        _, _, st = ch.export()
        ch.close()
        print("  [remc %s] %.3f s" % (mode, sec), file=sys.stderr, flush=True)
        out["remc_%s_trials_per_s" % mode] = C * rounds * per / sec
        out["remc_%s_time_s" % mode] = sec
        if mode == "eager":
            attempts = groups * sum(len(range(x % 2, R - 1, 2)) for x in range(rounds))
            out["remc_exchange_accept_rate"] = float(acc_sum.sum().item()) / attempts
            out["remc_trial_accept_rate"] = float(st["accepts"].sum()) / (C * rounds * per)
            out["remc_best_E_min"] = float(st["best_E"].min())
    out["remc_trials_per_s"] = out["remc_run_trials_per_s"]
    # short rounds (64 trials), where launching is a large part of a round: the
    # captured graph against the same rounds launched one call at a time
    short, srounds = 64, 200
    for mode in ("run", "graph", "eager"):
        ch = G.Chains(pb, occ0, G.GOAC_MIXED)
        ch.set_rows(np.tile(np.arange(R), groups))
        slot = torch.tensor(np.tile(np.arange(R, dtype=np.int32), groups), device=occ0.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode != "eager":
            ch.remc_run(R, ladder, short, srounds, 0, 1, slot, graph=(mode == "graph"))
        else:
            for x in range(srounds):
                ch.sweep(short, ladder[:, None], short, seed=1)
                ch.remc_exchange(R, ladder, x, 1, slot)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ch.close()
        out["remc_short_%s_rounds_per_s" % mode] = srounds / sec
    print("  [remc short] run %.0f, graph %.0f, eager %.0f rounds/s" % (
        out["remc_short_run_rounds_per_s"], out["remc_short_graph_rounds_per_s"], out["remc_short_eager_rounds_per_s"]),
        file=sys.stderr, flush=True)
    # the same rounds with the plain FP64 field (the hot replicas accept about
    # 40% of their trials, so the mixed field's in-kernel re-anchors recur there)
    ch = G.Chains(pb, occ0, G.GOAC_FP64)
    slot = torch.tensor(np.tile(np.arange(R, dtype=np.int32), groups), device=occ0.device)
    ch.autotune(per, float(ladder[0]))
    ch.remc_run(R, ladder, per, 1, 0, 1, slot.clone())          # warm-up on a copy of the slots
    ch.close()
    ch = G.Chains(pb, occ0, G.GOAC_FP64)
    ch.autotune(per, float(ladder[0]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.remc_run(R, ladder, per, rounds, 0, 1, slot)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ch.close()
    print("  [remc run fp64] %.3f s" % sec, file=sys.stderr, flush=True)
    out["remc_fp64_run_trials_per_s"] = C * rounds * per / sec
    out["remc_mixed_vs_fp64"] = out["remc_run_trials_per_s"] / out["remc_fp64_run_trials_per_s"]
    pb.close()
    return out


def hybrid(ctx, G, S, torch, stream):
    """REMC + GA hybrid on the 4x4x4 rock-salt cell: 256 groups of 16 replicas
    (ladder 0.02 -> 0.5 eV, mixed field) and a population of 1024; 5 rounds of
    (5 exchange steps after 1000 trials each, 10 GA generations with bf16
    energies, hand-over of the 8 best), after an untimed warm-up round."""
    cell = S.config2()
    V = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    R, groups, P, rounds = 16, 256, 1024, 5
    ladder = np.geomspace(0.02, 0.5, R)
    ch = G.Chains(pb, pb.init_occupations(R * groups, seed=0), G.GOAC_MIXED)
    slot = torch.tensor(np.tile(np.arange(R, dtype=np.int32), groups), device="cuda")
    pop = pb.init_occupations(P, seed=0, chain_base=1 << 20)
    # untimed warm-up round on copies (first launches load code)
    w = G.Chains(pb, pb.init_occupations(R * groups, seed=0), G.GOAC_MIXED)
    E = w.hybrid_round(slot.clone(), pop.clone(), R, ladder, trials=1000, exchanges=5, generations=10, seed=0,
                       round=0, n_elite=8, p_mut=0.2, inject=8, precision=G.GOAC_MIXED)
    float(E.min().item())
    w.close()
    best = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(rounds):
        E = ch.hybrid_round(slot, pop, R, ladder, trials=1000, exchanges=5, generations=10, seed=0, round=r,
                            n_elite=8, p_mut=0.2, inject=8, precision=G.GOAC_MIXED)
        best.append(float(E.min().item()))
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ch.close()
    pb.close()
    print("  [hybrid] %.3f s" % sec, file=sys.stderr, flush=True)
    trials = R * groups * 5 * 1000 * rounds
    return {"hybrid_round_ms": 1e3 * sec / rounds, "hybrid_trials_per_s": trials / sec,
            "hybrid_best_E_per_round": best}


def cpu_baseline(S):
    """The FP64 oracle (unchanged) on the host cores: one full step of the same
    workload (Ewald matrix, 4096 chains x 1e5 trials, energies of the bests, a
    GA generation, top-64), OpenMP over rows, chains and configurations."""
    import oracle as O
    cell = S.config2()
    nthreads = O.num_threads()
    t0 = time.perf_counter()
    V = O.cell_matrix(cell)
    occ0 = O.init_occupations(cell, CHAINS, seed=0)
    st = O.MCState(occ0)
    O.mc_run(V, cell, st, seed=0, n_trials=TRIALS, kT=np.geomspace(0.5, 0.01, BLOCKS), block_len=BLOCK_LEN)
    E = O.energies(V, st.best_occ, cell["charge"])
    O.ga_generation(cell, st.best_occ, E, seed=0, g=0, n_elite=8, p_mut=0.2)
    O.topk(V, st.best_occ, cell["charge"], 64)
    dt = time.perf_counter() - t0
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": CHAINS * TRIALS / dt, "unit": "swap-trials/s", "cores": nthreads, "kind": "oracle",
            "sample": "one full step of the workload (4096 chains x 1e5 trials plus Ewald, energies, GA, "
                      "top-64) in %.1f s" % dt, "cpu": model}


if __name__ == "__main__":
    main()
