"""Benchmark of the Coulomb cluster-expansion hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic input, the
16x16x8 rock-salt supercell (N = 16384: 8192 O2- fixed and 8192 cation positions
of Li+/Na+/Ni2+/Co3+/Mn4+/Ti4+ in charge-neutral proportions):
  1. FP64 Ewald pair matrix (real-space erfc + reciprocal sum on matrix cores)
  2. problem derivation (mobile block in FP64/FP32/bf16 hi+lo, fixed-ion field)
  3. 8192 random starts, 8192 chains
  4. 8192 chains x 1e5 swap trials, kT 0.5 -> 0.01 eV geometric over 100 blocks
     of 1000 trials; FP32 field with batched FP64 re-anchoring after 1024 field
     updates (between chunks of 8192 trials)
  5. a GA population of 512 (random starts), 100 generations, each followed by
     the children's energies on the bf16 hi+lo matrix-core product
  6. FP64 top-64 of the GA population and the 8192 chain bests
value = swap trials per second over whole steps (the cell's positions and
composition are host inputs of 0.4 MB; everything else lives on the GPU).

Also measured, as extra keys: the same step in plain FP64 (FP64 field and
energies, default launches); energies per second at configs 1, 3 and 5 (mixed
against FP64); the 4x4x4 cell's 4096-chain step; config 1's 64-chain run; the
512 uneven instances in one persistent autotuned launch against per-instance
FP64 launches; the NaCl, gradient-descent, replica-exchange and hybrid legs.
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
C5, T5, BLOCKS, BLOCK_LEN = 8192, 100000, 100, 1000
P5, GENS5, TOPK = 512, 100, 64
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit or FP64 VALU lane operations per second
ALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
BF16_PEAK = 2.5e15
FP64_PEAK = 78.6e12
# HBM bytes per k_mc<mixed, 256> launch of the step's sweep from FETCH_SIZE and
# WRITE_SIZE, each scaled by the same counter's reading for a plain copy of known
# size; valid only for the kernel sources they were taken on
# field updates between FP64 re-anchors of the 16x16x8 sweep: of 1024, 2048, 4096
# and 8192 the fastest sweep (fewer batched anchors against more exact fallbacks;
# the decisions, hence the trajectories, are the same for any interval)
REANCHOR5 = 2048
MC_TRAFFIC = {"bytes": 3.7804e11,
              "sources": ("paper_2409_08808_amd/csrc/mc.hip", "paper_2409_08808_amd/csrc/common.h"),
              "sha256": "5e1d376904bf237eb4dd30eedd326f699704660735d45650b20a655691edf7cb"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the step")
    ap.add_argument("--calibrate-copy", action="store_true", help="also run a copy kernel of known size")
    ap.add_argument("--ga-generations", type=int, default=200)
    ap.add_argument("--only", default="", help="comma list of extra legs: fp64, energies, cfg1, cfg2, ga, cfg4, "
                                                "nacl, gd, remc, hybrid (the step itself always runs)")
    ap.add_argument("--legs-only", action="store_true",
                    help="run the --only legs without the step and print their figures (for profiling)")
    return ap.parse_args()


def measured_traffic(entry):
    """The counter-based traffic figure, or None once its kernel sources changed."""
    import hashlib
    if entry["bytes"] is None:
        return None
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


def pop_flops(P, M):
    """Algorithmic flops of the energies of P rows (Eq. 2's quadratic form): 2 M^2
    + 4 M per row (the product with V_mm, the row dot, the linear term)."""
    return P * (2.0 * M * M + 4.0 * M)


def ev(torch):
    return torch.cuda.Event(enable_timing=True)


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
    cell = S.config5()
    kT = np.geomspace(0.5, 0.01, BLOCKS)
    M = int((cell["sublattice"] >= 0).sum())

    def step(seed, prec, timing=False, host_stats=False):
        """One pass of the path; prec GOAC_MIXED (FP32 field, bf16 hi+lo energies) or
        GOAC_FP64 (FP64 field and energies, the size rule's launch)."""
        V = ctx.build_ewald(cell["lattice"], cell["pos"])
        pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
        del V
        occ0 = pb.init_occupations(C5, seed=seed)
        ch = G.Chains(pb, occ0, prec)
        del occ0
        ch.sweep(T5, kT, BLOCK_LEN, seed=seed, reanchor_every=REANCHOR5, timing=timing)
        pop = pb.init_occupations(P5, seed=seed, chain_base=1 << 20)
        E = pb.energies(pop, prec)
        pb.ga_run(pop, E, seed=seed, generation=0, generations=GENS5, n_elite=8, p_mut=0.2, precision=prec)
        _, best, stats = ch.export(host_stats=host_stats, occ=False)
        cand = torch.cat([pop, best])
        idx, Ek = pb.topk(cand, TOPK)
        tm = ch.timing() if timing else None
        ch.close()
        pb.close()
        return stats, tm, Ek

    def timed(prec, steps, warmup):
        for w in range(warmup):
            step(1000 + w, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, tms, Ek = None, [], None
        for k in range(steps):
            stats, tm, Ek = step(k, prec, timing=True, host_stats=(k == steps - 1))
            tms.append(tm)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        print("  [step %s] %d steps in %.3f s" % ("mixed" if prec else "fp64", steps, wall), file=sys.stderr,
              flush=True)
        return wall, tms, stats, Ek

    def run_legs(result, legs):
        if "energies" in legs:
            result.update(energies_legs(ctx, G, S, torch, stream))
        if "cfg1" in legs:
            result.update(config1(ctx, G, S, torch, stream))
        if "cfg2" in legs:
            result.update(config2_step(ctx, G, S, torch, stream, max(2, args.steps)))
        if "ga" in legs:
            result.update(ga_energies(ctx, G, S, torch, stream, args.ga_generations))
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

    if args.legs_only:
        legs = set(args.only.split(",")) - {""}
        out = {"legs_only": sorted(legs)}
        run_legs(out, legs)
        print(json.dumps(out), flush=True)
        return
    wall, tms, stats, Ek = timed(G.GOAC_MIXED, args.steps, args.warmup)
    value = float(C5) * T5 * args.steps / wall
    upd = float(stats["updates"].sum())
    mc_s = np.mean([t[0] for t in tms])
    anchor_s = np.mean([t[1] for t in tms])
    launches = tms[-1][2]
    row_bytes = upd * 2.0 * M * 4.0            # two FP32 rows of V_mm per field update
    achieved = row_bytes / mc_s / 1e9
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
        "dtype": "f32+f64+bf16",
        "data": "synthetic",
        "config": {"workload": ("rock-salt 16x16x8 (N=16384, M=8192; Li/Na/Ni/Co/Mn/Ti, charge-neutral units), "
                                "Ewald + problem, 8192 chains x 1e5 trials, kT 0.5->0.01 eV over 100 blocks, FP32 "
                                "field + batched FP64 re-anchor/%d, GA P=512 x 100 generations with bf16 hi+lo "
                                "energies, FP64 top-64 of the GA population and the chain bests") % REANCHOR5,
                   "chains": C5, "trials_per_chain": T5, "ga_population": P5, "ga_generations": GENS5,
                   "topk": TOPK, "parallelism": "chains per workgroup, populations on matrix cores"},
        "mc_sweep_kernel_s": mc_s,
        "mc_anchor_s": anchor_s,
        "mc_launches_per_sweep": launches,
        "mc_trials_per_s_kernel": C5 * T5 / mc_s,
        "accept_rate": float(stats["accepts"].sum()) / (C5 * T5),
        "field_updates_per_chain": upd / C5,
        "fallbacks_per_chain": float(stats["fallbacks"].sum()) / C5,
        "anchors_per_chain": float(stats["anchors"].sum()) / C5,
        "best_E_topk_min": float(Ek.min().item()),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(MC_TRAFFIC),
                     "kernel": "k_mc<mixed,256>", "launches": launches,
                     "bytes_per_launch": row_bytes / launches, "launch_s": mc_s / launches},
    }
    legs = set(args.only.split(",")) - {""}
    if not legs and not args.no_extras:
        legs = {"fp64", "energies", "cfg1", "cfg2", "ga", "cfg4", "nacl", "gd", "remc", "hybrid"}
    if "fp64" in legs:
        n64 = max(1, min(2, args.steps))
        w64, tm64, s64, _ = timed(G.GOAC_FP64, n64, 1)
        result["plain_fp64_trials_per_s"] = float(C5) * T5 * n64 / w64
        result["plain_fp64_ms_per_step"] = 1e3 * w64 / n64
        result["plain_fp64_sweep_kernel_s"] = np.mean([t[0] for t in tm64])
        upd64 = float(s64["updates"].sum())
        result["plain_fp64_field_update_GBs"] = upd64 * 2.0 * M * 8.0 / result["plain_fp64_sweep_kernel_s"] / 1e9
        result["mixed_vs_fp64"] = result["value"] / result["plain_fp64_trials_per_s"]
        result["mixed_vs_fp64_sweep"] = result["plain_fp64_sweep_kernel_s"] / mc_s
    run_legs(result, legs)
    # context for the roofline: a plain 256 MiB device-to-device copy (read plus
    # write bytes over its time, HIP events on the stream, best of five)
    xc = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
    yc = torch.empty_like(xc)
    yc.copy_(xc)
    best = None
    for _ in range(5):
        a, b = ev(torch), ev(torch)
        a.record(stream)
        yc.copy_(xc)
        b.record(stream)
        b.synchronize()
        t = a.elapsed_time(b) * 1e-3
        best = t if best is None else min(best, t)
    result["device_copy_GBs"] = 2 * xc.numel() / best / 1e9
    del xc, yc
    if args.calibrate_copy:
        x = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = 2 * x.numel()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(S, kT)
    print(json.dumps(result), flush=True)


def timed_calls(torch, stream, fn, reps):
    """Mean device seconds of fn() over reps calls (HIP events on the stream)."""
    fn()
    a, b = ev(torch), ev(torch)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) * 1e-3 / reps


def energies_legs(ctx, G, S, torch, stream):
    """Population energies per second, mixed (bf16 hi+lo, FP32 accumulation) and
    FP64, on the 16x16x8 cell with the GA's 512 rows and on the 8x8x8 cell with
    1024 rows (calls back to back, each with its row check)."""
    out = {}
    for name, cfg, P in (("cfg5", S.config5, 512), ("cfg3", S.config3, 1024)):
        cell = cfg()
        V = ctx.build_ewald(cell["lattice"], cell["pos"])
        pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
        del V
        M = int((cell["sublattice"] >= 0).sum())
        pop = pb.init_occupations(P, seed=0)
        E = torch.empty(P, dtype=torch.float64, device=pop.device)
        for prec, pn in ((G.GOAC_MIXED, "mixed"), (G.GOAC_FP64, "fp64")):
            sec = timed_calls(torch, stream, lambda: pb.energies(pop, prec, out=E), 20)
            out["%s_%s_energies_per_s" % (name, pn)] = P / sec
            out["%s_%s_energy_call_us" % (name, pn)] = 1e6 * sec
            peak = BF16_PEAK if prec == G.GOAC_MIXED else FP64_PEAK
            out["%s_%s_energy_frac_of_peak" % (name, pn)] = pop_flops(P, M) / sec / peak
        out["%s_energies_mixed_vs_fp64" % name] = (out["%s_mixed_energies_per_s" % name] /
                                                   out["%s_fp64_energies_per_s" % name])
        pb.close()
        print("  [energies %s] mixed %.1f us, fp64 %.1f us" % (name, out["%s_mixed_energy_call_us" % name],
                                                              out["%s_fp64_energy_call_us" % name]),
              file=sys.stderr, flush=True)
    out["energies_per_s"] = out["cfg5_mixed_energies_per_s"]
    return out


def config1(ctx, G, S, torch, stream):
    """Config 1 (2x2x1 rock-salt, 16 Li+/M3+ positions, alpha = 5/L, r_c = 10 A,
    |n| <= 8): energies of all 12870 occupations, and 64 chains x 1e4 trials at kT
    = 0.05 eV, seed 0, mixed against FP64."""
    cell = S.config1()
    e = cell["ewald"]
    V = ctx.build_ewald(cell["lattice"], cell["pos"], e["alpha"], e["rcut"], e["kmax"])
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    occ = torch.from_numpy(S.config1_exhaustive_occupations(cell)).cuda()
    E = torch.empty(len(occ), dtype=torch.float64, device=occ.device)
    out = {}
    for prec, pn in ((G.GOAC_MIXED, "mixed"), (G.GOAC_FP64, "fp64")):
        sec = timed_calls(torch, stream, lambda: pb.energies(occ, prec, out=E), 20)
        out["cfg1_%s_energies_per_s" % pn] = len(occ) / sec
        occ0 = pb.init_occupations(64, seed=0)
        ch = G.Chains(pb, occ0, prec)
        ch.sweep(10000, [0.05], seed=1)
        ch.timing()
        ch.sweep(10000, [0.05], seed=0, timing=True)
        mc, _, _ = ch.timing()
        out["cfg1_%s_trials_per_s" % pn] = 64 * 10000 / mc
        ch.close()
    pb.close()
    return out


def config2_step(ctx, G, S, torch, stream, steps):
    """The 4x4x4 rock-salt cell (N = 512; Li/Ni/Co/Mn 128/32/64/32): Ewald, problem,
    4096 chains x 1e5 trials (kT 0.5 -> 0.01 eV, FP32 field + FP64 re-anchor every
    1024 updates inside the kernel), energies of the bests, one GA generation and
    the FP64 top-64; mixed against FP64."""
    cell = S.config2()
    kT = np.geomspace(0.5, 0.01, BLOCKS)
    out = {}

    def one(seed, prec):
        V = ctx.build_ewald(cell["lattice"], cell["pos"])
        pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
        ch = G.Chains(pb, pb.init_occupations(4096, seed=seed), prec)
        ch.sweep(100000, kT, BLOCK_LEN, seed=seed, reanchor_every=1024, timing=True)
        _, best, st = ch.export(host_stats=False, occ=False)
        E = pb.energies(best, prec)
        pb.ga_generation(best, E, seed=seed, generation=0, n_elite=8, p_mut=0.2)
        pb.topk(best, 64)
        tm = ch.timing()
        ch.close()
        pb.close()
        return tm

    for prec, pn in ((G.GOAC_MIXED, "mixed"), (G.GOAC_FP64, "fp64")):
        one(999, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tms = [one(k, prec) for k in range(steps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out["cfg2_%s_trials_per_s" % pn] = 4096 * 100000.0 * steps / wall
        out["cfg2_%s_ms_per_step" % pn] = 1e3 * wall / steps
        out["cfg2_%s_sweep_ms" % pn] = 1e3 * np.mean([t[0] for t in tms])
    out["cfg2_mixed_vs_fp64"] = out["cfg2_mixed_trials_per_s"] / out["cfg2_fp64_trials_per_s"]
    out["cfg2_mixed_vs_fp64_sweep"] = out["cfg2_fp64_sweep_ms"] / out["cfg2_mixed_sweep_ms"]
    print("  [cfg2] mixed %.2f ms, fp64 %.2f ms per step" % (out["cfg2_mixed_ms_per_step"],
                                                            out["cfg2_fp64_ms_per_step"]), file=sys.stderr, flush=True)
    return out


def ga_energies(ctx, G, S, torch, stream, generations):
    """GA workload of the 8x8x8 cell (N = 4096, P = 1024): generations of
    goac_ga_run (each followed by the children's energies, mixed or FP64), and on
    the 4x4x4 cell the same generations called one by one from Python against
    goac_ga_run (graph replays)."""
    out = {}
    cell = S.config3()
    V = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    del V
    pop = pb.init_occupations(1024, seed=0)
    out["ga_mixed_tile_autotuned"] = pb.energies_autotune(pop)
    out["ga_mixed_generation_ms"] = 1e3 * ga_run_time(G, pb, torch, G.GOAC_MIXED, 1024, generations)
    out["ga_fp64_generation_ms"] = 1e3 * ga_run_time(G, pb, torch, G.GOAC_FP64, 1024, max(10, generations // 10))
    pb.close()
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
    print("  [ga] cfg3 %.3f ms (mixed), %.3f ms (fp64) per generation" % (out["ga_mixed_generation_ms"],
                                                                         out["ga_fp64_generation_ms"]),
          file=sys.stderr, flush=True)
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


def batched_instances(ctx, G, S, torch, stream):
    """512 rock-salt/spinel instances (N log-uniform in [64, 2048]), 256 chains each,
    2e4 trials, kT 0.3 -> 0.01 eV over 20 blocks. Mixed+batched: one persistent
    launch of every chain, workgroup size and chains per compute unit from the
    autotuner (on a 2000-trial probe that leaves the chains unchanged, not timed).
    Batched FP64: the same launch with the FP64 field. Plain FP64: one chain set and
    one launch per instance with the size rule's configuration, no autotuning."""
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
    total = 512 * 256 * 20000
    out = {}
    for prec, name in ((G.GOAC_MIXED, "mixed"), (G.GOAC_FP64, "fp64")):
        ch = G.Chains.batch(pbs, [256] * len(pbs), flat, prec)
        out["cfg4_%s_autotune" % name] = list(ch.autotune(2000, 0.3))
        ch.sweep(20000, kT, 1000, seed=0, reanchor_every=1024, timing=True)
        sec = ch.timing()[0]
        out["cfg4_%s_trials_per_s" % name] = total / sec
        out["cfg4_%s_sweep_s" % name] = sec
        ch.close()
        print("  [cfg4 %s] %.3f s" % (name, sec), file=sys.stderr, flush=True)
    # plain FP64: per-instance chain sets and launches (events around all of them)
    sets = [G.Chains(pb, occs[i].view(256, -1), G.GOAC_FP64, instance=i) for i, pb in enumerate(pbs)]
    a, b = ev(torch), ev(torch)
    torch.cuda.synchronize()
    a.record(stream)
    for ch in sets:
        ch.sweep(20000, kT, 1000, seed=0, reanchor_every=1024)
    b.record(stream)
    b.synchronize()
    sec = a.elapsed_time(b) * 1e-3
    for ch in sets:
        ch.close()
    out["cfg4_plain_fp64_trials_per_s"] = total / sec
    out["cfg4_plain_fp64_sweep_s"] = sec
    out["cfg4_mixed_vs_plain_fp64"] = out["cfg4_mixed_trials_per_s"] / out["cfg4_plain_fp64_trials_per_s"]
    out["cfg4_setup_s"] = t_setup
    print("  [cfg4 plain fp64] %.3f s" % sec, file=sys.stderr, flush=True)
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


def cpu_baseline(S, kT):
    """The FP64 oracle (unchanged) on the host cores, on a bounded sample of the
    step: 640 of its 8192 chains with the full 1e5 trials and the same temperature
    schedule (about 10 s on 16 cores), OpenMP over chains. The oracle's own pair matrix of the cell (from one
    row relabelled by translation) is built first and timed apart; the rate counts
    the Monte Carlo alone and is the per-trial rate of the whole step's sweep."""
    import oracle as O
    cell = S.config5()
    nthreads = O.num_threads()
    t0 = time.perf_counter()
    V = O.grid_matrix(cell)
    t_v = time.perf_counter() - t0
    C = 640
    occ0 = O.init_occupations(cell, C, seed=0)
    st = O.MCState(occ0)
    t0 = time.perf_counter()
    O.mc_run(V, cell, st, seed=0, n_trials=T5, kT=kT, block_len=BLOCK_LEN)
    dt = time.perf_counter() - t0
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": C * T5 / dt, "unit": "swap-trials/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d of the step's 8192 chains x 1e5 trials (same schedule) in %.1f s, extrapolated per trial; "
                      "the oracle's pair matrix of the cell took %.1f s more, not counted" % (C, dt, t_v),
            "cpu": model}


if __name__ == "__main__":
    main()
