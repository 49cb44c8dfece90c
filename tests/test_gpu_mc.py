"""GPU parity of the swap Monte Carlo (FP64 and mixed), replica exchange and
the GA generation against the FP64 oracle.

Bar: trajectories (the per-trial hash summed over trials), final occupations and
accept counts bit-exact; tracked energies within 1e-6 eV per site (FP64) and
1e-4 eV per site (mixed); GA children bit-exact given identical energies."""
import numpy as np
import pytest
import torch

import oracle as O
import supercells as S
from gpu_common import (degenerate_sublattice_cell, long_window_cell, many_species_cell, near_copies,
                        two_sublattice_cell)

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_2409_08808_amd")
TOL = {0: 1e-6, 1: 1e-4}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G.Context(0)


@pytest.fixture(scope="module")
def cfg1():
    c = S.config1()
    return c, O.cell_matrix(c)


@pytest.fixture(scope="module")
def cfg2():
    c = S.config2()
    return c, O.cell_matrix(c)


def _compare(cell, stats, occ_g, best_g, st, prec, V):
    n = len(cell["pos"])
    assert np.array_equal(stats["t"], st.field("t"))
    assert np.array_equal(stats["hash"], st.field("hash")), "trajectory hash differs"
    assert np.array_equal(occ_g, st.occ), "final occupations differ"
    assert np.array_equal(stats["accepts"], st.field("accepts"))
    assert np.array_equal(stats["updates"], st.field("updates"))
    assert np.all(stats["status"] == 0)
    assert np.abs(stats["E"] - st.field("E")).max() / n <= TOL[prec]
    assert np.abs(stats["best_E"] - st.field("best_E")).max() / n <= TOL[prec]
    # the oracle's energy of the GPU's best occupation (ties among degenerate states)
    Eb = O.energies(V, best_g, cell["charge"])
    assert np.abs(Eb - stats["best_E"]).max() / n <= TOL[prec]


def _run_gpu(ctx, cell, V, occ0, prec, n_trials, kT, block_len, seed, reanchor=1024, variant=0, sweeps=1,
             chain_base=0):
    pb = G.Problem(ctx, torch.from_numpy(V) if isinstance(V, np.ndarray) else V, cell["sublattice"],
                   cell["species"], cell["charge"])
    ch = G.Chains(pb, torch.from_numpy(occ0), prec, chain_base=chain_base)
    per = n_trials // sweeps
    for _ in range(sweeps):
        ch.sweep(per, kT, block_len, seed=seed, reanchor_every=reanchor, trace=True, variant=variant)
    occ, best, stats = ch.export()
    return occ.cpu().numpy(), best.cpu().numpy(), stats


def _run_oracle(cell, V, occ0, n_trials, kT, block_len, seed, chain_base=0):
    st = O.MCState(occ0)
    O.mc_run(V, cell, st, seed=seed, n_trials=n_trials, kT=kT, block_len=block_len, chain_base=chain_base)
    return st


@pytest.mark.parametrize("prec", [0, 1])
def test_mc_config1(ctx, cfg1, prec):
    """Config 1 as stated: 64 chains x 1e4 trials, kT = 0.05 eV, seed 0."""
    cell, V = cfg1
    occ0 = O.init_occupations(cell, 64, seed=0)
    st = _run_oracle(cell, V, occ0, 10000, [0.05], 10 ** 9, 0)
    occ, best, stats = _run_gpu(ctx, cell, V, occ0, prec, 10000, [0.05], 10 ** 9, 0, reanchor=256)
    _compare(cell, stats, occ, best, st, prec, V)


def test_mc_config1_end_to_end(ctx, cfg1):
    # the GPU's own pair matrix (differs from the oracle's in the last bits)
    cell, V = cfg1
    e = cell["ewald"]
    Vg = ctx.build_ewald(cell["lattice"], cell["pos"], e["alpha"], e["rcut"], e["kmax"])
    occ0 = O.init_occupations(cell, 64, seed=0)
    st = _run_oracle(cell, V, occ0, 10000, [0.05], 10 ** 9, 0)
    occ, best, stats = _run_gpu(ctx, cell, Vg, occ0, 1, 10000, [0.05], 10 ** 9, 0)
    _compare(cell, stats, occ, best, st, 1, V)


@pytest.mark.parametrize("prec,reanchor,variant", [(0, 1024, 0), (1, 1024, 0), (1, 64, 0), (0, 1024, 256),
                                                   (1, 128, 256)])
def test_mc_config2_annealed(ctx, cfg2, prec, reanchor, variant):
    """Config 2 cell, annealed kT 0.5 -> 0.01 eV (geometric, 20 blocks of 1000)."""
    cell, V = cfg2
    kT = np.geomspace(0.5, 0.01, 20)
    occ0 = O.init_occupations(cell, 48, seed=7)
    st = _run_oracle(cell, V, occ0, 20000, kT, 1000, 7)
    occ, best, stats = _run_gpu(ctx, cell, V, occ0, prec, 20000, kT, 1000, 7, reanchor=reanchor, variant=variant)
    _compare(cell, stats, occ, best, st, prec, V)
    if prec == 1:
        # one FP64 anchor after every reanchor field updates
        assert np.array_equal(stats["anchors"], stats["updates"] // reanchor)


@pytest.mark.parametrize("which,kT", [("two", 5.0), ("two", 0.3), ("many", 0.1)])
@pytest.mark.parametrize("prec,variant", [(0, 64), (0, 256), (1, 64), (1, 256)])
def test_mc_frequent_accepts(ctx, which, kT, prec, variant):
    """Windows with many accepted trials: two mobile site classes at high kT, and a
    class whose species all carry the same charge (every swap has dE = 0 and is
    accepted). Multi-wave chains (256 lanes) go on within a window after each
    accepted swap, rescoring the later trials; one-wave chains start a new window.
    Both must follow the sequential chain exactly."""
    cell = two_sublattice_cell() if which == "two" else many_species_cell()
    V = O.cell_matrix(cell)
    occ0 = O.init_occupations(cell, 24, seed=5)
    st = _run_oracle(cell, V, occ0, 3000, [kT], 10 ** 9, 5)
    occ, best, stats = _run_gpu(ctx, cell, V, occ0, prec, 3000, [kT], 10 ** 9, 5, reanchor=64, variant=variant)
    _compare(cell, stats, occ, best, st, prec, V)
    assert stats["accepts"].sum() > 0.01 * 24 * 3000


@pytest.mark.parametrize("block_len", [7, 200])
@pytest.mark.parametrize("prec,variant", [(0, 64), (1, 64), (1, 256)])
def test_mc_degenerate_cell_and_temperature_extremes(ctx, prec, variant, block_len):
    """Edge cases against the oracle: a sublattice without a valid swap partner
    (its trials are rejected without a pick), temperatures below the FP32 filter's
    range (every trial is decided by the exact rule) and far above the energy
    scale, blocks shorter than a window (each lane finds its own temperature), and
    a trial count that ends inside a window. Near zero temperature a trial is
    accepted iff dE <= 0, and swaps that change nothing physically have dE = 0 up
    to the rounding of the field, whose summation order differs between the two
    sides; a symmetric integer pair matrix makes every field and dE exact, so the
    decisions are the same numbers on both sides."""
    cell = degenerate_sublattice_cell()
    n = len(cell["pos"])
    A = np.random.default_rng(3).integers(-4, 5, size=(n, n)).astype(np.float64)
    V = np.triu(A) + np.triu(A, 1).T
    kT = [1e-200, 1e6, 0.05, 1e-200, 2.0]
    occ0 = O.init_occupations(cell, 24, seed=9)
    st = _run_oracle(cell, V, occ0, 1001, kT, block_len, 9)
    occ, best, stats = _run_gpu(ctx, cell, V, occ0, prec, 1001, kT, block_len, 9, reanchor=32, variant=variant)
    _compare(cell, stats, occ, best, st, prec, V)
    assert np.all(stats["t"] == 1001)
    sub = cell["sublattice"]
    assert np.array_equal(occ[:, sub == 0], occ0[:, sub == 0])     # nothing moves there


@pytest.mark.parametrize("prec", [0, 1])
def test_mc_resume(ctx, cfg2, prec):
    cell, V = cfg2
    kT = np.geomspace(0.5, 0.05, 6)
    occ0 = O.init_occupations(cell, 16, seed=3)
    st = _run_oracle(cell, V, occ0, 6000, kT, 1000, 3)
    occ, best, stats = _run_gpu(ctx, cell, V, occ0, prec, 6000, kT, 1000, 3, sweeps=3)
    _compare(cell, stats, occ, best, st, prec, V)


@pytest.mark.parametrize("prec", [0, 1])
def test_mc_nacl_half_reaches_madelung(ctx, prec):
    """The half-filled NaCl workload (Results, "Atomistic Configurations in NaCl"):
    216 positions of one site class holding 108 Na+ and 108 Cl-, 256 chains x 1e5
    trials annealed kT 2 -> 0.02 eV. Bit-exact against the oracle; no chain goes
    below the rock-salt order's energy (the Madelung energy, pinned in the oracle
    tests) and some chain reaches it (the oracle finds it in about one chain of
    eight with this schedule)."""
    cell = S.nacl_half(3, 5.62)
    V = O.cell_matrix(cell)
    n = len(cell["pos"])
    kT = np.geomspace(2.0, 0.02, 100)
    occ0 = O.init_occupations(cell, 256, seed=11)
    st = _run_oracle(cell, V, occ0, 100000, kT, 1000, 11)
    occ, best, stats = _run_gpu(ctx, cell, V, occ0, prec, 100000, kT, 1000, 11)
    _compare(cell, stats, occ, best, st, prec, V)
    _, _, kind = S.rocksalt_conventional(3, 3, 3, 5.62)
    E_opt = O.energy_q(V, np.where(kind == 0, 1.0, -1.0))
    assert stats["best_E"].min() >= E_opt - TOL[prec] * n
    assert np.abs(stats["best_E"].min() - E_opt) <= TOL[prec] * n


@pytest.mark.parametrize("prec", [0, 1])
def test_mc_two_sublattices_interleaved(ctx, prec):
    cell = two_sublattice_cell()
    perm = np.random.default_rng(2).permutation(len(cell["pos"]))
    cell = S.make_cell(cell["lattice"], cell["pos"][perm], cell["sublattice"][perm], cell["species"][perm],
                       cell["charge"], cell["names"])
    V = O.cell_matrix(cell)
    occ0 = O.init_occupations(cell, 24, seed=5)
    kT = np.geomspace(1.0, 0.05, 8)
    st = _run_oracle(cell, V, occ0, 8000, kT, 1000, 5, chain_base=100)
    occ, best, stats = _run_gpu(ctx, cell, V, occ0, prec, 8000, kT, 1000, 5, reanchor=200, chain_base=100)
    _compare(cell, stats, occ, best, st, prec, V)


def test_mc_config2_full_launch_sampled(ctx, cfg2):
    """The benchmark's launch: 4096 chains x 1e5 trials, kT 0.5 -> 0.01 eV over
    100 blocks of 1000, mixed precision, seed 0. Six chains are replayed by the
    oracle one by one."""
    cell, V = cfg2
    pb = G.Problem(ctx, torch.from_numpy(V), cell["sublattice"], cell["species"], cell["charge"])
    occ0 = pb.init_occupations(4096, seed=0)
    ch = G.Chains(pb, occ0, G.GOAC_MIXED)
    kT = np.geomspace(0.5, 0.01, 100)
    ch.sweep(100000, kT, 1000, seed=0, reanchor_every=1024, trace=True)
    occ, best, stats = ch.export()
    occ, best = occ.cpu().numpy(), best.cpu().numpy()
    occ0 = occ0.cpu().numpy()
    assert np.all(stats["t"] == 100000) and np.all(stats["status"] == 0)
    for c in (0, 1, 777, 2048, 3001, 4095):
        st = _run_oracle(cell, V, occ0[c:c + 1], 100000, kT, 1000, 0, chain_base=c)
        assert stats["hash"][c] == st.stats[0].hash
        assert np.array_equal(occ[c], st.occ[0])
        assert abs(stats["E"][c] - st.stats[0].E) / 512 <= TOL[1]
    # every chain: tracked energy against the FP64 energy of its final occupation
    Ef = pb.energies(torch.from_numpy(occ), G.GOAC_FP64).cpu().numpy()
    assert np.abs(Ef - stats["E"]).max() / 512 <= TOL[1]


def test_mc_config5_mixed_equals_fp64(ctx):
    """Config 5 cell (N = 16384, M = 8192): the mixed chain must retrace the FP64
    chain exactly, and the tracked energies must match a fresh FP64 evaluation."""
    cell = S.config5()
    Vg = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, Vg, cell["sublattice"], cell["species"], cell["charge"])
    del Vg
    torch.cuda.empty_cache()
    occ0 = pb.init_occupations(64, seed=0)
    kT = np.geomspace(0.5, 0.01, 10)
    res = {}
    for prec in (0, 1):
        ch = G.Chains(pb, occ0, prec)
        ch.sweep(3000, kT, 300, seed=0, reanchor_every=1024, trace=True)
        res[prec] = ch.export()
        ch.close()
    (o0, b0, s0), (o1, b1, s1) = res[0], res[1]
    assert np.array_equal(s0["hash"], s1["hash"]) and torch.equal(o0, o1)
    n = 16384
    assert np.abs(s0["E"] - s1["E"]).max() / n <= TOL[1]
    Ef = pb.energies(o0, G.GOAC_FP64).cpu().numpy()
    assert np.abs(Ef - s0["E"]).max() / n <= TOL[0]
    assert np.abs(Ef - s1["E"]).max() / n <= TOL[1]


@pytest.mark.parametrize("prec", [0, 1])
def test_mc_batch_uneven_instances(ctx, prec):
    """Several uneven rock-salt/spinel instances in one persistent launch; each
    instance checked against the oracle with its own instance id."""
    cells = S.config4(n_instances=10, seed=3, nmin=40, nmax=420)
    Vs = [O.cell_matrix(c) for c in cells]
    pbs = [G.Problem(ctx, torch.from_numpy(V), c["sublattice"], c["species"], c["charge"]) for c, V in zip(cells, Vs)]
    cpi = [5 + (i % 3) for i in range(len(cells))]
    occ0 = [O.init_occupations(c, k, seed=9, instance=i) for i, (c, k) in enumerate(zip(cells, cpi))]
    flat = np.concatenate([o.reshape(-1) for o in occ0])
    ch = G.Chains.batch(pbs, cpi, torch.from_numpy(flat), prec)
    kT = np.geomspace(0.3, 0.01, 4)
    ch.sweep(4000, kT, 1000, seed=9, reanchor_every=256, trace=True)
    occ, best, stats = ch.export()
    occ = occ.cpu().numpy()
    start = 0
    row = 0
    for i, (c, V) in enumerate(zip(cells, Vs)):
        n = len(c["pos"])
        st = O.MCState(occ0[i])
        O.mc_run(V, c, st, seed=9, n_trials=4000, kT=kT, block_len=1000, instance=i)
        k = cpi[i]
        got = occ[start:start + k * n].reshape(k, n)
        assert np.array_equal(got, st.occ)
        assert np.array_equal(stats["hash"][row:row + k], st.field("hash"))
        assert np.abs(stats["E"][row:row + k] - st.field("E")).max() / n <= TOL[prec]
        start += k * n
        row += k


def test_remc_exchange_bitexact(ctx, cfg1):
    cell, V = cfg1
    R = 4
    ladder = np.array([0.05, 0.1, 0.2, 0.4])
    pb = G.Problem(ctx, torch.from_numpy(V), cell["sublattice"], cell["species"], cell["charge"])
    occ0 = pb.init_occupations(16, seed=4)
    ch = G.Chains(pb, occ0, G.GOAC_FP64)
    ch.set_rows(np.tile(np.arange(R), 4))
    slot = torch.tensor(np.tile(np.arange(R, dtype=np.int32), 4), device="cuda")
    acc = torch.zeros(16, dtype=torch.uint8, device="cuda")
    ref_slot = np.tile(np.arange(R, dtype=np.int32), (4, 1))
    for x in range(6):
        ch.sweep(500, ladder[:, None], seed=4)
        _, _, stats = ch.export()
        ch.remc_exchange(R, ladder, x, 77, slot, acc)
        for g in range(4):
            ref_slot[g], _ = O.remc_exchange(ladder, stats["E"][g * R:(g + 1) * R], ref_slot[g], x, 77, group=g)
        assert np.array_equal(slot.view(4, R).cpu().numpy(), ref_slot)
    _, _, stats = ch.export()
    rows = stats["row"].reshape(4, R)
    for g in range(4):
        assert np.array_equal(ref_slot[g][rows[g]], np.arange(R))


@pytest.mark.parametrize("R", [2, 5, 130, 600])
def test_remc_exchange_ladders(ctx, cfg1, R):
    """Odd and long ladders (several pairs per thread at R = 600) against the
    oracle's exchange; a group whose slots repeat a chain is left unchanged while
    the other group goes on."""
    cell, V = cfg1
    groups = 2
    ladder = np.geomspace(0.02, 0.6, R)
    pb = G.Problem(ctx, torch.from_numpy(V), cell["sublattice"], cell["species"], cell["charge"])
    occ0 = pb.init_occupations(R * groups, seed=R)
    ch = G.Chains(pb, occ0, G.GOAC_FP64)
    rng = np.random.default_rng(R)
    ref_slot = np.stack([rng.permutation(R).astype(np.int32) for _ in range(groups)])
    rows = np.argsort(ref_slot, axis=1).reshape(-1)
    ch.set_rows(rows)
    slot = torch.from_numpy(ref_slot.reshape(-1).copy()).cuda()
    acc = torch.zeros(R * groups, dtype=torch.uint8, device="cuda")
    ch.sweep(300, ladder[:, None], seed=2)
    _, _, stats = ch.export()
    for x in range(3):
        ch.remc_exchange(R, ladder, x, 9, slot, acc)
        got_acc = acc.view(groups, R).cpu().numpy()
        for g in range(groups):
            ref_slot[g], ref_acc = O.remc_exchange(ladder, stats["E"][g * R:(g + 1) * R], ref_slot[g], x, 9, group=g)
            assert np.array_equal(got_acc[g], ref_acc)
        assert np.array_equal(slot.view(groups, R).cpu().numpy(), ref_slot)
    _, _, stats = ch.export()
    rows = stats["row"].reshape(groups, R)
    for g in range(groups):
        assert np.array_equal(ref_slot[g][rows[g]], np.arange(R))
    # a repeated chain in group 1: that group keeps its slots and rows
    bad = ref_slot.copy()
    bad[1, 0] = bad[1, 1]
    slot = torch.from_numpy(bad.reshape(-1).copy()).cuda()
    ch.remc_exchange(R, ladder, 3, 9, slot, acc)
    ref0, _ = O.remc_exchange(ladder, stats["E"][:R], ref_slot[0], 3, 9, group=0)
    got = slot.view(groups, R).cpu().numpy()
    assert np.array_equal(got[0], ref0) and np.array_equal(got[1], bad[1])
    assert not acc.view(groups, R)[1].any()
    _, _, st2 = ch.export()
    assert np.array_equal(st2["row"].reshape(groups, R)[1], rows[1])
    ch.close()
    pb.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_leaves_chains_unchanged(ctx, cfg2, prec):
    """The tuner's probe sweeps leave the chains as they were, and sweeps with the
    chosen configuration stay bit-exact against the oracle."""
    cell, V = cfg2
    kT = np.geomspace(0.5, 0.01, 20)
    occ0 = O.init_occupations(cell, 48, seed=7)
    st = _run_oracle(cell, V, occ0, 20000, kT, 1000, 7)
    pb = G.Problem(ctx, torch.from_numpy(V), cell["sublattice"], cell["species"], cell["charge"])
    ch = G.Chains(pb, torch.from_numpy(occ0), prec)
    wg, pc = ch.autotune(2000, 0.05)
    assert wg in (64, 256) and pc >= 1
    occ, best, stats = ch.export()
    assert np.array_equal(occ.cpu().numpy(), occ0) and np.all(stats["t"] == 0) and np.all(stats["accepts"] == 0)
    ch.sweep(20000, kT, 1000, seed=7, trace=True)
    occ, best, stats = ch.export()
    _compare(cell, stats, occ.cpu().numpy(), best.cpu().numpy(), st, prec, V)


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("prec,groups", [(0, 16), (1, 16), (1, 1100)])
def test_remc_run_graph_matches_eager_rounds(ctx, cfg2, prec, groups, graph):
    """goac_remc_run's rounds, launched on the stream or replayed from one captured
    graph, equal the same rounds launched one by one (sweep + exchange), bit for
    bit; checked after several replays, after a second call that captures again,
    and with eager work and synchronisation between the calls. 4400 chains are more
    than the resident workgroups, so the sweep's work counter, cleared by each
    round's exchange, is in use."""
    cell, V = cfg2
    R = 4
    ladder = np.array([0.05, 0.1, 0.2, 0.4])
    occ0 = O.init_occupations(cell, R * groups, seed=12)
    pb = G.Problem(ctx, torch.from_numpy(V), cell["sublattice"], cell["species"], cell["charge"])
    a = G.Chains(pb, torch.from_numpy(occ0), prec)
    b = G.Chains(pb, torch.from_numpy(occ0), prec)
    sa = torch.tensor(np.tile(np.arange(R, dtype=np.int32), groups), device="cuda")
    sb = sa.clone()
    b.set_rows(np.tile(np.arange(R), groups))
    x = 0
    for rounds in (3, 1, 11):
        a.remc_run(R, ladder, 700, rounds, x, 5, sa, trace=True, graph=graph)
        for r in range(rounds):
            b.sweep(700, ladder[:, None], 700, seed=5, trace=True)
            b.remc_exchange(R, ladder, x + r, 5, sb)
        x += rounds
        oa, ba, st_a = a.export()
        ob, bb, st_b = b.export()
        assert np.array_equal(sa.cpu().numpy(), sb.cpu().numpy())
        assert np.array_equal(oa.cpu().numpy(), ob.cpu().numpy())
        for f in ("t", "hash", "accepts", "updates", "E", "best_E", "row"):
            assert np.array_equal(st_a[f], st_b[f]), f
        pb.energies(oa, 0)                        # eager work between the calls
        torch.cuda.synchronize()


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
def test_remc_run_on_a_cell_with_host_anchors(ctx, prec, graph):
    """goac_remc_run on the 8x8x8 cell (M = 2048): the mixed field there re-anchors
    between sweep chunks (2500 trials = two chunks at reanchor_every = 256), which
    runs every round from the host even when graph replay is asked for; rounds must
    equal sweeps and exchanges launched one by one, bit for bit."""
    cell = S.config3()
    Vg = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, Vg, cell["sublattice"], cell["species"], cell["charge"])
    del Vg
    R, groups = 4, 4
    ladder = np.array([0.05, 0.1, 0.2, 0.4])
    occ0 = pb.init_occupations(R * groups, seed=3)
    a = G.Chains(pb, occ0, prec)
    b = G.Chains(pb, occ0, prec)
    sa = torch.tensor(np.tile(np.arange(R, dtype=np.int32), groups), device="cuda")
    sb = sa.clone()
    b.set_rows(np.tile(np.arange(R), groups))
    x = 0
    for rounds in (2, 3):
        a.remc_run(R, ladder, 2500, rounds, x, 8, sa, trace=True, reanchor_every=256, graph=graph)
        for r in range(rounds):
            b.sweep(2500, ladder[:, None], 2500, seed=8, reanchor_every=256, trace=True)
            b.remc_exchange(R, ladder, x + r, 8, sb)
        x += rounds
        oa, _, st_a = a.export()
        ob, _, st_b = b.export()
        assert np.array_equal(sa.cpu().numpy(), sb.cpu().numpy())
        assert torch.equal(oa, ob)
        for f in ("t", "hash", "accepts", "updates", "E", "best_E", "row"):
            assert np.array_equal(st_a[f], st_b[f]), f
    Ef = pb.energies(oa, G.GOAC_FP64).cpu().numpy()
    assert np.abs(Ef - st_a["E"]).max() / len(cell["pos"]) <= TOL[prec]


# ------------------------------------------------------------------ GA

@pytest.mark.parametrize("P,prec,gens", [(203, 1, 21), (64, 0, 5), (128, 0, 17), (96, 1, 18)])
def test_ga_run_matches_generation_by_generation(ctx, cfg2, P, prec, gens):
    """goac_ga_run (graph replays of eight generations after the first, the rest on
    the stream) equals goac_ga_generation + goac_energies called generation by
    generation, bit for bit; a second call (captured again) after eager work too.
    The single generations are pinned to the oracle elsewhere."""
    cell, V = cfg2
    pb = G.Problem(ctx, torch.from_numpy(V), cell["sublattice"], cell["species"], cell["charge"])
    pop0 = pb.init_occupations(P, seed=P)
    E0 = pb.energies(pop0, prec)
    pa, Ea = pop0.clone(), E0.clone()
    pbk, Eb = pop0.clone(), E0.clone()
    g0 = 3
    for call in range(2):
        pb.ga_run(pa, Ea, seed=17, generation=g0, generations=gens, n_elite=4, p_mut=0.3, precision=prec)
        for k in range(gens):
            child = pb.ga_generation(pbk, Eb, seed=17, generation=g0 + k, n_elite=4, p_mut=0.3)
            Eb = pb.energies(child, prec)
            pbk = child
        assert torch.equal(pa, pbk), "populations differ (call %d)" % call
        assert torch.equal(Ea, Eb), "energies differ (call %d)" % call
        g0 += gens
        pb.energies(pop0, 0)                      # eager work between the calls
        torch.cuda.synchronize()
    pb.close()


def test_tiny_populations(ctx, cfg1):
    """P = 0 and P = 1 energies, top-k of all candidates, and a generation of a
    one-member population (zero roulette weight: the uniform pick)."""
    cell, V = cfg1
    pb = G.Problem(ctx, torch.from_numpy(V), cell["sublattice"], cell["species"], cell["charge"])
    n = len(cell["pos"])
    for prec in (G.GOAC_FP64, G.GOAC_MIXED):
        assert pb.energies(torch.zeros((0, n), dtype=torch.uint8), prec).numel() == 0
    pop = O.init_occupations(cell, 5, seed=4)
    Eo = O.energies(V, pop, cell["charge"])
    for prec, tol in ((G.GOAC_FP64, 1e-6), (G.GOAC_MIXED, 1e-4)):
        E1 = pb.energies(torch.from_numpy(pop[:1]), prec).cpu().numpy()
        assert abs(E1[0] - Eo[0]) / n <= tol
    idx, Ek = pb.topk(torch.from_numpy(pop), 5)
    idx_o, Ek_o = O.topk(V, pop, cell["charge"], 5)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    assert np.abs(Ek.cpu().numpy() - Ek_o).max() / n <= 1e-6
    one = pop[:1]
    got = pb.ga_generation(torch.from_numpy(one), torch.from_numpy(Eo[:1]), seed=2, generation=1, n_elite=0,
                           p_mut=1.0).cpu().numpy()
    assert np.array_equal(got, O.ga_generation(cell, one, Eo[:1], seed=2, g=1, n_elite=0, p_mut=1.0))
    pb.close()


def test_ga_generation_reports_roulette_overflow(ctx, cfg1):
    """An energy spread beyond the integer roulette weights' range is an error
    (set from the host, the kernels run normally); the next call starts clean."""
    cell, V = cfg1
    pb = G.Problem(ctx, torch.from_numpy(V), cell["sublattice"], cell["species"], cell["charge"])
    pop = O.init_occupations(cell, 64, seed=1)
    E = np.zeros(64)
    E[3] = -1e9
    with pytest.raises(G.GoacError, match="roulette"):
        pb.ga_generation(torch.from_numpy(pop), torch.from_numpy(E), seed=1, generation=0)
    E = -1000.0 + np.arange(64) * 0.01
    got = pb.ga_generation(torch.from_numpy(pop), torch.from_numpy(E), seed=1, generation=0).cpu().numpy()
    ref = O.ga_generation(cell, pop, E, seed=1, g=0)
    assert np.array_equal(got, ref)
    # a run of generations reports the failure after its last generation
    E_bad = torch.zeros(64, dtype=torch.float64, device="cuda")
    E_bad[3] = -1e9
    with pytest.raises(G.GoacError, match="roulette"):
        pb.ga_run(torch.from_numpy(pop).cuda(), E_bad, seed=1, generation=0, generations=3,
                  precision=G.GOAC_FP64)
    pb.close()


@pytest.mark.parametrize("which,P", [("config1", 64), ("config2", 203), ("config3", 1024), ("two", 96),
                                     ("config5", 24), ("many", 40)])
def test_ga_generation_bitexact(ctx, which, P):
    """Covers the byte walk (sublattices of up to 1024 positions, up to 20 species)
    and the window walk (the 2048-position sublattice of the 8x8x8 cell, the
    8192-position sublattice of the 16384-site cell)."""
    cell = {"two": two_sublattice_cell, "many": many_species_cell}.get(which, getattr(S, which, None))()
    V = torch.zeros((len(cell["pos"]),) * 2, dtype=torch.float64)
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    pop = O.init_occupations(cell, P, seed=1)
    rng = np.random.default_rng(P)
    E = -1000.0 + rng.normal(0.0, 3.0, P)
    E[5] = E[9]                                 # a tie for the elite order
    for g, (ne, pm) in enumerate([(8, 0.2), (0, 1.0), (3, 0.0)]):
        got = pb.ga_generation(torch.from_numpy(pop), torch.from_numpy(E), seed=31, generation=g, n_elite=ne,
                               p_mut=pm).cpu().numpy()
        ref = O.ga_generation(cell, pop, E, seed=31, g=g, n_elite=ne, p_mut=pm)
        assert np.array_equal(got, ref)
    # uniform selection when all energies are equal
    got = pb.ga_generation(torch.from_numpy(pop), torch.zeros(P, dtype=torch.float64), seed=3, generation=9,
                           n_elite=2, p_mut=0.5).cpu().numpy()
    assert np.array_equal(got, O.ga_generation(cell, pop, np.zeros(P), seed=3, g=9, n_elite=2, p_mut=0.5))


@pytest.mark.parametrize("parents", ["random", "near"])
def test_ga_window_walk_bitexact(ctx, parents):
    """The window walk on two long sublattices (1500 positions with a 28-position
    tail and 24 species, some with one or two ions, whose partners lie words ahead
    of the window; 1100 positions with four species), from random parents and from
    parents that agree on most words."""
    cell = long_window_cell()
    P = 96
    V = torch.zeros((len(cell["pos"]),) * 2, dtype=torch.float64)
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    pop = O.init_occupations(cell, P, seed=2) if parents == "random" else near_copies(cell, P, 40, seed=4)
    E = -10.0 + np.random.default_rng(11).normal(0.0, 1.0, P)
    for g, (ne, pm) in enumerate([(4, 0.3), (0, 0.0)]):
        got = pb.ga_generation(torch.from_numpy(pop), torch.from_numpy(E), seed=17, generation=g, n_elite=ne,
                               p_mut=pm).cpu().numpy()
        assert np.array_equal(got, O.ga_generation(cell, pop, E, seed=17, g=g, n_elite=ne, p_mut=pm))
    pb.close()


def test_ga_weight_overflow_is_an_error(ctx, cfg1):
    cell, V = cfg1
    pb = G.Problem(ctx, torch.from_numpy(V), cell["sublattice"], cell["species"], cell["charge"])
    pop = pb.init_occupations(8, seed=0)
    E = torch.tensor([0.0, 1e40] + [0.0] * 6, dtype=torch.float64)
    with pytest.raises(G.GoacError) as e:
        pb.ga_generation(pop, E, seed=0, generation=0)
    assert e.value.status == "EINVAL"


def test_chains_reject_broken_composition(ctx, cfg1):
    cell, V = cfg1
    pb = G.Problem(ctx, torch.from_numpy(V), cell["sublattice"], cell["species"], cell["charge"])
    occ = pb.init_occupations(4, seed=0)
    occ[2, 0] = 1 if occ[2, 0].item() == 2 else 2      # one Li <-> M change: counts break
    with pytest.raises(G.GoacError) as e:
        G.Chains(pb, occ, G.GOAC_FP64)
    assert e.value.status == "EINVAL"
