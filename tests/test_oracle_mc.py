"""Pins of the oracle's random start, Metropolis/annealed swap Monte Carlo and
replica exchange (SI, "Random", "Monte Carlo", "Simulated annealing", "Replica
Exchange Monte Carlo")."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle as O
import supercells as S

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available to build the rocrand cross-check")
    exe = str(tmp_path_factory.mktemp("philox") / "rocref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_ref", "rocrand_philox_ref.cpp")])
    return exe


def test_philox_against_rocrand_header(rocrand_ref):
    rng = np.random.default_rng(0)
    rows = rng.integers(0, 2 ** 32, size=(200, 6), dtype=np.uint64)
    rows[:, 1] %= 2 ** 30          # the header's offset encoding covers c1 < 2^30
    rows[0] = 0
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], np.uint64)
    mine = np.stack([O.philox(r[:4], r[4:]) for r in rows]).astype(np.uint64)
    assert np.array_equal(mine, ref)


@pytest.fixture(scope="module")
def cfg1():
    c = S.config1()
    V = O.cell_matrix(c)
    occ = S.config1_exhaustive_occupations(c)
    E = O.energies(V, occ, c["charge"])
    table = {r.tobytes(): e for r, e in zip(occ, E)}
    return c, V, occ, E, table


@pytest.fixture(scope="module")
def cfg2():
    c = S.config2()
    return c, O.cell_matrix(c)


def test_init_composition_and_uniformity():
    c = S.config1()
    occ = O.init_occupations(c, 20000, seed=123)
    assert np.all((occ[:, :16] == 1).sum(1) == 8) and np.all(occ[:, 16:] == 0)
    # each position holds Li with probability 1/2
    frac = (occ[:, :16] == 1).mean(0)
    assert np.all(np.abs(frac - 0.5) < 5 * np.sqrt(0.25 / 20000))
    # a four-position sublattice with four species: the 24 orders are uniform
    cell = dict(sublattice=np.array([0, 0, 0, 0, -1], np.int32),
                species=np.array([0, 1, 2, 3, 4], np.uint8), charge=np.zeros(5))
    occ = O.init_occupations(cell, 24000, seed=9)
    keys, counts = np.unique(occ[:, :4], axis=0, return_counts=True)
    assert len(keys) == 24
    assert stats.chisquare(counts).pvalue > 1e-3


def test_tracked_energy_equals_recompute(cfg2):
    """dE from the field (and the rank-2 field updates) must track the full
    recompute of 1/2 q^T V q over a long trajectory."""
    cell, V = cfg2
    st = O.MCState(O.init_occupations(cell, 4, seed=5))
    O.mc_run(V, cell, st, seed=5, n_trials=3000, kT=[0.5], block_len=10 ** 9)
    E = O.energies(V, st.occ, cell["charge"])
    assert np.all(st.field("accepts") > 100)
    assert np.allclose(st.field("E"), E, rtol=1e-11, atol=0)
    Eb = O.energies(V, st.best_occ, cell["charge"])
    assert np.allclose(st.field("best_E"), Eb, rtol=1e-11, atol=0)
    assert np.all(st.field("best_E") <= st.field("E"))
    # composition and perm consistency
    for p in range(4):
        assert (st.occ[p] == 1).sum() == 128
        assert sorted(st.perm[p].tolist()) == list(range(256))


def test_exhaustive_config1_chains(cfg1):
    """Config 1's MC run (64 chains x 1e4 trials, kT = 0.05 eV, seed 0): every
    final and best state's tracked energy equals its exhaustive-table value."""
    cell, V, occ, E, table = cfg1
    st = O.MCState(O.init_occupations(cell, 64, seed=0))
    O.mc_run(V, cell, st, seed=0, n_trials=10000, kT=[0.05], block_len=10 ** 9)
    for p in range(64):
        assert abs(st.stats[p].E - table[st.occ[p].tobytes()]) < 1e-9
        assert abs(st.stats[p].best_E - table[st.best_occ[p].tobytes()]) < 1e-9
    # a cold chain ends near the ground state
    assert st.field("best_E").min() - E.min() < 1e-9


def test_boltzmann_distribution(cfg1):
    """Long chains at kT = 2 eV sample exp(-E/kT) over the 12870 states of
    config 1 (levels of equal energy pooled), a chi-square test."""
    cell, V, occ, E, table = cfg1
    kT = 2.0
    C = 3000
    st = O.MCState(O.init_occupations(cell, C, seed=77))
    O.mc_run(V, cell, st, seed=77, n_trials=4000, kT=[kT], block_len=10 ** 9)
    levels, inv = np.unique(np.round(E, 6), return_inverse=True)
    w = np.exp(-(E - E.min()) / kT)
    p_level = np.bincount(inv, weights=w) / w.sum()
    lvl_of = {r.tobytes(): i for r, i in zip(occ, inv)}
    obs = np.bincount([lvl_of[o.tobytes()] for o in st.occ], minlength=len(levels))
    exp_ = p_level * C
    # pool levels with small expectation into one bin
    big = exp_ >= 10
    o2 = np.r_[obs[big], obs[~big].sum()]
    e2 = np.r_[exp_[big], exp_[~big].sum()]
    assert stats.chisquare(o2, e2).pvalue > 1e-4


def test_resume_identity(cfg2):
    cell, V = cfg2
    occ0 = O.init_occupations(cell, 3, seed=2)
    kT = np.geomspace(0.5, 0.01, 10)
    a = O.MCState(occ0)
    O.mc_run(V, cell, a, seed=2, n_trials=3000, kT=kT, block_len=300)
    b = O.MCState(occ0)
    O.mc_run(V, cell, b, seed=2, n_trials=1000, kT=kT, block_len=300)
    O.mc_run(V, cell, b, seed=2, n_trials=2000, kT=kT, block_len=300)
    assert np.array_equal(a.occ, b.occ) and np.array_equal(a.perm, b.perm)
    for f in ("t", "accepts", "updates", "hash"):
        assert np.array_equal(a.field(f), b.field(f))
    assert np.allclose(a.field("E"), b.field("E"), rtol=1e-12)


def test_zero_temperature_is_downhill(cfg2):
    cell, V = cfg2
    st = O.MCState(O.init_occupations(cell, 2, seed=8))
    E0 = O.energies(V, st.occ, cell["charge"])
    O.mc_run(V, cell, st, seed=8, n_trials=2000, kT=[1e-9], block_len=10 ** 9)
    assert np.all(st.field("E") < E0)
    assert np.allclose(st.field("best_E"), st.field("E"), rtol=0, atol=1e-9)


def test_hash_distinguishes_trajectories(cfg2):
    cell, V = cfg2
    occ0 = O.init_occupations(cell, 2, seed=3)
    a = O.MCState(occ0)
    O.mc_run(V, cell, a, seed=3, n_trials=500, kT=[0.3], block_len=10 ** 9)
    b = O.MCState(occ0)
    O.mc_run(V, cell, b, seed=4, n_trials=500, kT=[0.3], block_len=10 ** 9)
    assert np.all(a.field("hash") != b.field("hash"))
    # the hash is a sum of per-trial terms
    assert O.trial_hash(5, 1, 2, 1) != O.trial_hash(5, 1, 2, 0)


def test_remc_exchange_acceptance_rule():
    """Exchange between neighbouring temperatures is accepted with probability
    min(1, exp(dE (1/kT1 - 1/kT2)))."""
    kT = np.array([0.2, 0.5])
    E = np.array([-10.0, -10.1])           # the colder replica holds the higher energy
    slot, acc = O.remc_exchange(kT, E, [0, 1], 0, seed=1)
    assert acc[0] == 1 and list(slot) == [1, 0]
    E = np.array([-10.1, -10.0])
    p = np.exp((E[0] - E[1]) * (1 / kT[0] - 1 / kT[1]))
    n = 4000
    hits = sum(int(O.remc_exchange(kT, E, [0, 1], 2 * x, seed=5)[1][0]) for x in range(n))
    assert abs(hits / n - p) < 5 * np.sqrt(p * (1 - p) / n)
    # odd steps pair (1, 2), (3, 4), ...
    slot, acc = O.remc_exchange(np.array([0.1, 0.2, 0.3]), np.array([0., 0., 0.]), [0, 1, 2], 1, seed=1)
    assert acc[0] == 0 and acc[1] == 1 and list(slot) == [0, 2, 1]


def _stats_view(st):
    """The chains' counters as a numpy structured view (no copy)."""
    dt = np.dtype([(f, np.uint64 if t is O.C.c_uint64 else np.float64) for f, t in O.ChainStats._fields_])
    return np.frombuffer(memoryview(st.stats).cast("B"), dtype=dt)


def remc_rounds(cell, V, ladder, groups, rounds, trials, seed):
    """Replica exchange by the oracle's pieces: every round each chain runs
    `trials` trials at the temperature of its slot, then exchange step x in every
    group of R consecutive chains. Returns the final state and slots."""
    R = len(ladder)
    st = O.MCState(O.init_occupations(cell, R * groups, seed=seed))
    slot = np.tile(np.arange(R, dtype=np.int32), (groups, 1))
    base = (np.arange(groups) * R)[:, None]
    for x in range(rounds):
        rows = np.empty(R * groups, np.int32)
        rows[(base + slot).ravel()] = np.tile(np.arange(R, dtype=np.int32), groups)
        O.mc_run(V, cell, st, seed=seed, n_trials=trials, kT=np.asarray(ladder)[:, None], block_len=trials,
                 kT_row=rows)
        E = _stats_view(st)["E"].copy()
        for g in range(groups):
            slot[g], _ = O.remc_exchange(ladder, E[g * R:(g + 1) * R], slot[g], x, seed, group=g)
    return st, slot


def test_remc_stationary_distribution(cfg1):
    """Replica exchange leaves the product of the ladder's Boltzmann distributions
    invariant (SI, "Replica Exchange Monte Carlo"), so the configuration held at
    temperature k is distributed as exp(-E/kT_k) over the 12870 states of config 1.
    Many independent groups are run from random starts with few trials between
    exchanges (the exchanges carry much of the mixing) and sampled right after an
    exchange step; each temperature's energy levels get a chi-square test."""
    cell, V, occ, E, table = cfg1
    ladder = np.array([0.4, 0.8, 1.6, 3.2])
    groups = 1500
    st, slot = remc_rounds(cell, V, ladder, groups, rounds=300, trials=8, seed=21)
    levels, inv = np.unique(np.round(E, 6), return_inverse=True)
    lvl_of = {r.tobytes(): i for r, i in zip(occ, inv)}
    for k, kT in enumerate(ladder):
        held = st.occ[np.arange(groups) * len(ladder) + slot[:, k]]
        obs = np.bincount([lvl_of[o.tobytes()] for o in held], minlength=len(levels))
        w = np.exp(-(E - E.min()) / kT)
        exp_ = np.bincount(inv, weights=w) / w.sum() * groups
        big = exp_ >= 10
        o2 = np.r_[obs[big], obs[~big].sum()]
        e2 = np.r_[exp_[big], exp_[~big].sum()]
        if e2[-1] == 0:
            o2, e2 = o2[:-1], e2[:-1]
        assert stats.chisquare(o2, e2).pvalue > 1e-4, "temperature %g" % kT
