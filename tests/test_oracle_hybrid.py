"""Pins of the oracle's REMC + GA hybrid round (SI, "Hybrid Methods"): it is a
composition of pinned pieces, so the checks are the invariants the composition
must keep: compositions, slot permutations, energies of the returned population,
no loss of the best solution, and determinism."""
import numpy as np

import oracle as O
import supercells as S


def _setup(seed=3):
    cell = S.config1()
    V = O.cell_matrix(cell)
    R, G, P = 4, 4, 24
    occ0 = O.init_occupations(cell, R * G, seed=seed)
    st = O.MCState(occ0)
    pop = O.init_occupations(cell, P, seed=seed + 100, chain_base=1000)
    slot = np.tile(np.arange(R, dtype=np.int32), (G, 1))
    return cell, V, st, pop, slot, R


def _run(rounds=3):
    cell, V, st, pop, slot, R = _setup()
    ladder = np.array([0.05, 0.1, 0.2, 0.4])
    out = []
    for r in range(rounds):
        before_best = min(O.energies(V, pop, cell["charge"]).min(), st.field("best_E").min() if r else np.inf)
        chain_best = st.field("best_E").copy() if r else None
        pop, E, slot = O.hybrid_round(V, cell, st, slot, pop, r, R, ladder, trials=400, exchanges=2,
                                      generations=2, n_elite=2, p_mut=0.3, seed=9, inject=3)
        out.append((pop.copy(), E.copy(), slot.copy(), st.occ.copy(), st.field("best_E").copy()))
        assert np.allclose(E, O.energies(V, pop, cell["charge"]), atol=1e-9)
        assert E.min() <= before_best + 1e-9
        if chain_best is not None:
            assert np.all(st.field("best_E") <= chain_best + 1e-12)
        for row in np.concatenate([pop, st.occ]):
            assert np.array_equal(np.bincount(row, minlength=3), np.bincount(cell["species"], minlength=3))
        for g in slot:
            assert sorted(g.tolist()) == list(range(R))
    return out


def test_hybrid_round_invariants_and_determinism():
    a = _run()
    b = _run()
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)


# ---------------------------------------------------------------------------------------
# Hand-built hand-over cases. The pair matrix is an integer circulant over the 16
# mobile positions of the 2x2x1 rock-salt cell (no coupling to the fixed ions), so
# every energy is an exact half-integer and a cyclic shift of the mobile occupation
# has exactly the same energy as the original while being a different occupation.
# With zero trials and a ladder of 1e-3 and 1 eV, every exchange of these cases
# pairs a colder replica at least 4 eV lower than its hotter neighbour, so the
# acceptance exp(-4 * 999) rounds to zero and no slot moves. The expected
# populations and injections below are worked out by hand from the reading of the
# round (SI, "Hybrid Methods"): candidates are the population followed by the
# chains' BEST occupations, the P lowest by (energy, index) survive, and the
# coldest replica (slot[g][0]) of group g takes rank g mod min(inject, P) only when
# that individual is strictly lower than the replica's CURRENT energy.

def _circulant_problem():
    cell = S.config1()
    n, M = len(cell["species"]), 16
    f = np.array([6, 3, -2, 1, 4, -1, 2, 0, 5, 0, 2, -1, 4, 1, -2, 3], np.float64)
    V = np.zeros((n, n))
    i = np.arange(M)
    V[:M, :M] = f[(i[None, :] - i[:, None]) % M]
    A = np.random.default_rng(0).integers(-3, 4, (n - M, n - M)).astype(np.float64)
    V[M:, M:] = np.triu(A) + np.triu(A, 1).T
    table = S.config1_exhaustive_occupations(cell)
    E = O.energies(V, table, cell["charge"])
    levels = np.unique(E)

    def rep(k):
        return table[np.nonzero(E == levels[k])[0][0]].copy()

    def shifted(o):
        s = o.copy()
        s[:M] = np.roll(o[:M], 1)
        return s

    return cell, V, levels, rep, shifted


def _start(cell, V, occ):
    st = O.MCState(np.array(occ, np.uint8))
    O.mc_run(V, cell, st, seed=0, n_trials=0, kT=[1.0], block_len=1)
    return st


def test_hybrid_handover_by_hand():
    cell, V, L, rep, _ = _circulant_problem()
    ladder = [1e-3, 1.0]
    pop = np.stack([rep(9), rep(5), rep(11), rep(7)])
    # group 0: chain 0 hot, chain 1 cold; group 1: chain 2 cold, chain 3 hot;
    # group 2: chain 4 cold, chain 5 hot
    chains = [rep(30), rep(3), rep(1), rep(25), rep(8), rep(35)]
    slot = np.array([[1, 0], [0, 1], [0, 1]], np.int32)
    st = _start(cell, V, chains)
    # chain 1 moves on to a higher occupation: its best stays rep(3)
    moved = np.stack(chains)
    moved[1] = rep(20)
    O.mc_reload(st, V, cell["charge"], moved)
    assert st.field("E")[1] == L[20] and st.field("best_E")[1] == L[3]
    pop2, E2, slot2 = O.hybrid_round(V, cell, st, slot, pop, 0, 2, ladder, trials=0, exchanges=1, generations=0,
                                     n_elite=1, p_mut=0.0, seed=5, inject=2)
    assert np.array_equal(slot2, slot)
    # candidates: pop rows 0..3 at levels 9, 5, 11, 7; chain bests at 30, 3, 1, 25, 8, 35;
    # the four lowest are chain 2 (1), chain 1's best (3), pop 1 (5), pop 3 (7)
    assert np.array_equal(pop2, np.stack([rep(1), rep(3), rep(5), rep(7)]))
    assert np.array_equal(E2, [L[1], L[3], L[5], L[7]])
    # hand-over with inject = 2: group 0's coldest is chain 1 (slot [1, 0]), current
    # level 20 > 1: takes rank 0; group 1's coldest, chain 2 at level 1, is offered rank 1
    # (level 3): not lower, kept; group 2's coldest, chain 4 at level 8, is offered
    # rank 2 mod 2 = 0 (level 1): takes it
    want = np.stack([rep(30), rep(1), rep(1), rep(25), rep(1), rep(35)])
    assert np.array_equal(st.occ, want)
    assert np.array_equal(st.field("E"), [L[30], L[1], L[1], L[25], L[1], L[35]])
    assert np.array_equal(st.field("best_E"), [L[30], L[1], L[1], L[25], L[1], L[35]])
    assert np.array_equal(st.best_occ[1], rep(1)) and np.array_equal(st.best_occ[4], rep(1))


def test_hybrid_handover_needs_strictly_lower():
    cell, V, L, rep, shifted = _circulant_problem()
    o3, s3 = rep(3), shifted(rep(3))
    assert not np.array_equal(o3, s3)
    assert O.energies(V, s3[None], cell["charge"])[0] == L[3]
    st = _start(cell, V, [s3, rep(30)])
    pop = np.stack([o3, rep(12)])
    pop2, E2, slot2 = O.hybrid_round(V, cell, st, np.array([[0, 1]], np.int32), pop, 0, 2, [1e-3, 1.0], trials=0,
                                     exchanges=1, generations=0, n_elite=1, p_mut=0.0, seed=5, inject=1)
    # candidates o3 (3), rep 12, the shifted o3 (3), rep 30: the two at level 3 survive in index order
    assert np.array_equal(pop2, np.stack([o3, s3])) and np.array_equal(E2, [L[3], L[3]])
    # rank 0 (o3) ties with the coldest replica's energy: no hand-over
    assert np.array_equal(st.occ[0], s3) and np.array_equal(st.occ[1], rep(30))
