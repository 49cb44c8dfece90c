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
