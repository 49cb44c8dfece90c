"""Pins of the oracle's best-swap descent (SI, "Gradient Descent") against a
brute-force descent that scores every neighbour by a full energy recomputation,
and against the exhaustive configuration table of the 16-site cell."""
import sys
import os

import numpy as np
import pytest

import oracle as O
import supercells as S

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import two_sublattice_cell  # noqa: E402  (plain cell builder, no GPU use)

TOL = 1e-9


def brute_descent(V, cell, occ, tol=TOL, max_steps=10 ** 9):
    """Each step: energies of all single swaps of different species within a site
    class by 1/2 q'^T V q', then the lexicographically first swap within tol of
    the lowest; stop when nothing lies lower than -tol."""
    charge = np.asarray(cell["charge"], float)
    sub = cell["sublattice"]
    mob = np.nonzero(sub >= 0)[0]
    o = occ.copy()
    steps = 0
    while steps < max_steps:
        q = charge[o]
        E = 0.5 * q @ V @ q
        cand = []
        for a in range(len(mob)):
            for b in range(a + 1, len(mob)):
                i, j = mob[a], mob[b]
                if sub[i] != sub[j] or o[i] == o[j]:
                    continue
                q2 = q.copy()
                q2[i], q2[j] = q[j], q[i]
                cand.append((0.5 * q2 @ V @ q2 - E, a, b))
        if not cand:
            break
        lo = min(c[0] for c in cand)
        if not lo < -tol:
            break
        _, a, b = min((c for c in cand if c[0] <= lo + tol), key=lambda c: (c[1], c[2]))
        i, j = mob[a], mob[b]
        o[i], o[j] = o[j], o[i]
        steps += 1
    q = charge[o]
    return o, steps, 0.5 * q @ V @ q


@pytest.mark.parametrize("which", ["config1", "two"])
def test_descent_matches_brute_force(which):
    cell = two_sublattice_cell() if which == "two" else S.config1()
    V = O.cell_matrix(cell)
    occ = O.init_occupations(cell, 6, seed=5)
    got, steps, E = O.gd_run(V, cell, occ)
    for p in range(len(occ)):
        o, st, Eb = brute_descent(V, cell, occ[p])
        assert np.array_equal(got[p], o)
        assert steps[p] == st
        assert abs(E[p] - Eb) < 1e-9 * len(o)


def test_endpoints_are_local_minima_of_the_exhaustive_table():
    """Every endpoint is a local minimum: no single Li <-> M swap of the 16-site
    cell's exhaustive table lies lower; the tracked energy is the table's."""
    cell = S.config1()
    V = O.cell_matrix(cell)
    table = S.config1_exhaustive_occupations(cell)
    E_tab = O.energies(V, table, cell["charge"])
    index = {row.tobytes(): k for k, row in enumerate(table)}
    occ = O.init_occupations(cell, 64, seed=2)
    got, steps, E = O.gd_run(V, cell, occ)
    mob = np.nonzero(cell["sublattice"] >= 0)[0]
    for p in range(len(got)):
        k = index[got[p].tobytes()]
        assert abs(E_tab[k] - E[p]) < 1e-9 * len(mob)
        for a in range(len(mob)):
            for b in range(a + 1, len(mob)):
                i, j = mob[a], mob[b]
                if got[p][i] == got[p][j]:
                    continue
                o = got[p].copy()
                o[i], o[j] = o[j], o[i]
                assert E_tab[index[o.tobytes()]] >= E[p] - TOL


def test_step_limit_and_monotone_descent():
    cell = S.config2()
    V = O.cell_matrix(cell)
    occ = O.init_occupations(cell, 4, seed=9)
    E0 = O.energies(V, occ, cell["charge"])
    prev = E0
    cur = occ
    for _ in range(3):
        cur, steps, E = O.gd_run(V, cell, cur, max_steps=2)
        assert np.all(steps <= 2)
        assert np.all(E <= prev + 1e-9)
        assert np.allclose(E, O.energies(V, cur, cell["charge"]), atol=1e-9 * len(cell["pos"]))
        prev = E
