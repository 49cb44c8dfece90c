"""Pins of the oracle's genetic-algorithm generation (SI, "Genetic Algorithm":
roulette-wheel parents, swap crossover accepting each differing swap with
probability 1/2, swap mutation at a rate, elitism) and of the top-k ranking."""
import numpy as np
from scipy import stats

import oracle as O
import supercells as S


def _cfg1():
    c = S.config1()
    return c, O.cell_matrix(c)


def test_composition_elites_and_inheritance():
    cell, V = _cfg1()
    pop = S.random_occupations(cell, 64, seed=3)
    E = O.energies(V, pop, cell["charge"])
    out = O.ga_generation(cell, pop, E, seed=1, g=0, n_elite=8, p_mut=0.2)
    assert np.all((out[:, :16] == 1).sum(1) == 8) and np.all(out[:, 16:] == 0)
    order = np.lexsort((np.arange(64), E))
    assert np.array_equal(out[:8], pop[order[:8]])


def test_crossover_three_cycle_path():
    # three species in a 3-cycle: the path from A to B is two overlapping swaps;
    # every subset keeps the composition and the all-swaps child is B
    cell = dict(sublattice=np.array([0, 0, 0], np.int32), species=np.array([0, 1, 2], np.uint8),
                charge=np.zeros(3))
    A = np.array([0, 1, 2], np.uint8)
    B = np.array([1, 2, 0], np.uint8)
    P = 4000
    pop = np.stack([A, B] * (P // 2))
    out = O.ga_generation(cell, pop, np.zeros(P), seed=6, g=0, n_elite=0, p_mut=0.0)
    assert np.all(np.sort(out, axis=1) == [0, 1, 2])
    # children of (A, B): A, swap(0,1) -> [1,0,2], swap(1,2) of A -> [0,2,1], both -> B
    seen = {tuple(r) for r in out}
    assert {(0, 1, 2), (1, 0, 2), (0, 2, 1), (1, 2, 0)} <= seen


def test_crossover_keeps_agreeing_positions():
    cell, _ = _cfg1()
    pop = S.random_occupations(cell, 2, seed=5)
    A, B = pop
    agree = A == B
    out = O.ga_generation(cell, np.repeat(pop, 200, axis=0), np.zeros(400), seed=2, g=3,
                          n_elite=0, p_mut=0.0)
    assert np.all(out[:, agree] == A[agree])
    assert np.all((out[:, :16] == 1).sum(1) == 8)
    # the children spread between the two parents
    dist_a = (out != A).sum(1)
    assert dist_a.min() == 0 and dist_a.max() == (A != B).sum()


def test_crossover_half_of_swaps_for_two_species():
    # with two species the swap path from A to B is k disjoint swaps (k = half the
    # differing positions), each taken with probability 1/2: a child of (A, B)
    # differs from A in 2 x Binomial(k, 1/2) positions
    cell, _ = _cfg1()
    pop = S.random_occupations(cell, 2, seed=21)
    A, B = pop
    k = (A != B).sum() // 2
    assert k >= 3
    # equal energies: uniform parents, so (A,A), (A,B), (B,A), (B,B) each 1/4
    P = 6000
    out = O.ga_generation(cell, np.repeat(pop, P // 2, axis=0), np.zeros(P), seed=9, g=1,
                          n_elite=0, p_mut=0.0)
    d = (out != A).sum(1) // 2
    # mixture: (A,A) -> 0, (B,B) -> k, (A,B) -> Bin(k,1/2), (B,A) -> k - Bin(k,1/2)
    probs = np.zeros(k + 1)
    probs[0] += 0.25
    probs[k] += 0.25
    probs += 0.5 * stats.binom.pmf(np.arange(k + 1), k, 0.5)
    obs = np.bincount(d, minlength=k + 1)
    assert stats.chisquare(obs, probs * P).pvalue > 1e-4


def test_roulette_frequencies():
    # rows 0..2 distinct, the rest copies of row 3 with the highest energy (zero
    # weight); w = (3, 2, 1, 0, ...): parents are drawn with pi = (1/2, 1/3, 1/6).
    # A child equals row p when both parents are p, or when the parents are p and
    # q != p and none (p first) or all (p second) of the k_pq path swaps are taken
    cell, _ = _cfg1()
    base = S.random_occupations(cell, 4, seed=13)
    P = 4000
    pop = np.repeat(base[3:4], P, axis=0)
    pop[:3] = base[:3]
    E = np.full(P, 3.0)
    E[:3] = [0.0, 1.0, 2.0]
    out = O.ga_generation(cell, pop, E, seed=4, g=0, n_elite=0, p_mut=0.0)
    pi = np.array([1 / 2, 1 / 3, 1 / 6])
    for p in range(3):
        prob = pi[p] ** 2
        for q in range(3):
            if q != p:
                k = (base[p] != base[q]).sum() // 2
                prob += 2 * pi[p] * pi[q] * 0.5 ** k
        hits = np.all(out == base[p], axis=1).sum()
        assert abs(hits / P - prob) < 5 * np.sqrt(prob * (1 - prob) / P)
    assert not np.any(np.all(out == base[3], axis=1))


def test_mutation_rate_and_single_swap():
    cell, _ = _cfg1()
    row = S.random_occupations(cell, 1, seed=2)[0]
    P = 5000
    pop = np.repeat(row[None], P, axis=0)
    out = O.ga_generation(cell, pop, np.zeros(P), seed=3, g=0, n_elite=0, p_mut=1.0)
    assert np.all((out != row).sum(1) == 2)
    out = O.ga_generation(cell, pop, np.zeros(P), seed=3, g=0, n_elite=0, p_mut=0.0)
    assert np.all(out == row)
    out = O.ga_generation(cell, pop, np.zeros(P), seed=3, g=0, n_elite=0, p_mut=0.3)
    frac = np.mean((out != row).sum(1) == 2)
    assert abs(frac - 0.3) < 5 * np.sqrt(0.21 / P)


def test_elitism_best_never_increases():
    cell, V = _cfg1()
    pop = O.init_occupations(cell, 32, seed=1)
    best = []
    for g in range(12):
        E = O.energies(V, pop, cell["charge"])
        best.append(E.min())
        pop = O.ga_generation(cell, pop, E, seed=7, g=g, n_elite=4, p_mut=0.2)
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:]))


def test_topk_is_sorted_exhaustive_table():
    cell, V = _cfg1()
    occ = S.config1_exhaustive_occupations(cell)
    E = O.energies(V, occ, cell["charge"])
    idx, Ek = O.topk(V, occ, cell["charge"], 40)
    order = np.lexsort((np.arange(len(E)), E))[:40]
    assert np.array_equal(idx, order) and np.array_equal(Ek, E[order])
