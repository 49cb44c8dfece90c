"""Shared helpers of the GPU parity tests (inputs and plain definitions only)."""
import numpy as np

import supercells as S


def two_sublattice_cell():
    """Rock-salt 2x2x2 conventional cell with both site classes mobile: 32 cation
    positions with 10 Li+, 6 Co3+, 16 Ni2+ (sublattice 0) and 32 anion positions
    with 4 F- and 28 O2- (sublattice 1); total charge 60 - 60 = 0."""
    lat, pos, kind = S.rocksalt_conventional(2, 2, 2, 4.2)
    names = ["Li", "Co", "Ni", "F", "O"]
    charge = [1.0, 3.0, 2.0, -1.0, -2.0]
    sub = kind.astype(np.int32)
    spc = np.zeros(len(pos), np.uint8)
    spc[kind == 0] = np.array([0] * 10 + [1] * 6 + [2] * 16, np.uint8)
    spc[kind == 1] = np.array([3] * 4 + [4] * 28, np.uint8)
    return S.make_cell(lat, pos, sub, spc, charge, names)


def many_species_cell():
    """Rock-salt 2x2x2 conventional cell whose 32 cation positions hold 20 species
    (ids 0..19, all 2+: twelve with two ions, eight with one) over 32 fixed O2-;
    more species than a register-resident crossover walk holds."""
    lat, pos, kind = S.rocksalt_conventional(2, 2, 2, 4.2)
    names = ["M%d" % e for e in range(20)] + ["O"]
    charge = [2.0] * 20 + [-2.0]
    sub = np.where(kind == 0, 0, -1).astype(np.int32)
    spc = np.full(len(pos), 20, np.uint8)
    spc[kind == 0] = np.array(sum(([e, e] for e in range(12)), []) + list(range(12, 20)), np.uint8)
    return S.make_cell(lat, pos, sub, spc, charge, names)


def swap_energy_difference(Vi, Vj, q, i, j):
    """E(q') - E(q) for q' = q with entries i and j exchanged, from rows i and j of
    the pair matrix only: with delta = q' - q (non-zero at i and j),
    1/2 q'^T V q' - 1/2 q^T V q = 1/2 delta^T V (q + q')."""
    q2 = q.copy()
    q2[i], q2[j] = q[j], q[i]
    s = q + q2
    return 0.5 * ((q2[i] - q[i]) * (Vi @ s) + (q2[j] - q[j]) * (Vj @ s))


def degenerate_sublattice_cell():
    """Config-1 geometry with the 16 cation positions split into two sublattices:
    eight hold Mg2+ only (no swap there has a valid partner) and eight hold four
    Li+ and four M3+; 16 fixed O2-; total charge 16 + 16 - 32 = 0."""
    lat, pos, kind = S.rocksalt_conventional(2, 2, 1, 4.2)
    names = ["O", "Li", "M", "Mg"]
    charge = [-2.0, 1.0, 3.0, 2.0]
    cat = np.nonzero(kind == 0)[0]
    sub = np.full(len(pos), -1, np.int32)
    sub[cat[:8]] = 0
    sub[cat[8:]] = 1
    spc = np.zeros(len(pos), np.uint8)
    spc[cat[:8]] = 3
    spc[cat[8:]] = np.array([1, 2] * 4, np.uint8)
    return S.make_cell(lat, pos, sub, spc, charge, names)


def long_window_cell(seed=5):
    """3072 sites of a 16x16x12 simple-cubic grid (a = 3 A) in seeded random site
    order: sublattice 0 has 1500 positions (23 words of 64 and a 28-position tail)
    holding 24 species with counts from 1 to 300, so that some partners lie many
    words ahead; sublattice 1 has 1100 positions holding four species; 472 sites
    are fixed. The pair matrix is not used, so the charges are placeholders."""
    g = np.stack(np.meshgrid(np.arange(16), np.arange(16), np.arange(12), indexing="ij"), -1).reshape(-1, 3)
    lat = np.diag([48.0, 48.0, 36.0])
    pos = g * 3.0
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(len(pos))
    sub = np.full(len(pos), -1, np.int32)
    sub[order[:1500]] = 0
    sub[order[1500:2600]] = 1
    small = [1, 1, 2, 3, 5, 8, 13, 21, 34, 55] + [25] * 9 + [32]
    counts0 = [300, 300, 250, 250] + small
    assert sum(counts0) == 1500 and len(counts0) == 24
    spc = np.full(len(pos), 28, np.uint8)
    spc[order[:1500]] = np.repeat(np.arange(24), counts0).astype(np.uint8)
    spc[order[1500:2600]] = np.repeat(np.arange(24, 28), [500, 300, 200, 100]).astype(np.uint8)
    names = ["X%d" % e for e in range(29)]
    return S.make_cell(lat, pos, sub, spc, [0.0] * 29, names)


def near_copies(cell, P, swaps, seed):
    """P occupations that each differ from one seeded random occupation by up to
    `swaps` random exchanges inside the mobile sublattices (parents that agree on
    most 64-position words)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = S.random_occupations(cell, 1, seed)[0]
    out = np.repeat(base[None, :], P, axis=0)
    subs = sorted(set(cell["sublattice"].tolist()) - {-1})
    for p in range(P):
        for _ in range(int(rng.integers(0, swaps + 1))):
            idx = np.nonzero(cell["sublattice"] == subs[int(rng.integers(len(subs)))])[0]
            i, j = rng.choice(idx, 2, replace=False)
            out[p, i], out[p, j] = out[p, j], out[p, i]
    return out
