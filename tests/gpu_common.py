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
