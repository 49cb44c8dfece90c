"""Pins of the oracle's Ewald pair matrix against values the paper and the
mathematics fix (Methodology, "Cluster Expansion of Coulomb Energy": periodic
point-charge energies by Ewald summation; Results, "Atomistic Configurations in
NaCl", Eq. 3 and the Madelung constant 1.74756)."""
import json
import os

import numpy as np
import pytest

import oracle as O
import supercells as S

KE = O.coulomb_constant()
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))

# Madelung constants (textbook lattice sums): NaCl 1.747565 (the paper prints
# 1.74756), CsCl 1.762675.
M_NACL = 1.747565
M_CSCL = 1.762675


def madelung(E, r, n_ions):
    # Eq. 3 with E in eV: M = r |E| / ((N/2) k_e)
    return r * abs(E) / ((n_ions / 2) * KE)


def test_coulomb_constant_codata():
    # e/(4 pi eps0) in eV*A from CODATA 2018: 14.3996454784
    assert abs(KE - 14.3996454784) < 1e-9


@pytest.mark.parametrize("reps,alpha", [(1, 0.6), (1, 0.9), (2, 0.45)])
def test_madelung_nacl_matrix(reps, alpha):
    lat, pos, kind = S.rocksalt_conventional(reps, reps, reps, 5.62)
    q = np.where(kind == 0, 1.0, -1.0)
    V = O.ewald_matrix(lat, pos, alpha)
    E = 0.5 * q @ V @ q
    assert abs(madelung(E, 2.81, len(q)) - M_NACL) < 5e-7
    assert round(madelung(E, 2.81, len(q)), 5) == 1.74756


def test_madelung_nacl_paper_cell():
    # the paper's 3x3x3 cell with its printed ion count, nearest-neighbour
    # distance and Madelung constant (tests/golden/paper_values.json), in the
    # structure-factor form
    g = GOLDEN["nacl_madelung"]
    lat, pos, kind = S.rocksalt_conventional(3, 3, 3, 2 * g["r_angstrom"])
    q = np.where(kind == 0, 1.0, -1.0)
    E = O.ewald_energy(lat, pos, q)
    assert len(q) == g["n_ions"]
    M = madelung(E, g["r_angstrom"], g["n_ions"])
    assert round(M, g["digits"]) == g["M"]
    assert abs(M - M_NACL) < 5e-7


def test_madelung_nacl_rhombohedral_cell():
    # a non-orthogonal (FCC primitive) supercell must give the same constant
    lat, pos, kind = S.rocksalt_primitive(2, 3, 2, 5.62)
    q = np.where(kind == 0, 1.0, -1.0)
    V = O.ewald_matrix(lat, pos)
    assert abs(madelung(0.5 * q @ V @ q, 2.81, len(q)) - M_NACL) < 5e-7


@pytest.mark.parametrize("alpha", [0.5, 0.8])
def test_madelung_cscl(alpha):
    a = 4.11
    lat, pos, kind = S.cscl(2, a)
    q = np.where(kind == 0, 1.0, -1.0)
    E = O.ewald_energy(lat, pos, q, alpha)
    assert abs(madelung(E, a * np.sqrt(3) / 2, len(q)) - M_CSCL) < 5e-7


@pytest.mark.parametrize("alpha", [0.4, 1.1])
def test_simple_cubic_single_charge(alpha):
    # a unit charge on a simple-cubic lattice with neutralising background:
    # V_ii L / k_e = -2.837297 (textbook lattice sum)
    L = 3.7
    lat, pos, _ = S.simple_cubic(L)
    V = O.ewald_matrix(lat, pos, alpha)
    assert abs(V[0, 0] * L / KE - (-2.837297)) < 1e-6


def _cfg1_cell():
    c = S.config1()
    return c["lattice"], c["pos"]


def test_alpha_invariance_entrywise():
    lat, pos = _cfg1_cell()
    Vs = [O.ewald_matrix(lat, pos, a, 0, 0) for a in (0.55, 0.75, 1.05)]
    scale = np.abs(Vs[0]).max()
    for V in Vs[1:]:
        assert np.abs(V - Vs[0]).max() < 1e-10 * scale


def test_config1_parameters_converged():
    # the stated config-1 parameters (alpha = 5/L, rc = 10 A, |n| <= 8) against
    # the derived, tighter defaults: the index sphere of radius 8 stops at
    # G^2/(4 alpha^2) ~ 16 along the 4.2 A axis, a truncation near 1e-7 eV per entry
    c = S.config1()
    e = c["ewald"]
    V1 = O.cell_matrix(c)
    V2 = O.ewald_matrix(c["lattice"], c["pos"], e["alpha"])
    assert np.abs(V1 - V2).max() < 2e-7


def test_symmetry_and_constant_diagonal():
    c = S.config2()
    idx = np.r_[0:24, 256:280]
    pos = c["pos"]
    V = O.ewald_matrix(c["lattice"], pos)
    assert np.abs(V - V.T).max() < 1e-13
    d = np.diag(V)
    assert np.ptp(d) < 1e-12


def test_translation_and_wrap_invariance():
    lat, pos = _cfg1_cell()
    V = O.ewald_matrix(lat, pos)
    shifted = pos + np.array([0.37, -1.21, 2.05])
    assert np.abs(O.ewald_matrix(lat, shifted) - V).max() < 1e-11
    wrapped = pos.copy()
    wrapped[5] += lat[0] - 2 * lat[2]
    assert np.abs(O.ewald_matrix(lat, wrapped) - V).max() < 1e-11


def test_scaling_covariance():
    lat, pos = _cfg1_cell()
    lam = 1.37
    V = O.ewald_matrix(lat, pos, 0.75, 9.0, 9)
    Vs = O.ewald_matrix(lat * lam, pos * lam, 0.75 / lam, 9.0 * lam, 9)
    assert np.abs(Vs - V / lam).max() < 1e-12


def test_permutation_covariance():
    lat, pos = _cfg1_cell()
    V = O.ewald_matrix(lat, pos)
    perm = np.random.default_rng(3).permutation(len(pos))
    Vp = O.ewald_matrix(lat, pos[perm])
    assert np.abs(Vp - V[np.ix_(perm, perm)]).max() < 1e-13


@pytest.mark.parametrize("charged", [False, True])
def test_structure_factor_energy_matches_pair_matrix(charged):
    # 1/2 q^T V q against the independent structure-factor form, also for a net
    # charge (the sub-structures of the expansion are charged)
    lat, pos = _cfg1_cell()
    rng = np.random.default_rng(7)
    q = rng.integers(-3, 4, len(pos)).astype(np.float64)
    if not charged:
        q[-1] -= q.sum()
    V = O.ewald_matrix(lat, pos)
    E1 = 0.5 * q @ V @ q
    E2 = O.ewald_energy(lat, pos, q)
    assert abs(E1 - E2) < 1e-11 * max(1.0, abs(E2))


def test_entry_matches_matrix_on_general_cell():
    c = S.config4(n_instances=3, seed=5)[1]
    lat, pos = c["lattice"], c["pos"][:20]
    V = O.ewald_matrix(lat, pos)
    for (i, j) in [(0, 0), (3, 11), (19, 2)]:
        assert O.ewald_entry(lat, pos, i, j) == V[i, j]


def test_defaults_rule():
    a, rc, k = O.ewald_defaults(S.config2()["lattice"])
    assert abs(a - 5 / 16.8) < 1e-15 and abs(rc - 6 / a) < 1e-12 and k == 10
    a, rc, k = O.ewald_defaults(S.config5()["lattice"])
    assert k == 13


@pytest.mark.parametrize("reps", [(2, 2, 1), (2, 2, 2), (3, 2, 1)])
def test_grid_matrix_equals_entry_by_entry(reps):
    """The pair matrix of a rock-salt cell relabelled from its first row equals
    the entry-by-entry matrix (translation invariance of every Ewald entry)."""
    lat, pos, kind = S.rocksalt_conventional(*reps, 4.2)
    cell = S.make_cell(lat, pos, np.where(kind == 0, 0, -1), np.where(kind == 0, 1, 0).astype(np.uint8),
                       [-2.0, 2.0], ["O", "M"])
    full = O.cell_matrix(cell)
    fast = O.grid_matrix(cell)
    assert np.abs(fast - full).max() <= 1e-12 * np.abs(full).max()


def test_grid_matrix_refuses_other_cells():
    lat, pos, kind = S.spinel_primitive(1, 1, 1, 8.1)
    cell = S.make_cell(lat, pos, np.full(len(pos), -1, np.int32), np.zeros(len(pos), np.uint8), [0.0], ["X"])
    with pytest.raises(ValueError):
        O.grid_matrix(cell)
