"""Seeded synthetic ionic supercells: the inputs both the CPU oracle and the HIP
path are fed.

This module holds geometry and composition sampling only. It computes no
energies, no Ewald sums and no Monte Carlo or GA steps, so that neither side of
a parity test can inherit a mistake from it.

A *cell* is a dict with
  lattice     (3, 3) float64, rows are the lattice vectors a1, a2, a3 in Angstrom
  pos         (n, 3) float64 Cartesian positions in Angstrom
  sublattice  (n,)   int32, -1 for a fixed site, else the id of the site class
              whose positions exchange ions (the "site" s of Eq. 1)
  species     (n,)   uint8, species id on each site (the initial occupation)
  charge      (n_species,) float64 valence of each species in units of e
  names       list of species names
  ewald       dict(alpha, rcut, kmax) with 0 meaning "derive it"

Species counts per sublattice follow from ``species``; every occupation a
caller later passes must keep them (constraint (2b) of Eq. 2, the occupancy
targets O_i).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = [
    "rocksalt_conventional", "rocksalt_primitive", "spinel_primitive", "cscl", "simple_cubic",
    "make_cell", "config1", "config2", "config3", "config4", "config5", "nacl_half",
    "config1_exhaustive_occupations", "random_occupations",
    "composition", "cell_volume",
]

# ----------------------------------------------------------------------------------------
# Lattices (geometry only)
# ----------------------------------------------------------------------------------------

# Rock-salt conventional cell in fractions of a: four cation and four anion positions.
_RS_CATION = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], dtype=np.float64)
_RS_ANION = np.array([[.5, 0, 0], [0, .5, 0], [0, 0, .5], [.5, .5, .5]], dtype=np.float64)

# FCC primitive vectors in units of the conventional a.
_FCC_PRIM = np.array([[0, .5, .5], [.5, 0, .5], [.5, .5, 0]], dtype=np.float64)

# Ideal spinel AB2O4 (Fd-3m, origin at a tetrahedral A site, oxygen parameter 3/8):
# representatives of the 8a, 16d and 32e orbits modulo the FCC translations, in
# fractions of the conventional a. Two A, four B and eight O per primitive cell.
_SP_A = np.array([[0, 0, 0], [.25, .25, .25]])
_SP_B = np.array([[5, 5, 5], [3, 7, 1], [7, 1, 3], [1, 3, 7]]) / 8.0
_SP_O = np.array([[3, 3, 3], [5, 1, 7], [1, 7, 5], [7, 5, 1],
                  [1, 5, 3], [7, 7, 7], [5, 3, 1], [3, 1, 5]]) / 8.0


def cell_volume(lattice) -> float:
    return float(abs(np.linalg.det(np.asarray(lattice, dtype=np.float64))))


def _tile(frac_basis, prim, reps):
    """Replicate fractional basis positions (fractions of ``prim`` rows) over an
    n1 x n2 x n3 block; return Cartesian positions and the block index of each."""
    n1, n2, n3 = reps
    out = []
    for i in range(n1):
        for j in range(n2):
            for k in range(n3):
                shift = np.array([i, j, k], dtype=np.float64)
                out.append((frac_basis + shift) @ prim)
    return np.concatenate(out, axis=0)


def rocksalt_conventional(n1, n2, n3, a):
    """Rock-salt (NaCl type) n1 x n2 x n3 conventional supercell. Cation positions
    first, then anions. Returns (lattice, pos, kind) with kind 0 cation, 1 anion."""
    prim = np.eye(3) * a
    cat = _tile(_RS_CATION, prim, (n1, n2, n3))
    an = _tile(_RS_ANION, prim, (n1, n2, n3))
    lattice = np.diag([n1 * a, n2 * a, n3 * a]).astype(np.float64)
    pos = np.concatenate([cat, an])
    kind = np.concatenate([np.zeros(len(cat), np.int32), np.ones(len(an), np.int32)])
    return lattice, pos, kind


def rocksalt_primitive(n1, n2, n3, a):
    """Rock-salt built from FCC primitive cells (2 sites each); the supercell is
    rhombohedral. kind 0 cation, 1 anion."""
    prim = _FCC_PRIM * a
    # fractional (in primitive basis) positions: cation at 0, anion at (1/2,1/2,1/2)
    cat = _tile(np.zeros((1, 3)), prim, (n1, n2, n3))
    an = _tile(np.full((1, 3), 0.5), prim, (n1, n2, n3))
    lattice = prim * np.array([[n1], [n2], [n3]], dtype=np.float64)
    pos = np.concatenate([cat, an])
    kind = np.concatenate([np.zeros(len(cat), np.int32), np.ones(len(an), np.int32)])
    return lattice, pos, kind


def spinel_primitive(n1, n2, n3, a):
    """Ideal spinel from FCC primitive cells (14 sites each). kind 0 = tetrahedral
    8a, 1 = octahedral 16d, 2 = oxygen 32e."""
    prim = _FCC_PRIM * a
    inv = np.linalg.inv(prim)
    blocks, kinds = [], []
    for kd, rep in enumerate((_SP_A, _SP_B, _SP_O)):
        cart = rep * a
        frac = np.mod(cart @ inv, 1.0)          # into the primitive cell
        blocks.append(_tile(frac, prim, (n1, n2, n3)))
        kinds.append(np.full(len(blocks[-1]), kd, np.int32))
    lattice = prim * np.array([[n1], [n2], [n3]], dtype=np.float64)
    return lattice, np.concatenate(blocks), np.concatenate(kinds)


def cscl(n, a):
    """CsCl type: simple cubic a with cation at 0 and anion at the body centre."""
    prim = np.eye(3) * a
    cat = _tile(np.zeros((1, 3)), prim, (n, n, n))
    an = _tile(np.full((1, 3), 0.5), prim, (n, n, n))
    lattice = np.eye(3) * (n * a)
    return lattice, np.concatenate([cat, an]), np.concatenate(
        [np.zeros(len(cat), np.int32), np.ones(len(an), np.int32)])


def simple_cubic(L):
    """One site in a cube of edge L."""
    return np.eye(3) * L, np.zeros((1, 3)), np.zeros(1, np.int32)


# ----------------------------------------------------------------------------------------
# Cells with compositions
# ----------------------------------------------------------------------------------------

def make_cell(lattice, pos, sublattice, species, charge, names, ewald=None):
    sub = np.ascontiguousarray(sublattice, dtype=np.int32)
    spc = np.ascontiguousarray(species, dtype=np.uint8)
    return dict(lattice=np.ascontiguousarray(lattice, dtype=np.float64),
                pos=np.ascontiguousarray(pos, dtype=np.float64),
                sublattice=sub, species=spc,
                charge=np.ascontiguousarray(charge, dtype=np.float64),
                names=list(names),
                ewald=dict(ewald or dict(alpha=0.0, rcut=0.0, kmax=0)))


def composition(cell):
    """{sublattice: {species: count}} of the cell's current occupation."""
    out = {}
    for s, e in zip(cell["sublattice"].tolist(), cell["species"].tolist()):
        if s < 0:
            continue
        out.setdefault(s, {}).setdefault(e, 0)
        out[s][e] += 1
    return out


def _assign(n_sites, counts, rng=None):
    """Species list for n_sites positions from {species: count}; canonical
    (sorted) order unless an rng is given, then a seeded shuffle."""
    arr = np.concatenate([np.full(c, e, np.uint8) for e, c in sorted(counts.items()) if c > 0])
    assert len(arr) == n_sites, (len(arr), n_sites)
    if rng is not None:
        rng.shuffle(arr)
    return arr


def config1():
    """2x2x1 conventional rock-salt cell, a = 4.2 A: 16 fixed O2- plus 16 cation
    positions holding 8 Li+ and 8 M3+. Ewald alpha = 5/L with L = volume^(1/3),
    real-space cutoff 10 A, reciprocal index radius 8."""
    lat, pos, kind = rocksalt_conventional(2, 2, 1, 4.2)
    names = ["O", "Li", "M"]
    charge = [-2.0, 1.0, 3.0]
    sub = np.where(kind == 0, 0, -1)
    spc = np.zeros(len(pos), np.uint8)
    spc[kind == 0] = _assign(16, {1: 8, 2: 8})
    L = cell_volume(lat) ** (1.0 / 3.0)
    return make_cell(lat, pos, sub, spc, charge, names, dict(alpha=5.0 / L, rcut=10.0, kmax=8))


def config1_exhaustive_occupations(cell=None):
    """All C(16,8) = 12870 occupations of config 1, in lexicographic order of the
    8-subset of cation positions that hold Li (rows are full-site occupations)."""
    cell = cell or config1()
    cat = np.nonzero(cell["sublattice"] >= 0)[0]
    base = cell["species"].copy()
    rows = []
    for subset in itertools.combinations(range(len(cat)), 8):
        occ = base.copy()
        occ[cat] = 2
        occ[cat[list(subset)]] = 1
        rows.append(occ)
    return np.stack(rows)


def config2():
    """4x4x4 conventional rock-salt (16.8 A cube), N = 512: 256 fixed O2- and 256
    cation positions with Li+ 128, Ni2+ 32, Co3+ 64, Mn4+ 32."""
    lat, pos, kind = rocksalt_conventional(4, 4, 4, 4.2)
    names = ["O", "Li", "Ni", "Co", "Mn"]
    charge = [-2.0, 1.0, 2.0, 3.0, 4.0]
    sub = np.where(kind == 0, 0, -1)
    spc = np.zeros(len(pos), np.uint8)
    spc[kind == 0] = _assign(256, {1: 128, 2: 32, 3: 64, 4: 32})
    return make_cell(lat, pos, sub, spc, charge, names)


def config3():
    """8x8x8 conventional rock-salt, N = 4096: 2048 O2- fixed; cations Mg/Co/Ni/Cu/Zn
    369/369/369/369/368 plus 102 Li+ and 102 Ga3+ (5 % of the positions replaced by
    charge-neutral Li/Ga pairs)."""
    lat, pos, kind = rocksalt_conventional(8, 8, 8, 4.2)
    names = ["O", "Mg", "Co", "Ni", "Cu", "Zn", "Li", "Ga"]
    charge = [-2.0, 2.0, 2.0, 2.0, 2.0, 2.0, 1.0, 3.0]
    sub = np.where(kind == 0, 0, -1)
    spc = np.zeros(len(pos), np.uint8)
    spc[kind == 0] = _assign(2048, {1: 369, 2: 369, 3: 369, 4: 369, 5: 368, 6: 102, 7: 102})
    return make_cell(lat, pos, sub, spc, charge, names)


def _near_cubic_reps(target_cells):
    """Integer n1 <= n2 <= n3 balancing the product against target_cells and the
    shape: minimise |ln(n1 n2 n3 / target)| + ln(n3 / n1) / 2 (ties broken by
    lexicographic order), so that cells stay near-cubic in the lattice basis."""
    best = None
    hi = max(2, int(round(target_cells ** (1 / 3))) * 2 + 2)
    for n1 in range(1, hi + 1):
        for n2 in range(n1, hi + 1):
            for n3 in range(n2, hi + 1):
                p = n1 * n2 * n3
                if p > 2 * target_cells + 2:
                    break
                cost = abs(math.log(p / target_cells)) + 0.5 * math.log(n3 / n1)
                key = (round(cost, 12), (n1, n2, n3))
                if best is None or key < best:
                    best = key
    return best[1]


def config4(n_instances=512, seed=0, nmin=64, nmax=2048):
    """512 uneven instances: rock-salt (a = 4.2 A, 2 sites per primitive cell) or
    spinel (a = 8.1 A, 14 sites per primitive cell) with probability 1/2 each, target
    N log-uniform on [nmin, nmax] (numpy PCG64 seed 0). Rock-salt cations: Ni2+ plus
    a seeded fraction of Li+/Co3+ pairs; spinel cations: 2+ and 3+ in 1:2 on one
    8a+16d sublattice."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cells = []
    for _ in range(n_instances):
        spinel = bool(rng.random() < 0.5)
        target = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        per = 14 if spinel else 2
        reps = _near_cubic_reps(max(1, target / per))
        if spinel:
            lat, pos, kind = spinel_primitive(*reps, 8.1)
            names = ["O", "Mg", "Al"]
            charge = [-2.0, 2.0, 3.0]
            sub = np.where(kind < 2, 0, -1)
            spc = np.zeros(len(pos), np.uint8)
            ncat = int((kind < 2).sum())
            spc[kind < 2] = _assign(ncat, {1: ncat // 3, 2: 2 * ncat // 3}, rng)
        else:
            lat, pos, kind = rocksalt_primitive(*reps, 4.2)
            names = ["O", "Ni", "Li", "Co"]
            charge = [-2.0, 2.0, 1.0, 3.0]
            sub = np.where(kind == 0, 0, -1)
            spc = np.zeros(len(pos), np.uint8)
            ncat = int((kind == 0).sum())
            frac = rng.uniform(0.1, 0.5)
            pairs = max(1, int(round(frac * ncat / 2)))
            spc[kind == 0] = _assign(ncat, {1: ncat - 2 * pairs, 2: pairs, 3: pairs}, rng)
        cells.append(make_cell(lat, pos, sub, spc, charge, names))
    return cells


def config5(seed=0):
    """16x16x8 conventional rock-salt (67.2 x 67.2 x 33.6 A), N = 16384, 8192 cation
    positions filled from charge-neutral units drawn with Dirichlet(1) weights
    (PCG64 seed 0): Ni2+, Li+ + Co3+, Na+ + Co3+, 2 Li+ + Mn4+, 2 Na+ + Ti4+; the
    remainder is Ni2+."""
    lat, pos, kind = rocksalt_conventional(16, 16, 8, 4.2)
    names = ["O", "Li", "Na", "Ni", "Co", "Mn", "Ti"]
    charge = [-2.0, 1.0, 1.0, 2.0, 3.0, 4.0, 4.0]
    LI, NA, NI, CO, MN, TI = 1, 2, 3, 4, 5, 6
    units = [({NI: 1}, 1), ({LI: 1, CO: 1}, 2), ({NA: 1, CO: 1}, 2),
             ({LI: 2, MN: 1}, 3), ({NA: 2, TI: 1}, 3)]
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.dirichlet(np.ones(len(units)))
    M = int((kind == 0).sum())
    counts = {}
    used = 0
    for (u, size), wt in zip(units, w):
        k = int(wt * M) // size
        for e, c in u.items():
            counts[e] = counts.get(e, 0) + c * k
        used += size * k
    counts[NI] = counts.get(NI, 0) + (M - used)
    sub = np.where(kind == 0, 0, -1)
    spc = np.zeros(len(pos), np.uint8)
    spc[kind == 0] = _assign(M, counts, rng)
    return make_cell(lat, pos, sub, spc, charge, names)


def nacl_half(n=3, a=5.62):
    """NaCl n x n x n conventional cell whose 8 n^3 positions all hold Na+ or Cl-
    at 50/50 on one exchangeable site class (216 positions for n = 3, the count
    whose Eq. 1 value is the 1e64 the paper quotes). The optimum is the
    alternating rock-salt order."""
    lat, pos, kind = rocksalt_conventional(n, n, n, a)
    names = ["Na", "Cl"]
    charge = [1.0, -1.0]
    sub = np.zeros(len(pos), np.int32)
    spc = _assign(len(pos), {0: len(pos) // 2, 1: len(pos) // 2})
    return make_cell(lat, pos, sub, spc, charge, names)


def random_occupations(cell, P, seed):
    """P seeded random occupations with the cell's composition (numpy PCG64); a
    plain input generator, independent of the method's own Fisher-Yates start."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.repeat(cell["species"][None, :], P, axis=0)
    for s in sorted(set(cell["sublattice"].tolist()) - {-1}):
        idx = np.nonzero(cell["sublattice"] == s)[0]
        for p in range(P):
            out[p, idx] = rng.permutation(out[p, idx])
    return out
