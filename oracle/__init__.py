"""FP64 CPU oracle (ctypes front-end of ``goac_oracle.c``).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` import this package. It shares no code with the HIP
library and never calls it; the product path never calls this.

Every routine is a plain transcription of the definition or of the algorithm's
steps (see the C source for the per-function citations of the paper). Eq. 1's
configuration count is implemented here in Python.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "goac_oracle.c")
_LIB = os.path.join(_HERE, "libgoac_oracle.so")

# Counter tags of the Philox draws (fourth counter word, low byte)
TAG_MC, TAG_INIT, TAG_SEL, TAG_X, TAG_MUT, TAG_REMC = 1, 2, 3, 4, 5, 6


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class ChainStats(C.Structure):
    _fields_ = [("t", C.c_uint64), ("accepts", C.c_uint64), ("updates", C.c_uint64),
                ("hash", C.c_uint64), ("E", C.c_double), ("best_E", C.c_double),
                ("min_margin", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_philox.argtypes = [P, P, P]
        L.or_trial_hash.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.or_trial_hash.restype = C.c_uint64
        L.or_coulomb_constant.restype = C.c_double
        L.or_ewald_defaults.argtypes = [P, P, P, P]
        L.or_ewald_entry.argtypes = [P, P, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_int, P]
        L.or_ewald_matrix.argtypes = [P, C.c_int64, P, C.c_double, C.c_double, C.c_int, P]
        L.or_ewald_energy.argtypes = [P, C.c_int64, P, P, C.c_double, C.c_double, C.c_int]
        L.or_ewald_energy.restype = C.c_double
        L.or_energy_q.argtypes = [P, C.c_int64, P]
        L.or_energy_q.restype = C.c_double
        L.or_energies.argtypes = [P, C.c_int64, C.c_int64, P, P, P]
        L.or_init_occupations.argtypes = [C.c_int64, P, P, C.c_int32, C.c_int64, C.c_uint64,
                                          C.c_uint32, C.c_uint32, P]
        L.or_mc_run.argtypes = [P, C.c_int64, P, P, C.c_int32, C.c_int64, P, P, P, P,
                                C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64,
                                P, C.c_int32, C.c_uint64, P, C.c_int32]
        L.or_gd_run.argtypes = [P, C.c_int64, P, P, C.c_int32, C.c_int64, P, C.c_int64, C.c_double, P, P]
        L.or_remc_exchange.argtypes = [C.c_int32, P, P, P, C.c_uint64, C.c_uint64, C.c_uint32, P]
        L.or_ga_generation.argtypes = [C.c_int64, P, C.c_int32, C.c_int64, P, P, C.c_uint64,
                                       C.c_uint32, C.c_int32, C.c_double, P]
        L.or_topk.argtypes = [P, C.c_int64, C.c_int64, P, P, C.c_int32, P, P]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------- RNG

def philox(ctr, key):
    """Philox4x32-10 of one 4-word counter and 2-word key."""
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox(_p(c), _p(k), _p(out))
    return out


def trial_hash(t, i, j, acc):
    return int(lib().or_trial_hash(t, i, j, acc))


# ---------------------------------------------------------------- Ewald

def coulomb_constant():
    return float(lib().or_coulomb_constant())


def ewald_defaults(lattice, alpha=0.0, rcut=0.0, kmax=0):
    lat = _c(lattice, np.float64).reshape(-1)
    a = np.array([alpha], np.float64)
    r = np.array([rcut], np.float64)
    k = np.array([kmax], np.int32)
    lib().or_ewald_defaults(_p(lat), _p(a), _p(r), _p(k))
    return float(a[0]), float(r[0]), int(k[0])


def ewald_matrix(lattice, pos, alpha=0.0, rcut=0.0, kmax=0):
    """Full n x n FP64 pair matrix V (eV per e^2)."""
    lat = _c(lattice, np.float64).reshape(-1)
    pos = _c(pos, np.float64)
    n = len(pos)
    V = np.zeros((n, n), np.float64)
    rc = lib().or_ewald_matrix(_p(lat), n, _p(pos), alpha, rcut, kmax, _p(V))
    if rc:
        raise ValueError("bad Ewald parameters")
    return V


def ewald_entry(lattice, pos, i, j, alpha=0.0, rcut=0.0, kmax=0):
    lat = _c(lattice, np.float64).reshape(-1)
    pos = _c(pos, np.float64)
    out = np.zeros(1, np.float64)
    if lib().or_ewald_entry(_p(lat), _p(pos), int(i), int(j), alpha, rcut, kmax, _p(out)):
        raise ValueError("bad Ewald parameters")
    return float(out[0])


def ewald_energy(lattice, pos, q, alpha=0.0, rcut=0.0, kmax=0):
    """Ewald energy in the structure-factor form (an independent route to 1/2 q^T V q)."""
    lat = _c(lattice, np.float64).reshape(-1)
    pos = _c(pos, np.float64)
    q = _c(q, np.float64)
    return float(lib().or_ewald_energy(_p(lat), len(pos), _p(pos), _p(q), alpha, rcut, kmax))


def cell_matrix(cell):
    e = cell["ewald"]
    return ewald_matrix(cell["lattice"], cell["pos"], e["alpha"], e["rcut"], e["kmax"])


def grid_matrix(cell):
    """The pair matrix of a cell whose sites fill a whole grid of its lattice (a
    conventional rock-salt supercell: cations and anions together form the simple
    cubic grid of spacing a/2), from one row. Every Ewald entry is a sum over the
    lattice images of r_j - r_i, so it depends only on r_j - r_i modulo the lattice,
    and V_ij = V_0k for the site k at r_0 + r_j - r_i. Row 0 is computed entry by
    entry (the plain definition); the rest is that relabelling. For cells whose
    entry-by-entry matrix takes too long; pinned against it on smaller cells.
    Raises ValueError when the sites are not a whole grid."""
    lat = np.asarray(cell["lattice"], np.float64)
    pos = np.asarray(cell["pos"], np.float64)
    n = len(pos)
    frac = np.linalg.solve(lat.T, pos.T).T % 1.0
    D = np.array([len(np.unique(np.round(frac[:, a] * 2 ** 20).astype(np.int64) % 2 ** 20)) for a in range(3)])
    g = np.round(frac * D).astype(np.int64) % D
    if int(np.prod(D)) != n or np.abs(frac * D - np.round(frac * D)).max() > 1e-6:
        raise ValueError("the sites do not fill a grid of the lattice")
    flat = lambda d: (d[..., 0] * D[1] + d[..., 1]) * D[2] + d[..., 2]
    site_of = np.full(n, -1, np.int64)
    site_of[flat((g - g[0]) % D)] = np.arange(n)
    if (site_of < 0).any():
        raise ValueError("the sites do not fill a grid of the lattice")
    e = cell["ewald"]
    row = np.array([ewald_entry(lat, pos, 0, j, e["alpha"], e["rcut"], e["kmax"]) for j in range(n)])
    V = np.empty((n, n), np.float64)
    for i0 in range(0, n, 512):
        d = (g[None, :, :] - g[i0:i0 + 512, None, :]) % D
        V[i0:i0 + 512] = row[site_of[flat(d)]]
    return V


# ---------------------------------------------------------------- energies

def energy_q(V, q):
    V = _c(V, np.float64)
    q = _c(q, np.float64)
    return float(lib().or_energy_q(_p(V), len(q), _p(q)))


def energies(V, occ, charge):
    V = _c(V, np.float64)
    occ = _c(np.atleast_2d(occ), np.uint8)
    charge = _c(charge, np.float64)
    P, n = occ.shape
    E = np.zeros(P, np.float64)
    lib().or_energies(_p(V), n, P, _p(occ), _p(charge), _p(E))
    return E


# ---------------------------------------------------------------- stochastic routines

def init_occupations(cell, C_, seed, chain_base=0, instance=0):
    sub = _c(cell["sublattice"], np.int32)
    spc = _c(cell["species"], np.uint8)
    n = len(sub)
    occ = np.zeros((C_, n), np.uint8)
    rc = lib().or_init_occupations(n, _p(sub), _p(spc), len(cell["charge"]), C_, seed,
                                   chain_base, instance, _p(occ))
    if rc:
        raise ValueError("bad problem")
    return occ


class MCState:
    """State of C chains: occupations, perm arrays, best occupations and counters."""

    def __init__(self, occ):
        self.occ = _c(occ, np.uint8).copy()
        self.perm = None
        self.best_occ = self.occ.copy()
        self.stats = (ChainStats * len(self.occ))()

    def field(self, name):
        return np.array([getattr(s, name) for s in self.stats])


def mc_reload(state: "MCState", V, charge, occ):
    """Continue the chains of ``state`` from new occupations: counters and trial
    indices kept, energies recomputed, the best replaced where the new occupation
    is strictly lower; the next mc_run rebuilds the position lists."""
    occ = np.asarray(occ, np.uint8)
    E = energies(V, occ, charge)
    for c in range(len(occ)):
        state.stats[c].E = E[c]
        if E[c] < state.stats[c].best_E:
            state.stats[c].best_E = E[c]
            state.best_occ[c] = occ[c]
    state.occ[:] = occ
    state.reload = True
    return state


def mc_run(V, cell, state: MCState, seed, n_trials, kT, block_len, chain_base=0, instance=0,
           kT_row=None):
    """Advance every chain in ``state`` by n_trials trials (resumable)."""
    V = _c(V, np.float64)
    sub = _c(cell["sublattice"], np.int32)
    charge = _c(cell["charge"], np.float64)
    n = len(sub)
    C_ = len(state.occ)
    M = int((sub >= 0).sum())
    init = state.perm is None
    if init:
        state.perm = np.zeros((C_, max(M, 1)), np.int32)
    kT = _c(np.atleast_2d(kT), np.float64)
    nb = kT.shape[1]
    rows = None if kT_row is None else _c(kT_row, np.int32)
    rc = lib().or_mc_run(_p(V), n, _p(sub), _p(charge), len(charge), C_, _p(state.occ),
                         _p(state.perm), _p(state.best_occ), C.cast(state.stats, C.c_void_p),
                         seed, chain_base, instance, n_trials, _p(kT), nb, block_len,
                         None if rows is None else _p(rows),
                         1 if init else (2 if getattr(state, "reload", False) else 0))
    state.reload = False
    if rc:
        raise ValueError("oracle MC failed")
    return state


def gd_run(V, cell, occ, max_steps=1 << 30, tol=1e-9):
    """Best-swap descent of each row of ``occ`` (SI, "Gradient Descent"); returns
    (local minima, swaps taken, energies)."""
    V = _c(V, np.float64)
    sub = _c(cell["sublattice"], np.int32)
    charge = _c(cell["charge"], np.float64)
    occ = _c(np.atleast_2d(occ), np.uint8).copy()
    P, n = occ.shape
    steps = np.zeros(P, np.int64)
    E = np.zeros(P, np.float64)
    rc = lib().or_gd_run(_p(V), n, _p(sub), _p(charge), len(charge), P, _p(occ), max_steps, tol, _p(steps), _p(E))
    if rc:
        raise ValueError("oracle gradient descent failed")
    return occ, steps, E


def remc_exchange(kT_ladder, E, slot, x, seed, group=0):
    kT = _c(kT_ladder, np.float64)
    E = _c(E, np.float64)
    slot = _c(slot, np.int32).copy()
    acc = np.zeros(len(kT), np.uint8)
    lib().or_remc_exchange(len(kT), _p(kT), _p(E), _p(slot), x, seed, group, _p(acc))
    return slot, acc


def ga_generation(cell, pop, E, seed, g, n_elite=8, p_mut=0.2):
    sub = _c(cell["sublattice"], np.int32)
    pop = _c(pop, np.uint8)
    E = _c(E, np.float64)
    P, n = pop.shape
    out = np.zeros_like(pop)
    rc = lib().or_ga_generation(n, _p(sub), len(cell["charge"]), P, _p(pop), _p(E), seed, g,
                                n_elite, p_mut, _p(out))
    if rc:
        raise ValueError("oracle GA failed (%d)" % rc)
    return out


def topk(V, occ, charge, k):
    V = _c(V, np.float64)
    occ = _c(np.atleast_2d(occ), np.uint8)
    charge = _c(charge, np.float64)
    P, n = occ.shape
    kk = min(k, P)
    idx = np.zeros(kk, np.int64)
    E = np.zeros(kk, np.float64)
    lib().or_topk(_p(V), n, P, _p(occ), _p(charge), k, _p(idx), _p(E))
    return idx, E


def hybrid_round(V, cell, state, slot, pop, r, R, kT, trials, exchanges, generations, n_elite, p_mut, seed,
                 inject):
    """One round of the replica-exchange + GA hybrid (SI, "Hybrid Methods": the
    two heuristics run alternately and hand their best solutions on). Reading:
      1. REMC phase: `exchanges` times, every chain runs `trials` trials at the
         temperature of its slot, then one exchange step x = r exchanges + e in
         every group of R consecutive chains;
      2. REMC -> GA: the population becomes the P lowest, by (FP64 energy, index),
         of the population followed by the chains' best occupations;
      3. GA phase: `generations` generations g = r generations + k, each followed
         by FP64 energies of the children;
      4. GA -> REMC: the coldest replica of group k takes the individual of rank
         k mod min(inject, P) (order (E, index)) when that individual is strictly
         lower than the replica's current energy; all chains continue from their
         (possibly new) occupations.
    ``state`` (MCState), ``slot`` (groups x R) and the returned population carry
    over between rounds. Returns (population, its energies, slot)."""
    charge = np.asarray(cell["charge"], np.float64)
    kT = np.asarray(kT, np.float64)
    C = len(state.occ)
    G = C // R
    P = len(pop)
    slot = np.array(slot, np.int32).reshape(G, R)
    for e in range(exchanges):
        rows = np.empty(C, np.int32)
        for g in range(G):
            rows[g * R + slot[g]] = np.arange(R)
        mc_run(V, cell, state, seed=seed, n_trials=trials, kT=kT[:, None], block_len=max(trials, 1),
               kT_row=rows)
        E = state.field("E")
        for g in range(G):
            slot[g], _ = remc_exchange(kT, E[g * R:(g + 1) * R], slot[g], r * exchanges + e, seed, group=g)
    cand = np.concatenate([np.asarray(pop, np.uint8), state.best_occ])
    idx, E = topk(V, cand, charge, P)
    pop = cand[idx]
    for k in range(generations):
        pop = ga_generation(cell, pop, E, seed=seed, g=r * generations + k, n_elite=n_elite, p_mut=p_mut)
        E = energies(V, pop, charge)
    n_inj = max(1, min(inject, P))
    order = np.lexsort((np.arange(P), E))[:n_inj]
    occ = state.occ.copy()
    Ech = state.field("E")
    for g in range(G):
        c = g * R + slot[g][0]
        i = order[g % n_inj]
        if E[i] < Ech[c]:
            occ[c] = pop[i]
    mc_reload(state, V, charge, occ)
    return pop, E, slot


def num_threads():
    return int(lib().or_num_threads())


# ---------------------------------------------------------------- Eq. 1

def log10_configurations(counts_per_site):
    """log10 C of Eq. 1, C = prod_s P_s! / prod_e N_{s,e}!, for per-site lists of
    element counts (a vacancy counts as an element)."""
    tot = 0.0
    for counts in counts_per_site:
        P = sum(counts)
        tot += math.lgamma(P + 1) - sum(math.lgamma(c + 1) for c in counts)
    return tot / math.log(10.0)
