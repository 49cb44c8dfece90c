"""MI355X (gfx950) library for the pairwise Coulomb cluster-expansion optimiser of
Koester, Binninger and Kaghazchi (arXiv 2409.08808): Ewald pair matrix, batched
configuration energies, swap Monte Carlo (Metropolis, annealing, replica
exchange), genetic-algorithm generations and top-k ranking.

This module is a thin ctypes binding over ``libgoac.so`` (C ABI in
``include/goac.h``). torch supplies device memory and the stream; every step of
the computation runs in the library's HIP kernels. Importing it without the
built library raises ImportError: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgoac.so")

GOAC_FP64, GOAC_MIXED = 0, 1
EDRIFT = -6
TRACE_HASH = 1
REMC_GRAPH = 2
MC_TIMING = 4
EWALD_GENERAL = 1

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTNEUTRAL", -5: "EINEXACT",
           -6: "EDRIFT", -7: "ESTATE"}


class GoacError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_STATUS.get(code, "?"), code, msg))
        self.code = code
        self.status = _STATUS.get(code, "?")


class EwaldParams(C.Structure):
    _fields_ = [("alpha", C.c_double), ("rcut", C.c_double), ("kmax", C.c_int32), ("flags", C.c_int32)]


class ProblemInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("M", C.c_int64), ("n_sublattices", C.c_int32), ("n_species", C.c_int32),
                ("E_fixed", C.c_double), ("mixed_exact", C.c_int32), ("reserved", C.c_int32)]


class MCParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_trials", C.c_uint64), ("kT_host", C.c_void_p), ("n_rows", C.c_int32),
                ("n_blocks", C.c_int32), ("block_len", C.c_uint64), ("reanchor_every", C.c_int32),
                ("flags", C.c_uint32), ("variant", C.c_int32), ("reserved", C.c_int32)]


class GAParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("generation", C.c_uint32), ("n_elite", C.c_int32), ("p_mut", C.c_double)]


class HybridParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("round", C.c_uint64), ("trials", C.c_int64), ("kT_host", C.c_void_p),
                ("R", C.c_int32), ("exchanges", C.c_int32), ("generations", C.c_int32), ("n_elite", C.c_int32),
                ("p_mut", C.c_double), ("inject", C.c_int32), ("precision", C.c_int32),
                ("reanchor_every", C.c_int32), ("reserved", C.c_int32)]


# goac_chain_stats
STATS_DTYPE = np.dtype([("t", "<u8"), ("accepts", "<u8"), ("updates", "<u8"), ("hash", "<u8"),
                        ("fallbacks", "<u8"), ("anchors", "<u8"), ("E", "<f8"), ("best_E", "<f8"),
                        ("status", "<i4"), ("row", "<i4")])
assert STATS_DTYPE.itemsize == 72

_lib = None
EXPORTED = ["goac_ctx_create", "goac_ctx_destroy", "goac_last_error", "goac_ctx_synchronize", "goac_build_ewald",
            "goac_problem_create", "goac_problem_destroy", "goac_problem_get_info", "goac_init_occupations",
            "goac_energies", "goac_topk_fp64", "goac_chains_create", "goac_chains_destroy",
            "goac_chains_create_batch", "goac_chains_set_rows", "goac_mc_sweep", "goac_chains_export",
            "goac_remc_exchange", "goac_ga_generation", "goac_gd_run", "goac_chains_load",
            "goac_hybrid_round", "goac_chains_autotune", "goac_remc_run", "goac_ga_run", "goac_energies_tile",
            "goac_energies_autotune", "goac_energies_noalloc", "goac_chains_timing"]


def load():
    """Load libgoac.so (ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgoac.so is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    P, I64, I32, U64, U32 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_uint32
    sig = {
        "goac_ctx_create": ([C.c_int, P, P], I32),
        "goac_ctx_destroy": ([P], None),
        "goac_last_error": ([P], C.c_char_p),
        "goac_ctx_synchronize": ([P], I32),
        "goac_build_ewald": ([P, P, I64, P, P, P], I32),
        "goac_problem_create": ([P, P, I64, P, P, I32, P, P], I32),
        "goac_problem_destroy": ([P], None),
        "goac_problem_get_info": ([P, P], I32),
        "goac_init_occupations": ([P, I64, U64, U32, U32, P], I32),
        "goac_energies": ([P, I64, P, I32, P], I32),
        "goac_energies_noalloc": ([P, I64, P, I32, P], I32),
        "goac_topk_fp64": ([P, I64, P, I32, P, P], I32),
        "goac_chains_create": ([P, I64, P, I32, U32, U32, P], I32),
        "goac_chains_destroy": ([P], None),
        "goac_chains_create_batch": ([P, I32, P, P, I32, P], I32),
        "goac_chains_set_rows": ([P, P], I32),
        "goac_mc_sweep": ([P, P], I32),
        "goac_chains_export": ([P, P, P, P], I32),
        "goac_chains_timing": ([P, P, P, P], I32),
        "goac_remc_exchange": ([P, I32, P, U64, U64, P, P], I32),
        "goac_ga_generation": ([P, I64, P, P, P, P], I32),
        "goac_ga_run": ([P, I64, P, P, P, I32, I32], I32),
        "goac_energies_tile": ([P, I64, I32], I32),
        "goac_energies_autotune": ([P, I64, P, P], I32),
        "goac_gd_run": ([P, I64, P, I64, C.c_double, P, P], I32),
        "goac_chains_load": ([P, P], I32),
        "goac_hybrid_round": ([P, P, I64, P, P, P], I32),
        "goac_chains_autotune": ([P, U64, C.c_double, P, P], I32),
        "goac_remc_run": ([P, I32, P, U64, U64, U64, U64, U32, I32, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _dev(t, dtype, device):
    if not torch.is_tensor(t):
        t = torch.as_tensor(np.asarray(t))
    t = t.to(device=device, dtype=dtype)
    return t.contiguous()


class Context:
    """A library context bound to one HIP device and a torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        L = load()
        self.device = torch.device("cuda", device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = L.goac_ctx_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise GoacError(rc, "context creation failed")
        self._h = h

    def check(self, rc):
        if rc != 0:
            raise GoacError(rc, load().goac_last_error(self._h).decode())

    def synchronize(self):
        self.check(load().goac_ctx_synchronize(self._h))

    def build_ewald(self, lattice, pos, alpha=0.0, rcut=0.0, kmax=0, out=None, general=False):
        """The n x n pair matrix; general=True sums every entry (GOAC_EWALD_GENERAL)."""
        lat = _np(lattice, np.float64).reshape(9)
        pos = _np(pos, np.float64)
        n = len(pos)
        V = out if out is not None else torch.empty((n, n), dtype=torch.float64, device=self.device)
        prm = EwaldParams(alpha, rcut, kmax, EWALD_GENERAL if general else 0)
        self.check(load().goac_build_ewald(self._h, lat.ctypes.data_as(C.c_void_p), n,
                                           pos.ctypes.data_as(C.c_void_p), C.byref(prm), _ptr(V)))
        return V

    def close(self):
        if getattr(self, "_h", None):
            load().goac_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """An optimisation problem (Eq. 2): pair matrix, site classes, composition."""

    def __init__(self, ctx: Context, V, sublattice, species, charge):
        self.ctx = ctx
        V = _dev(V, torch.float64, ctx.device)
        self.n = V.shape[0]
        self.sub = _np(sublattice, np.int32)
        self.species = _np(species, np.uint8)
        self.charge = _np(charge, np.float64)
        h = C.c_void_p()
        ctx.check(load().goac_problem_create(ctx._h, _ptr(V), self.n, self.sub.ctypes.data_as(C.c_void_p),
                                             self.species.ctypes.data_as(C.c_void_p), len(self.charge),
                                             self.charge.ctypes.data_as(C.c_void_p), C.byref(h)))
        self._h = h
        self._info = None

    def info(self):
        """The problem's sizes and fixed-ion energy (the first call waits for the
        stream: the energy is derived on the device)."""
        if self._info is None:
            info = ProblemInfo()
            self.ctx.check(load().goac_problem_get_info(self._h, C.byref(info)))
            self._info = info
        return self._info

    @property
    def M(self):
        return int(self.info().M)

    @property
    def E_fixed(self):
        return float(self.info().E_fixed)

    @property
    def mixed_exact(self):
        return bool(self.info().mixed_exact)

    def init_occupations(self, C_, seed, chain_base=0, instance=0):
        occ = torch.empty((C_, self.n), dtype=torch.uint8, device=self.ctx.device)
        self.ctx.check(load().goac_init_occupations(self._h, C_, seed, chain_base, instance, _ptr(occ)))
        return occ

    def energies(self, occ, precision=GOAC_FP64, out=None):
        occ = _dev(occ, torch.uint8, self.ctx.device)
        P = occ.shape[0]
        E = out if out is not None else torch.empty(P, dtype=torch.float64, device=self.ctx.device)
        self.ctx.check(load().goac_energies(self._h, P, _ptr(occ), precision, _ptr(E)))
        return E

    def energies_noalloc(self, occ, precision, out):
        """goac_energies_noalloc: energies of occ (P x n, device uint8) into out (P
        doubles, device), with no allocation by the library or here."""
        P = occ.shape[0]
        self.ctx.check(load().goac_energies_noalloc(self._h, P, _ptr(occ), precision, _ptr(out)))
        return out

    def energies_tile(self, P, kt):
        """Set the mixed population product's grid setting for P rows (0: the default)."""
        self.ctx.check(load().goac_energies_tile(self._h, P, kt))

    def energies_autotune(self, occ):
        """Time every tile on this population and keep the fastest for its size;
        returns the tile."""
        occ = _dev(occ, torch.uint8, self.ctx.device)
        kt = C.c_int32(0)
        self.ctx.check(load().goac_energies_autotune(self._h, occ.shape[0], _ptr(occ), C.byref(kt)))
        return kt.value

    def topk(self, occ, k):
        occ = _dev(occ, torch.uint8, self.ctx.device)
        P = occ.shape[0]
        idx = torch.empty(k, dtype=torch.int64, device=self.ctx.device)
        E = torch.empty(k, dtype=torch.float64, device=self.ctx.device)
        self.ctx.check(load().goac_topk_fp64(self._h, P, _ptr(occ), k, _ptr(idx), _ptr(E)))
        return idx, E

    def ga_generation(self, pop, E, seed, generation, n_elite=8, p_mut=0.2, out=None):
        pop = _dev(pop, torch.uint8, self.ctx.device)
        E = _dev(E, torch.float64, self.ctx.device)
        P = pop.shape[0]
        o = out if out is not None else torch.empty_like(pop)
        prm = GAParams(seed, generation, n_elite, p_mut)
        self.ctx.check(load().goac_ga_generation(self._h, P, _ptr(pop), _ptr(E), C.byref(prm), _ptr(o)))
        return o

    def ga_run(self, pop, E, seed, generation, generations, n_elite=8, p_mut=0.2, precision=GOAC_MIXED):
        """`generations` generations (indices generation, generation + 1, ...), each
        followed by the children's energies; pop (P x n) and E (P) are device
        tensors updated in place."""
        P = pop.shape[0]
        prm = GAParams(seed, generation, n_elite, p_mut)
        self.ctx.check(load().goac_ga_run(self._h, P, _ptr(pop), _ptr(E), C.byref(prm), generations, precision))
        return pop, E

    def gd_run(self, occ, max_steps=1 << 40, tol=1e-9):
        """Best-swap descent of each row of occ (modified in place, on the device);
        returns (occ, steps, E)."""
        occ = _dev(occ, torch.uint8, self.ctx.device)
        P = occ.shape[0] if occ.dim() > 1 else 1
        steps = torch.empty(P, dtype=torch.int64, device=occ.device)
        E = torch.empty(P, dtype=torch.float64, device=occ.device)
        self.ctx.check(load().goac_gd_run(self._h, P, _ptr(occ), max_steps, tol, _ptr(steps), _ptr(E)))
        return occ, steps, E

    def close(self):
        if getattr(self, "_h", None):
            load().goac_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Chains:
    """A set of swap Monte Carlo chains on one problem or a batch of problems."""

    def __init__(self, problem: Problem | None, occ=None, precision=GOAC_FP64, chain_base=0, instance=0,
                 _handle=None, _ctx=None, _rows_n=None, _keep=None):
        L = load()
        if _handle is not None:
            self._h, self.ctx, self.C, self._n_per, self._keep = _handle, _ctx, _rows_n[0], _rows_n[1], _keep
            return
        self.ctx = problem.ctx
        occ = _dev(occ, torch.uint8, self.ctx.device)
        self.C = occ.shape[0]
        self._n_per = [(self.C, problem.n)]
        self._keep = [problem]
        h = C.c_void_p()
        self.ctx.check(L.goac_chains_create(problem._h, self.C, _ptr(occ), precision, chain_base, instance,
                                            C.byref(h)))
        self._h = h

    @classmethod
    def batch(cls, problems, chains_per_instance, occ, precision=GOAC_FP64):
        """occ: 1-D uint8 tensor holding every chain's start occupation, instance
        after instance (rows of length n_i)."""
        ctx = problems[0].ctx
        occ = _dev(occ, torch.uint8, ctx.device)
        n_inst = len(problems)
        hs = (C.c_void_p * n_inst)(*[p._h.value for p in problems])
        cpi = _np(chains_per_instance, np.int64)
        h = C.c_void_p()
        ctx.check(load().goac_chains_create_batch(hs, n_inst, cpi.ctypes.data_as(C.c_void_p), _ptr(occ),
                                                  precision, C.byref(h)))
        per = [(int(c), p.n) for c, p in zip(cpi, problems)]
        return cls(None, _handle=h, _ctx=ctx, _rows_n=(int(cpi.sum()), per), _keep=list(problems))

    def set_rows(self, rows):
        r = _np(rows, np.int32)
        self.ctx.check(load().goac_chains_set_rows(self._h, r.ctypes.data_as(C.c_void_p)))

    def sweep(self, n_trials, kT, block_len=None, seed=0, reanchor_every=1024, trace=False, variant=0,
              timing=False):
        kT = _np(np.atleast_2d(kT), np.float64)
        rows, nb = kT.shape
        if block_len is None:
            block_len = max(1, int(n_trials))
        prm = MCParams(seed, n_trials, kT.ctypes.data_as(C.c_void_p), rows, nb, block_len, reanchor_every,
                       (TRACE_HASH if trace else 0) | (MC_TIMING if timing else 0), variant, 0)
        self._kT = kT  # the library copies the table before returning; kept for clarity
        self.ctx.check(load().goac_mc_sweep(self._h, C.byref(prm)))

    def timing(self):
        """(Monte Carlo launch seconds, batched anchor seconds, Monte Carlo launches)
        of the sweeps run with timing=True since the last call (waits for them)."""
        mc, an, n = C.c_double(0.0), C.c_double(0.0), C.c_int64(0)
        self.ctx.check(load().goac_chains_timing(self._h, C.byref(mc), C.byref(an), C.byref(n)))
        return mc.value, an.value, n.value

    def export(self, host_stats=True, drift_ok=False, occ=True):
        """(occupations, best occupations, stats) with stats a numpy structured array,
        or, with host_stats=False, the raw uint8 device tensor. The library call
        waits for the copies and raises EDRIFT when a chain's FP32 field has left its
        error bound, unless drift_ok (the copies are made either way; the chains'
        status field says which). occ=False skips the current occupations (None)."""
        tot = sum(c * n for c, n in self._n_per)
        want_occ = occ
        occ = torch.empty(tot, dtype=torch.uint8, device=self.ctx.device) if want_occ else None
        best = torch.empty(tot, dtype=torch.uint8, device=self.ctx.device)
        st = torch.empty(self.C * STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.ctx.device)
        rc = load().goac_chains_export(self._h, _ptr(occ), _ptr(best), _ptr(st))
        if not (drift_ok and rc == EDRIFT):
            self.ctx.check(rc)
        if host_stats:
            self.ctx.synchronize()
            stats = st.cpu().numpy().view(STATS_DTYPE)
        else:
            stats = st
        if len(self._n_per) == 1:
            c, n = self._n_per[0]
            occ, best = (occ.view(c, n) if occ is not None else None), best.view(c, n)
        return occ, best, stats

    def remc_exchange(self, R, kT_ladder, x, seed, slot, acc=None):
        kT = _np(kT_ladder, np.float64)
        self.ctx.check(load().goac_remc_exchange(self._h, R, kT.ctypes.data_as(C.c_void_p), x, seed,
                                                 _ptr(slot), _ptr(acc)))

    def remc_run(self, R, kT_ladder, trials, rounds, x0, seed, slot, trace=False, reanchor_every=1024,
                 graph=False):
        """`rounds` replica-exchange rounds (sweep + exchange step x0 + r), launched
        round after round or, with graph=True, replayed from a captured graph; slot
        is updated in place."""
        kT = _np(kT_ladder, np.float64)
        flags = (TRACE_HASH if trace else 0) | (REMC_GRAPH if graph else 0)
        self.ctx.check(load().goac_remc_run(self._h, R, kT.ctypes.data_as(C.c_void_p), trials, rounds, x0, seed,
                                            flags, reanchor_every, _ptr(slot)))

    def autotune(self, probe_trials=2000, kT=0.05):
        """Pick the fastest launch configuration on a probe sweep (state unchanged);
        returns (threads per chain, chains per compute unit)."""
        wg, pc = C.c_int32(0), C.c_int32(0)
        self.ctx.check(load().goac_chains_autotune(self._h, probe_trials, kT, C.byref(wg), C.byref(pc)))
        return wg.value, pc.value

    def load(self, occ):
        """Continue every chain from new occupations (counters and rows kept)."""
        occ = _dev(occ, torch.uint8, self.ctx.device)
        self.ctx.check(load().goac_chains_load(self._h, _ptr(occ)))

    def hybrid_round(self, slot, pop, R, kT, trials, exchanges, generations, seed, round, n_elite=8, p_mut=0.2,
                     inject=8, precision=GOAC_MIXED, reanchor_every=1024, E_out=None):
        """One REMC + GA hybrid round; pop (P x n, device) and slot are updated in
        place. Returns the energies of the returned population."""
        kT = _np(kT, np.float64)
        P = pop.shape[0]
        E = E_out if E_out is not None else torch.empty(P, dtype=torch.float64, device=pop.device)
        prm = HybridParams(seed, round, trials, kT.ctypes.data_as(C.c_void_p), R, exchanges, generations, n_elite,
                           p_mut, inject, precision, reanchor_every, 0)
        self.ctx.check(load().goac_hybrid_round(self._h, _ptr(slot), P, _ptr(pop), _ptr(E), C.byref(prm)))
        return E

    def close(self):
        if getattr(self, "_h", None):
            load().goac_chains_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
