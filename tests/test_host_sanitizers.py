"""Host code under the address and undefined-behaviour sanitizers (CPU only).

* The context lifetime and block cache of the library (csrc/lifetime.h, included
  unchanged) in a host-only program on a stub device: every destroy order of a
  context, a problem and a chain set, cache reuse, the cap, a full device,
  repeated releases and random orders run clean, with no block leaked.
* The same program with the context freed at the caller's release although a
  problem still holds it: the problem's destroy then hands its arena to the freed
  context's cache, and the sanitizer reports that write (the failure the holder
  count prevents).
* The FP64 oracle, rebuilt with the sanitizers, runs each of its routines on small
  inputs, the replica-exchange + GA hybrid round included."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _gcc_lib(name):
    return subprocess.check_output(["gcc", "-print-file-name=" + name], text=True).strip()


@pytest.fixture(scope="module")
def lifetime_exe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("lifetime") / "lifetime_check")
    subprocess.check_call(["g++", "-std=c++17", "-Wall", "-Werror", *SAN, "-o", exe,
                           os.path.join(ROOT, "tests", "host_lifetime", "lifetime_check.cpp")])
    return exe


def test_context_lifetime_every_order(lifetime_exe):
    r = subprocess.run([lifetime_exe], capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "lifetime: ok" in r.stdout


def test_context_freed_under_a_problem_is_caught(lifetime_exe):
    r = subprocess.run([lifetime_exe, "early-free"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "heap-use-after-free" in r.stderr
    assert "BlockCache" in r.stderr and "put" in r.stderr


def test_oracle_routines_under_sanitizers(tmp_path):
    lib = str(tmp_path / "libgoac_oracle_san.so")
    subprocess.check_call(["gcc", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                           "-shared", *SAN, "-o", lib, os.path.join(ROOT, "oracle", "goac_oracle.c"), "-lm"])
    script = textwrap.dedent("""
        import sys
        import numpy as np
        sys.path.insert(0, %r)
        import oracle as O
        import supercells as S
        O._LIB = %r
        O.build = lambda force=False: O._LIB
        cell = S.config1()
        V = O.cell_matrix(cell)
        q = np.asarray(cell["charge"])[cell["species"]]
        O.ewald_energy(cell["lattice"], cell["pos"], q, 0.75, 10.0, 8)
        O.ewald_entry(cell["lattice"], cell["pos"], 3, 17, 0.75, 10.0, 8)
        occ = S.config1_exhaustive_occupations(cell)[::50]
        O.energies(V, occ, cell["charge"])
        O.topk(V, occ, cell["charge"], 7)
        occ0 = O.init_occupations(cell, 12, seed=1)
        st = O.MCState(occ0)
        O.mc_run(V, cell, st, seed=2, n_trials=3000, kT=[[0.05, 0.01], [0.4, 0.2]], block_len=1000,
                 kT_row=np.arange(12) %% 2)
        O.mc_reload(st, V, cell["charge"], O.init_occupations(cell, 12, seed=5))
        O.mc_run(V, cell, st, seed=2, n_trials=500, kT=[0.05], block_len=100)
        O.gd_run(V, cell, occ0[:4])
        O.remc_exchange([0.05, 0.1, 0.2, 0.4, 0.8], np.arange(5.0), np.arange(5), 3, 7)
        pop = O.init_occupations(cell, 16, seed=9)
        O.ga_generation(cell, pop, O.energies(V, pop, cell["charge"]), seed=1, g=0, n_elite=2, p_mut=0.5)
        slot = np.tile(np.arange(4, dtype=np.int32), (3, 1))
        st = O.MCState(occ0)
        for r in range(2):
            pop, E, slot = O.hybrid_round(V, cell, st, slot, pop, r, 4, [0.05, 0.1, 0.2, 0.4], trials=200,
                                          exchanges=2, generations=2, n_elite=2, p_mut=0.3, seed=4, inject=2)
        two = S.make_cell(*S.rocksalt_conventional(1, 1, 1, 4.2)[:2], np.array([0] * 4 + [1] * 4, np.int32),
                          np.array([0, 0, 1, 1, 2, 2, 3, 3], np.uint8), [1.0, 3.0, -1.0, -3.0],
                          ["A", "B", "C", "D"])
        O.ga_generation(two, O.init_occupations(two, 6, seed=1), np.linspace(0, 1, 6), seed=3, g=1)
        print("oracle: ok")
    """) % (ROOT, lib)
    env = dict(os.environ, LD_PRELOAD=_gcc_lib("libasan.so") + ":" + _gcc_lib("libubsan.so"),
               ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
