"""The C ABI library builds, loads and exports every entry point include/goac.h
declares; the Python binding refuses to run without it. No device calls."""
import ctypes
import os
import subprocess
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "goac.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(goac_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    import paper_2409_08808_amd as G
    if not os.path.exists(G.LIB_PATH):
        from paper_2409_08808_amd import _build
        _build.build()
    return G.LIB_PATH


def test_header_declares_the_hot_path():
    syms = declared_symbols()
    for s in ("goac_build_ewald", "goac_energies", "goac_mc_sweep", "goac_ga_generation", "goac_topk_fp64",
              "goac_problem_create", "goac_chains_create", "goac_chains_create_batch", "goac_remc_exchange"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_the_header():
    import paper_2409_08808_amd as G
    assert sorted(G.EXPORTED) == declared_symbols()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2409_08808_amd as G
    monkeypatch.setattr(G, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(G, "_lib", None)
    with pytest.raises(ImportError):
        G.load()


def test_struct_layouts_match_header(tmp_path):
    """The binding's structures have the size and field offsets that a C compiler
    gives the header's."""
    import paper_2409_08808_amd as G
    structs = {"goac_mc_params": G.MCParams, "goac_ga_params": G.GAParams, "goac_ewald_params": G.EwaldParams,
               "goac_hybrid_params": G.HybridParams, "goac_problem_info": G.ProblemInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "goac.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append('printf("goac_chain_stats %zu\\n", sizeof(goac_chain_stats));')
    for f in G.STATS_DTYPE.names:
        lines.append('printf("goac_chain_stats.%s %%zu\\n", offsetof(goac_chain_stats, %s));' % (f, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(py, f).offset, (cname, f)
    assert int(got["goac_chain_stats"]) == G.STATS_DTYPE.itemsize
    for f in G.STATS_DTYPE.names:
        assert int(got["goac_chain_stats.%s" % f]) == G.STATS_DTYPE.fields[f][1], f


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2409_08808_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "goac_oracle" not in text, f
