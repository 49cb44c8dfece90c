"""The C ABI library builds, loads and exports every entry point include/goac.h
declares; the Python binding refuses to run without it. No device calls."""
import ctypes
import os
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


def test_struct_layouts_match_header():
    import paper_2409_08808_amd as G
    assert ctypes.sizeof(G.MCParams) == 56
    assert ctypes.sizeof(G.GAParams) == 24
    assert ctypes.sizeof(G.EwaldParams) == 24
    assert G.STATS_DTYPE.itemsize == 72


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2409_08808_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "goac_oracle" not in text, f
