"""The allocation-free energies entry point (goac_energies_noalloc) against
goac_energies, both through the C ABI: two calls in a row, the second with a
smaller input (fewer rows of a smaller cell), in both precisions, bit for bit
(the same kernels with the same tiles and splits); the mixed result of the small
cell is also within the mixed bound of the oracle. Rows that break the
composition are rejected with the output untouched, and a population whose
scratch exceeds the fixed array is rejected before anything runs."""
import numpy as np
import pytest
import torch

import oracle as O
import supercells as S

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_2409_08808_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G.Context(0)


def _problem(ctx, cell):
    e = cell["ewald"]
    V = ctx.build_ewald(cell["lattice"], cell["pos"], e["alpha"], e["rcut"], e["kmax"])
    return G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_energies_equal_energies(ctx, prec):
    big, small = S.config2(), S.config1()
    pb_big, pb_small = _problem(ctx, big), _problem(ctx, small)
    for pb, P, seed in ((pb_big, 1024, 1), (pb_small, 100, 2)):
        occ = pb.init_occupations(P, seed=seed)
        ref = pb.energies(occ, prec)
        out = torch.full((P,), np.nan, dtype=torch.float64, device="cuda")
        pb.energies_noalloc(occ, prec, out)
        assert torch.equal(out, ref), "P = %d: the allocation-free energies differ" % P
    Vo = O.cell_matrix(small)
    Eo = O.energies(Vo, occ.cpu().numpy(), small["charge"])
    tol = 1e-6 if prec == G.GOAC_FP64 else 1e-4
    assert np.abs(out.cpu().numpy() - Eo).max() / len(small["pos"]) < tol


def test_noalloc_rejects_broken_rows_and_oversized_calls(ctx):
    cell = S.config1()
    pb = _problem(ctx, cell)
    occ = pb.init_occupations(16, seed=3)
    occ[4, 0] = 1 if occ[4, 0].item() == 2 else 2
    out = torch.full((16,), 7.0, dtype=torch.float64, device="cuda")
    for prec in (0, 1):
        with pytest.raises(G.GoacError) as e:
            pb.energies_noalloc(occ, prec, out)
        assert e.value.status == "EINVAL"
        del e
        assert torch.all(out == 7.0)
    # 8x8x8 cell, 1024 FP64 rows: Q and the field alone take 32 MiB
    pb3 = _problem(ctx, S.config3())
    occ3 = pb3.init_occupations(1024, seed=0)
    out3 = torch.zeros(1024, dtype=torch.float64, device="cuda")
    with pytest.raises(G.GoacError, match="scratch") as e:
        pb3.energies_noalloc(occ3, G.GOAC_FP64, out3)
    assert e.value.status == "EINVAL"
    del e
    # the same rows in the mixed precision fit, and equal goac_energies
    pb3.energies_noalloc(occ3, G.GOAC_MIXED, out3)
    assert torch.equal(out3, pb3.energies(occ3, G.GOAC_MIXED))
