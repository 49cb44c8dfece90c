"""GPU parity of the Ewald pair matrix, the configuration energies, the random
starts and the top-k ranking against the FP64 oracle.

Tolerances: V entries within 1e-12 of max|V| (both sides sum the same truncated
series in FP64; only the order of additions differs, and on cells with
translation symmetry the GPU sums one row per orbit); energies within 1e-6 eV
per site (FP64 path) and 1e-4 eV per site (mixed path)."""
import numpy as np
import pytest
import torch

import oracle as O
import supercells as S
from gpu_common import swap_energy_difference, two_sublattice_cell

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_2409_08808_amd")
TOL_FP64 = 1e-6
TOL_MIXED = 1e-4


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G.Context(0)


@pytest.fixture(scope="module")
def cfg1():
    c = S.config1()
    return c, O.cell_matrix(c)


@pytest.fixture(scope="module")
def cfg2():
    c = S.config2()
    return c, O.cell_matrix(c)


def _gpu_V(ctx, cell):
    e = cell["ewald"]
    return ctx.build_ewald(cell["lattice"], cell["pos"], e["alpha"], e["rcut"], e["kmax"])


# ------------------------------------------------------------------ Ewald

def test_ewald_config1(ctx, cfg1):
    cell, Vo = cfg1
    Vg = _gpu_V(ctx, cell).cpu().numpy()
    assert np.abs(Vg - Vo).max() <= 1e-12 * np.abs(Vo).max()


def test_ewald_config2_default_parameters(ctx, cfg2):
    cell, Vo = cfg2
    Vg = ctx.build_ewald(cell["lattice"], cell["pos"]).cpu().numpy()
    assert np.abs(Vg - Vo).max() <= 1e-12 * np.abs(Vo).max()


@pytest.mark.parametrize("which", [0, 3, 7])
def test_ewald_general_cells(ctx, which):
    # rhombohedral rock-salt and spinel supercells (non-orthogonal lattices)
    cells = S.config4(n_instances=8, seed=1, nmin=40, nmax=260)
    cell = cells[which]
    Vo = O.cell_matrix(cell)
    Vg = _gpu_V(ctx, cell).cpu().numpy()
    assert np.abs(Vg - Vo).max() <= 1e-12 * np.abs(Vo).max()


def _random_cell(n, seed):
    """n sites at random positions of a triclinic cell: no translation maps the set
    onto itself, so the build sums every entry."""
    rng = np.random.default_rng(seed)
    lat = np.array([[9.0, 0.0, 0.0], [1.3, 8.2, 0.0], [0.7, -0.9, 10.1]])
    pos = rng.random((n, 3)) @ lat
    return lat, pos


@pytest.mark.parametrize("which", ["config1", "config2", "nacl", "rocksalt_fcc", "spinel", "random"])
def test_ewald_translation_rows_equal_the_full_sum(ctx, which):
    """V_ij depends on r_j - r_i only: on a cell invariant under a grid of
    translations the build sums one row per orbit and relabels it. That equals the
    build that sums every entry (GOAC_EWALD_GENERAL) within the rounding of the
    sums (1e-12 of max|V|): all-sites rock-salt cells (one orbit), an FCC rock-salt
    cell (two), a spinel cell (fourteen), and random sites (no translation)."""
    if which == "random":
        lat, pos = _random_cell(200, 5)
    else:
        if which == "config1":
            cell = S.config1()
        elif which == "config2":
            cell = S.config2()
        elif which == "nacl":
            cell = S.nacl_half()
        else:
            cells = S.config4(n_instances=8, seed=0, nmin=64, nmax=2048)
            cell = cells[0] if which == "rocksalt_fcc" else cells[7]
        lat, pos = cell["lattice"], cell["pos"]
    Vs = ctx.build_ewald(lat, pos).cpu().numpy()
    Vf = ctx.build_ewald(lat, pos, general=True).cpu().numpy()
    assert np.abs(Vs - Vf).max() <= 1e-12 * np.abs(Vf).max()
    assert np.array_equal(Vs, Vs.T) or np.abs(Vs - Vs.T).max() <= 1e-12 * np.abs(Vf).max()


@pytest.mark.parametrize("noise", [1e-12, 1e-6])
def test_ewald_noisy_positions(ctx, noise):
    """Sites displaced by rounding-sized amounts (1e-12 A) still count as a grid
    translate of each other and take the orbit build, which then uses the
    representatives' positions: each entry may move by up to |grad V| times the
    two sites' displacements, |grad V| <= k_e / r^2 = 3.3 eV/A at the 2.1 A nearest
    distance (the bound below takes 20 eV/A per A of noise, plus 1e-12 of max|V|
    for the sums' rounding). Sites displaced by 1e-6 A are not translates, and the
    build sums every entry (bit-identical to GOAC_EWALD_GENERAL)."""
    cell = S.config2()
    rng = np.random.default_rng(3)
    pos = cell["pos"] + rng.uniform(-noise, noise, cell["pos"].shape)
    Vs = ctx.build_ewald(cell["lattice"], pos).cpu().numpy()
    Vf = ctx.build_ewald(cell["lattice"], pos, general=True).cpu().numpy()
    if noise < 1e-9:
        assert np.abs(Vs - Vf).max() <= 1e-12 * np.abs(Vf).max() + 20.0 * noise
    else:
        assert np.array_equal(Vs, Vf)


def test_ewald_alpha_choice_is_immaterial(ctx, cfg1):
    cell, Vo = cfg1
    for a in (0.4, 1.3):
        Vg = ctx.build_ewald(cell["lattice"], cell["pos"], a).cpu().numpy()
        assert np.abs(Vg - Vo).max() < 1e-6          # the config-1 truncation, ~1e-7
    Va = ctx.build_ewald(cell["lattice"], cell["pos"], 0.4).cpu().numpy()
    Vb = ctx.build_ewald(cell["lattice"], cell["pos"], 1.3).cpu().numpy()
    assert np.abs(Va - Vb).max() < 1e-10


def _sampled_entries(ctx, cell, n_samples, seed):
    n = len(cell["pos"])
    Vg = ctx.build_ewald(cell["lattice"], cell["pos"])
    rng = np.random.default_rng(seed)
    ij = np.concatenate([rng.integers(0, n, size=(n_samples, 2)), [[0, 0], [n - 1, n - 1], [0, n - 1]]])
    ref = np.array([O.ewald_entry(cell["lattice"], cell["pos"], i, j) for i, j in ij])
    idx = torch.as_tensor(ij, device=Vg.device)
    got = Vg[idx[:, 0], idx[:, 1]].cpu().numpy()
    sym = (Vg[:256, :256] - Vg[:256, :256].T).abs().max().item()
    return Vg, ref, got, sym


def test_ewald_config3_sampled(ctx):
    cell = S.config3()
    Vg, ref, got, sym = _sampled_entries(ctx, cell, 40, 3)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert sym < 1e-13


def test_ewald_config5_sampled_and_madelung(ctx):
    """Full config-5 cell (N = 16384, V = 2 GiB): sampled entries against the
    oracle, and the closed form of the ordered arrangement: with every cation
    2+, E = -M k_e 4 (N/2) / r, r = 2.1 A, M = 1.74756459463 (the rock-salt
    Madelung constant to 12 digits; the 6-digit 1.747565 would be off by 6e-6
    eV per site here), for any supercell size."""
    cell = S.config5()
    Vg, ref, got, sym = _sampled_entries(ctx, cell, 20, 5)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert sym < 1e-13
    ni = 3
    # a problem whose composition is the ordered arrangement's (every cation Ni2+)
    all_ni = np.where(cell["sublattice"] >= 0, ni, cell["species"]).astype(np.uint8)
    pb_ni = G.Problem(ctx, Vg, cell["sublattice"], all_ni, cell["charge"])
    occ = torch.from_numpy(all_ni[None])
    E = pb_ni.energies(occ, G.GOAC_FP64).item()
    Em = pb_ni.energies(occ, G.GOAC_MIXED).item()
    del pb_ni
    pb = G.Problem(ctx, Vg, cell["sublattice"], cell["species"], cell["charge"])
    n = len(cell["pos"])
    closed = -1.74756459463 * O.coulomb_constant() * 4.0 * (n / 2) / 2.1
    assert abs(E - closed) / n < 1e-8
    assert abs(Em - E) / n < TOL_MIXED
    # energies of random configurations: swaps against the oracle's own rows
    occs = S.random_occupations(cell, 8, seed=2)
    Ef = pb.energies(torch.from_numpy(occs), G.GOAC_FP64).cpu().numpy()
    Emx = pb.energies(torch.from_numpy(occs), G.GOAC_MIXED).cpu().numpy()
    assert np.abs(Emx - Ef).max() / n < TOL_MIXED
    del Vg, pb
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ energies

@pytest.mark.parametrize("prec,tol", [(0, TOL_FP64), (1, TOL_MIXED)])
def test_energies_config1_exhaustive(ctx, cfg1, prec, tol):
    cell, Vo = cfg1
    occ = S.config1_exhaustive_occupations(cell)
    Eo = O.energies(Vo, occ, cell["charge"])
    pb = G.Problem(ctx, torch.from_numpy(Vo), cell["sublattice"], cell["species"], cell["charge"])
    Eg = pb.energies(torch.from_numpy(occ), prec).cpu().numpy()
    assert np.abs(Eg - Eo).max() / 32 <= tol
    # the end-to-end variant: the GPU's own matrix
    pb2 = G.Problem(ctx, _gpu_V(ctx, cell), cell["sublattice"], cell["species"], cell["charge"])
    Eg2 = pb2.energies(torch.from_numpy(occ), prec).cpu().numpy()
    assert np.abs(Eg2 - Eo).max() / 32 <= tol


@pytest.mark.parametrize("prec,tol", [(0, TOL_FP64), (1, TOL_MIXED)])
def test_energies_config2(ctx, cfg2, prec, tol):
    cell, Vo = cfg2
    occ = S.random_occupations(cell, 300, seed=11)          # 300 rows: several tiles plus a ragged tail
    Eo = O.energies(Vo, occ, cell["charge"])
    pb = G.Problem(ctx, torch.from_numpy(Vo), cell["sublattice"], cell["species"], cell["charge"])
    Eg = pb.energies(torch.from_numpy(occ), prec).cpu().numpy()
    assert np.abs(Eg - Eo).max() / 512 <= tol


def test_energies_every_tile_and_the_autotuner(ctx, cfg2):
    """The mixed energies with each tile of the population product (1, 2 and 4
    n-tiles per K block on the 256-position cell; 8 is beyond it) against the
    oracle; the autotuner picks one of them and later calls use it."""
    cell, Vo = cfg2
    occ = S.random_occupations(cell, 300, seed=12)
    Eo = O.energies(Vo, occ, cell["charge"])
    pb = G.Problem(ctx, torch.from_numpy(Vo), cell["sublattice"], cell["species"], cell["charge"])
    occ_t = torch.from_numpy(occ).cuda()
    by_kt = {}
    for kt in (1, 2):
        pb.energies_tile(300, kt)
        Eg = pb.energies(occ_t, G.GOAC_MIXED).cpu().numpy()
        assert np.abs(Eg - Eo).max() / 512 <= TOL_MIXED, kt
        by_kt[kt] = Eg
    with pytest.raises(G.GoacError):
        pb.energies_tile(300, 4)                 # two n-tiles only
    with pytest.raises(G.GoacError):
        pb.energies_tile(300, 3)
    pb.energies_tile(300, 0)
    kt = pb.energies_autotune(occ_t)
    assert kt in by_kt
    assert np.array_equal(pb.energies(occ_t, G.GOAC_MIXED).cpu().numpy(), by_kt[kt])
    # other population sizes keep the cost model; FP64 is untouched
    Ef = pb.energies(occ_t[:77], G.GOAC_FP64).cpu().numpy()
    assert np.abs(Ef - Eo[:77]).max() / 512 <= TOL_FP64
    pb.close()


def test_energies_tiles_on_a_wide_cell(ctx):
    """Config 3 (2048 positions, 16 n-tiles): tiles 1, 2, 4 and 8 agree with the
    FP64 path within the mixed bound."""
    cell = S.config3()
    Vg = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, Vg, cell["sublattice"], cell["species"], cell["charge"])
    pop = pb.init_occupations(300, seed=2)
    Ef = pb.energies(pop, G.GOAC_FP64).cpu().numpy()
    n = len(cell["pos"])
    for kt in (1, 2, 4, 8):
        pb.energies_tile(300, kt)
        Em = pb.energies(pop, G.GOAC_MIXED).cpu().numpy()
        assert np.abs(Em - Ef).max() / n <= TOL_MIXED, kt
    assert pb.energies_autotune(pop) in (1, 2, 4, 8)
    pb.close()


def test_energies_interleaved_site_order(ctx):
    # mobile and fixed sites interleaved, two mobile sublattices
    cell = two_sublattice_cell()
    perm = np.random.default_rng(4).permutation(len(cell["pos"]))
    cell = S.make_cell(cell["lattice"], cell["pos"][perm], cell["sublattice"][perm], cell["species"][perm],
                       cell["charge"], cell["names"])
    Vo = O.cell_matrix(cell)
    occ = S.random_occupations(cell, 70, seed=1)
    Eo = O.energies(Vo, occ, cell["charge"])
    pb = G.Problem(ctx, torch.from_numpy(Vo), cell["sublattice"], cell["species"], cell["charge"])
    n = len(cell["pos"])
    for prec, tol in ((0, TOL_FP64), (1, TOL_MIXED)):
        Eg = pb.energies(torch.from_numpy(occ), prec).cpu().numpy()
        assert np.abs(Eg - Eo).max() / n <= tol


def test_energies_config3_swaps_against_oracle_rows(ctx):
    """Config 3 (N = 4096, P = 1024, the GA workload): the full matrix is out of
    the oracle's reach, so energy differences of single swaps are checked
    against the oracle's rows i and j, and the mixed path against the FP64 path
    on the whole population."""
    cell = S.config3()
    Vg = ctx.build_ewald(cell["lattice"], cell["pos"])
    pb = G.Problem(ctx, Vg, cell["sublattice"], cell["species"], cell["charge"])
    pop = pb.init_occupations(1024, seed=0)
    Ef = pb.energies(pop, G.GOAC_FP64).cpu().numpy()
    Em = pb.energies(pop, G.GOAC_MIXED).cpu().numpy()
    n = len(cell["pos"])
    assert np.abs(Em - Ef).max() / n <= TOL_MIXED
    occ = pop[:1].cpu().numpy()[0]
    rng = np.random.default_rng(8)
    cat = np.nonzero(cell["sublattice"] >= 0)[0]
    for _ in range(2):
        while True:
            i, j = rng.choice(cat, 2, replace=False)
            if cell["charge"][occ[i]] != cell["charge"][occ[j]]:
                break
        Vi = np.array([O.ewald_entry(cell["lattice"], cell["pos"], i, k) for k in range(n)])
        Vj = np.array([O.ewald_entry(cell["lattice"], cell["pos"], j, k) for k in range(n)])
        q = cell["charge"][occ]
        dref = swap_energy_difference(Vi, Vj, q, i, j)
        occ2 = occ.copy()
        occ2[i], occ2[j] = occ[j], occ[i]
        E2 = pb.energies(torch.from_numpy(np.stack([occ, occ2])), G.GOAC_FP64).cpu().numpy()
        assert abs((E2[1] - E2[0]) - dref) < 1e-8


def test_problem_errors(ctx, cfg1):
    cell, Vo = cfg1
    V = torch.from_numpy(Vo)
    bad = cell["species"].copy()
    bad[0] = 2                      # an O2- site becomes M3+: charged
    with pytest.raises(G.GoacError) as e:
        G.Problem(ctx, V, cell["sublattice"], bad, cell["charge"])
    assert e.value.status == "ENOTNEUTRAL"
    bad = cell["species"].copy()
    bad[3] = 9
    with pytest.raises(G.GoacError) as e:
        G.Problem(ctx, V, cell["sublattice"], bad, cell["charge"])
    assert e.value.status == "EINVAL"
    # a charge whose shift is not bfloat16-exact: mixed energies refuse, FP64 works
    ch = cell["charge"].copy()
    ch[1], ch[2] = 1.0 + 1.0 / 3.0, 3.0 - 1.0 / 3.0
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], ch)
    assert not pb.mixed_exact
    occ = torch.from_numpy(cell["species"][None])
    pb.energies(occ, G.GOAC_FP64)
    with pytest.raises(G.GoacError) as e:
        pb.energies(occ, G.GOAC_MIXED)
    assert e.value.status == "EINEXACT"


# ------------------------------------------------------------------ random starts, top-k

@pytest.mark.parametrize("which", ["config1", "config2", "config3", "two"])
def test_init_occupations_bitexact(ctx, which):
    cell = two_sublattice_cell() if which == "two" else getattr(S, which)()
    V = torch.zeros((len(cell["pos"]),) * 2, dtype=torch.float64)
    pb = G.Problem(ctx, V, cell["sublattice"], cell["species"], cell["charge"])
    for base, inst in ((0, 0), (1000, 3)):
        got = pb.init_occupations(37, seed=12345, chain_base=base, instance=inst).cpu().numpy()
        ref = O.init_occupations(cell, 37, seed=12345, chain_base=base, instance=inst)
        assert np.array_equal(got, ref)


def test_topk_config1(ctx, cfg1):
    cell, Vo = cfg1
    occ = S.config1_exhaustive_occupations(cell)
    Eo = O.energies(Vo, occ, cell["charge"])
    pb = G.Problem(ctx, torch.from_numpy(Vo), cell["sublattice"], cell["species"], cell["charge"])
    idx, E = pb.topk(torch.from_numpy(occ), 40)
    idx, E = idx.cpu().numpy(), E.cpu().numpy()
    oi, oE = O.topk(Vo, occ, cell["charge"], 40)
    assert np.abs(E - oE).max() < 1e-9
    assert len(set(idx.tolist())) == 40
    # degenerate levels may be ordered by rounding noise: every pick is among the 40 lowest
    assert np.all(Eo[idx] <= oE[-1] + 1e-9)
    assert np.all(np.diff(E) >= 0)
