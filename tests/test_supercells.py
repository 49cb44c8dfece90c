"""Geometry and composition checks of the seeded input generator."""
import numpy as np

import supercells as S


def _min_image_dists(lat, pos, i):
    inv = np.linalg.inv(lat)
    d = pos - pos[i]
    f = d @ inv
    f -= np.round(f)
    return np.linalg.norm(f @ lat, axis=1)


def test_spinel_coordination():
    a = 8.1
    lat, pos, kind = S.spinel_primitive(2, 2, 2, a)
    assert [(kind == k).sum() for k in range(3)] == [16, 32, 64]
    tol = 1e-9
    for i in np.nonzero(kind == 0)[0][:4]:
        d = _min_image_dists(lat, pos, i)
        assert ((np.abs(d - a * np.sqrt(3) / 8) < tol) & (kind == 2)).sum() == 4
    for i in np.nonzero(kind == 1)[0][:4]:
        d = _min_image_dists(lat, pos, i)
        assert ((np.abs(d - a / 4) < tol) & (kind == 2)).sum() == 6
    for i in np.nonzero(kind == 2)[0][:4]:
        d = _min_image_dists(lat, pos, i)
        near = d < a / 4 + tol
        assert (near & (kind == 0)).sum() == 1 and (near & (kind == 1)).sum() == 3
    for i in range(len(pos)):
        d = _min_image_dists(lat, pos, i)
        d[i] = np.inf
        assert d.min() > 1.7


def test_rocksalt_nearest_neighbours():
    lat, pos, kind = S.rocksalt_primitive(3, 2, 2, 4.2)
    for i in range(len(pos)):
        d = _min_image_dists(lat, pos, i)
        d[i] = np.inf
        assert abs(d.min() - 2.1) < 1e-9
        assert np.all(kind[np.abs(d - 2.1) < 1e-9] != kind[i])


def test_config_compositions_neutral():
    for cell in [S.config1(), S.config2(), S.config3(), S.config5(), S.nacl_half()] + S.config4(8):
        q = cell["charge"][cell["species"]]
        assert abs(q.sum()) < 1e-9
    c3 = S.composition(S.config3())[0]
    assert c3 == {1: 369, 2: 369, 3: 369, 4: 369, 5: 368, 6: 102, 7: 102}
    assert S.composition(S.config2())[0] == {1: 128, 2: 32, 3: 64, 4: 32}


def test_config4_sizes():
    cells = S.config4()
    N = np.array([len(c["pos"]) for c in cells])
    assert len(cells) == 512 and N.min() >= 28 and N.max() <= 2300
    # log-uniform target between 64 and 2048
    assert 0.2 < np.mean(N < 362) < 0.8


def test_exhaustive_occupations():
    occ = S.config1_exhaustive_occupations()
    assert occ.shape == (12870, 32)
    assert len({r.tobytes() for r in occ}) == 12870
    assert np.all((occ[:, :16] == 1).sum(1) == 8)
    assert np.all(occ[:, 16:] == 0)
    assert list(occ[0, :16]) == [1] * 8 + [2] * 8
