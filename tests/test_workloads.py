"""The seeded input generators produce valid, reproducible meshes."""

import numpy as np

from workloads import config_inputs, disk_mesh, star_mesh


def _vols(m):
    P = m.X[m.elems]
    return np.linalg.det(P[:, 1:] - P[:, :1])


def test_disk_mesh_is_reproducible_and_oriented():
    a = disk_mesh(seed=1001)
    b = disk_mesh(seed=1001)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.elems, b.elems)
    assert np.all(_vols(a) > 0)
    assert 900 <= a.nv <= 1300


def test_star_mesh_area_and_orientation():
    m = star_mesh(12, 3000)
    assert np.all(_vols(m) > 0)
    assert 2000 < m.nv < 4000


def test_c1_config_shapes(c1):
    g = c1["grid"]
    assert (g.N, g.W, g.h) == (32, 65, 1.0 / 32)
    assert c1["f"][0].shape == (65, 65)
