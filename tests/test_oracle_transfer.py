"""Pins for point location, the transfer matrix and D (Section 3.1)."""

import math

import numpy as np
import pytest

from oracle import grid as ogrid, predicates, transfer
from workloads import disk_mesh, grid_for_box, structured_box_mesh, structured_box_mesh_3d


def _int_orient2(a, b, c, scale):
    """Exact orientation on dyadic inputs with Python integers (independent of Fraction)."""
    A = [int(round(v * scale)) for v in a]
    B = [int(round(v * scale)) for v in b]
    C = [int(round(v * scale)) for v in c]
    det = (B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0])
    return (det > 0) - (det < 0)


def test_exact_orientation_on_near_collinear_points():
    rng = np.random.default_rng(0)
    scale = 2.0 ** 62
    cases, ref = [], []
    for _ in range(400):
        a = rng.integers(-2 ** 20, 2 ** 20, size=2) / 2.0 ** 20
        b = rng.integers(-2 ** 20, 2 ** 20, size=2) / 2.0 ** 20
        t = rng.integers(0, 2 ** 10) / 2.0 ** 10
        p = a + t * (b - a)                      # exactly on the line (all values dyadic)
        dp = rng.integers(-2, 3, size=2) * 2.0 ** -60
        p = p + dp
        for q in (p, a + t * (b - a)):
            assert all(float(v * scale).is_integer() for v in q)
            cases.append([a, b, q])
            ref.append(_int_orient2(a, b, q, scale))
    got = predicates.orient_signs(np.array(cases))
    assert np.array_equal(got, np.array(ref, dtype=np.int8))
    assert np.count_nonzero(got == 0) >= 400


def test_locate_bucketed_equals_bruteforce():
    mesh = disk_mesh(seed=7, n_boundary=40, spacing=0.15)
    g = grid_for_box(2, 16, R=1.1)
    bf = transfer.locate_bruteforce(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    bk = transfer.locate(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    assert np.array_equal(bf, bk)
    assert np.count_nonzero(bk >= 0) > 100


def test_node_on_shared_edge_and_vertex_takes_smallest_element():
    # two triangles sharing the edge (0,0)-(1,1); grid nodes hit the edge and the vertices
    X = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    elems = np.array([[0, 1, 2], [0, 2, 3]])
    N, R, c = 2, 1.0, (0.0, 0.0)         # nodes at -1, -0.5, 0, 0.5, 1
    el = transfer.locate(X, elems, 2, N, R, c)
    W = 5
    k = lambda i, j: i + W * j            # x index i, y index j
    assert el[k(2, 2)] == 0               # (0,0): vertex of both
    assert el[k(3, 3)] == 0               # (0.5,0.5): on the shared edge
    assert el[k(3, 2)] == 0               # (0.5,0): edge of triangle 0 only
    assert el[k(2, 3)] == 1               # (0,0.5): edge of triangle 1 only
    assert el[k(4, 4)] == 0 and el[k(2, 4)] == 1
    assert el[k(1, 1)] == -1
    # same answer for the reversed orientation of one element
    el2 = transfer.locate(X, np.array([[0, 2, 1], [0, 2, 3]]), 2, N, R, c)
    assert np.array_equal(el, el2)


def test_grid_coincident_mesh_gives_selection():
    g = grid_for_box(2, 16, R=1.0)
    h = g.h
    lo = ogrid.axis_coords(0.0, g.R, g.N)[4]               # vertex grid starts at node 4
    mesh = structured_box_mesh((lo, lo), h, 8, 8)
    tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    assert tr.inside.size == mesh.nv
    lam = tr.lam
    assert np.all(np.isclose(lam.max(axis=1), 1.0, atol=1e-14, rtol=0))
    assert np.all(np.abs(np.sort(lam, axis=1)[:, :-1]) < 1e-14)
    assert np.allclose(tr.D, 1.0, atol=1e-13, rtol=0)


def test_grid_coincident_mesh_3d_gives_selection():
    g = grid_for_box(3, 8, R=1.0)
    lo = ogrid.axis_coords(0.0, g.R, g.N)[2]
    mesh = structured_box_mesh_3d((lo, lo, lo), g.h, 3, 3, 3)
    tr = transfer.Transfer(mesh.X, mesh.elems, 3, g.N, g.R, g.center)
    assert tr.inside.size == mesh.nv
    assert np.allclose(tr.D, 1.0, atol=1e-13, rtol=0)


def test_linear_reproduction_row_sums_and_bounds(c1):
    m, g = c1["mesh"], c1["grid"]
    tr = transfer.Transfer(m.X, m.elems, 2, g.N, g.R, g.center)
    coef, c0 = np.array([0.3, -1.2]), 0.7
    v = tr.I @ (m.X @ coef + c0)
    pts = tr.node_pts[tr.inside]
    assert np.max(np.abs(v[tr.inside] - (pts @ coef + c0))) < 1e-13   # P1 reproduces linears
    rs = np.asarray(tr.I.sum(axis=1)).ravel()
    assert np.allclose(rs[tr.inside], 1.0, atol=1e-14) and np.all(rs[tr.elem < 0] == 0)   # Lemma IhFD-1(iii)
    assert tr.lam.min() > -1e-14 and tr.lam.max() < 1 + 1e-14                            # Lemma IhFD-1(i)
    assert tr.D[tr.J].min() > 0
    # the Dirichlet vertices of the disk are exactly its 100 boundary points
    assert np.count_nonzero(tr.bnd) == 100
    assert np.allclose(np.linalg.norm(m.X[tr.bnd], axis=1), 1.0)


def test_column_sum_lower_bound_under_grid_condition():
    mesh = disk_mesh(seed=11, n_boundary=24, spacing=0.25)
    d = 2
    tr0 = transfer.Transfer(mesh.X, mesh.elems, 2, 4, 1.0, (0.0, 0.0))
    a_h, hmax = tr0.min_height(), tr0.max_diameter()
    hfd_max = a_h / ((d + 1) * math.sqrt(d))                         # eq. hFD-1
    N = int(math.ceil(1.0 / hfd_max))
    tr = transfer.Transfer(mesh.X, mesh.elems, 2, N, 1.0, (0.0, 0.0))
    assert tr.h <= hfd_max
    bound = a_h / ((d + 1) * math.sqrt(d) * hmax)                    # Thm IhFD (i)
    assert tr.D.min() >= bound
    ItI = (tr.I.T @ tr.I).toarray()
    np.linalg.cholesky(ItI)                                          # full column rank (iii)
