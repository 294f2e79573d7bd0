"""Pins for the GoFD operator, the solve, the preconditioner and the exact solutions."""

import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import afd, exact, fdweights as fw, grid as ogrid, operator, precond, solve, transfer
from workloads import disk_mesh, grid_for_box, structured_box_mesh


@pytest.fixture(scope="module")
def c1_setup(c1):
    m, g = c1["mesh"], c1["grid"]
    tr = transfer.Transfer(m.X, m.elems, 2, g.N, g.R, g.center)
    T = fw.filon_richardson(0.5, 2, 2 * g.N, 1024)
    return tr, T


def test_transfer_back_preserves_constants(c1_setup):
    tr, _ = c1_setup
    ones = np.ones(tr.W ** 2)
    assert np.allclose((tr.I.T @ ones) / tr.D, 1.0, rtol=1e-14)            # remark after eq. Ah-1


def test_grid_coincident_K_is_interior_block_of_AFD():
    g = grid_for_box(2, 16, R=1.0)
    lo = ogrid.axis_coords(0.0, g.R, g.N)[3]
    mesh = structured_box_mesh((lo, lo), g.h, 10, 10, flip=True)
    tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    T = fw.filon_richardson(0.6, 2, 2 * g.N, 256)
    K = operator.dense_K(tr, T)
    A = afd.dense(T, 2, g.W)
    # node number of each interior vertex
    node_of_vertex = np.empty(mesh.nv, dtype=np.int64)
    for row, k in enumerate(tr.inside):
        node_of_vertex[tr.verts[row][np.argmax(tr.lam[row])]] = k
    nodes = node_of_vertex[tr.J]
    assert np.max(np.abs(K - A[np.ix_(nodes, nodes)])) < 1e-13            # GoFD reduces to eq. FD-1


def test_Ah_similar_to_spd():
    mesh = disk_mesh(seed=3, n_boundary=20, spacing=0.3)
    g = grid_for_box(2, 16, R=1.1)
    tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    T = fw.filon_richardson(0.5, 2, 2 * g.N, 256)
    Ah = operator.dense_Ah(tr, T)
    r = 1 / np.sqrt(tr.D)
    At = r[:, None] * (tr.I.T.toarray() @ afd.dense(T, 2, g.W) @ tr.I.toarray()) * r[None, :]
    assert np.allclose(At, At.T, atol=1e-14)
    e1 = np.sort(np.linalg.eigvals(Ah).real)
    e2 = np.linalg.eigvalsh(At)
    assert e2[0] > 0                                                         # Thm Ah-1
    assert np.allclose(e1, e2, rtol=1e-9, atol=1e-12)
    u = np.random.default_rng(0).standard_normal(mesh.nv)
    assert np.allclose(operator.apply_Ah(tr, T, u, "direct"), Ah @ u, atol=1e-13)
    assert np.allclose(operator.apply_Ah(tr, T, u, "fft"), Ah @ u, atol=1e-13)
    assert np.allclose(operator.apply_Ah_sym(tr, T, u), At @ u, atol=1e-13)


def test_solvers_agree(c1_setup):
    tr, T = c1_setup
    f = np.ones((tr.W, tr.W))
    K = operator.dense_K(tr, T)
    b = operator.rhs_grid(tr, 0.5, f)
    x = solve.solve_dense(K, b)
    xc, it0, _ = solve.pcg(lambda v: K @ v, b, tol=1e-13)
    A9 = precond.Ah_pattern(tr, T, 9)
    L9, a9 = precond.ic1(A9)
    x9, it9, _ = solve.pcg(lambda v: K @ v, b, tol=1e-13, precond=lambda r: precond.apply_ic(L9, r))
    A5 = precond.Ah_pattern(tr, T, 5)
    L5, a5 = precond.ic1(A5)
    x5, it5, _ = solve.pcg(lambda v: K @ v, b, tol=1e-13, precond=lambda r: precond.apply_ic(L5, r))
    for y in (xc, x9, x5):
        assert np.max(np.abs(y - x)) < 1e-11 * np.max(np.abs(x))
    assert it9 <= it5 < it0                                                  # Example 1 (qualitative)


def test_ic1_defining_properties(c1_setup):
    tr, T = c1_setup
    A = precond.Ah_pattern(tr, T, 9)
    L, alpha = precond.ic1(A)
    assert alpha == 0.0
    LLt = (L @ L.T).tocoo()
    Lc = L.tocoo()
    Ad = A.toarray()
    M = LLt.toarray()
    # (L L^T)_ij = a_ij on the kept (lower) pattern
    assert np.max(np.abs(M[Lc.row, Lc.col] - Ad[Lc.row, Lc.col])) < 1e-12 * np.abs(Ad).max()
    # the kept pattern contains the lower pattern of A
    Al = sp.tril(A).tocsr()
    Al.data[:] = 1
    Lp = L.copy()
    Lp.data[:] = 1
    assert (Al - Al.multiply(Lp)).nnz == 0


def test_ic1_pattern_on_five_point_laplacian():
    # textbook case: natural ordering of an n x n 5-point Laplacian, level-1 fill
    # adds exactly the (i, i-n+1) entries to the lower factor
    n = 6
    lap1 = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(n, n))
    A = (sp.kron(sp.eye(n), lap1) + sp.kron(lap1, sp.eye(n))).tocsr()
    rows = precond.ic1_pattern(A, 1)
    for i, r in enumerate(rows):
        x, y = i % n, i // n
        want = {i}
        if x > 0:
            want.add(i - 1)
        if y > 0:
            want.add(i - n)
            if x < n - 1:
                want.add(i - n + 1)
        assert set(r) == want
    rows0 = precond.ic1_pattern(A, 0)
    assert all(set(r) == set(sp.tril(A).tocsr()[i].indices) for i, r in enumerate(rows0))


def test_preconditioner_more_effective_as_s_grows():
    mesh = disk_mesh(seed=5, n_boundary=60, spacing=0.09)
    g = grid_for_box(2, 48, R=1.1)
    tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    ratio = {}
    for s in (0.3, 0.9):
        T = fw.filon_richardson(s, 2, 2 * g.N, 512)
        K = operator.dense_K(tr, T)
        b = operator.rhs_grid(tr, s, np.ones((g.W, g.W)))
        _, it0, _ = solve.pcg(lambda v: K @ v, b, tol=1e-10)
        L, _ = precond.ic1(precond.Ah_pattern(tr, T, 9))
        _, it1, _ = solve.pcg(lambda v: K @ v, b, tol=1e-10, precond=lambda r: precond.apply_ic(L, r))
        ratio[s] = it0 / it1
    assert ratio[0.9] > ratio[0.3] > 1.0


def test_closed_form_constants():
    # f = 1 on the unit ball: u(0) = Gamma(d/2) / (2^{2s} Gamma(1+s) Gamma(d/2+s))
    assert exact.u_ball_unit_rhs(np.zeros(2), 0.5, 2) == pytest.approx(2 / math.pi, rel=1e-15)
    assert exact.u_ball_unit_rhs(np.zeros(3), 0.5, 3) == pytest.approx(0.5, rel=1e-15)
    # k = 0: f is the constant 2^{2s} Gamma(1+s) Gamma(d/2+s) / Gamma(d/2), u = (1-|x|^2)^s
    x = np.array([[0.3, 0.4], [0.0, 0.9]])
    f0 = exact.f_ball(x, 0.7, 2, 0)
    assert np.allclose(f0, f0[0]) and np.allclose(exact.u_ball(x, 0.7, 2, 0) / f0[0],
                                                  exact.u_ball_unit_rhs(x, 0.7, 2))


def test_mass_matrix_integrates_constants(c1):
    m = c1["mesh"]
    M = exact.mass_matrix(m.X, m.elems)
    area = np.abs(np.linalg.det(m.X[m.elems][:, 1:] - m.X[m.elems][:, :1])).sum() / 2
    assert np.ones(m.nv) @ (M @ np.ones(m.nv)) == pytest.approx(area, rel=1e-13)


def test_disk_solution_converges_at_expected_rate():
    # Example 1: L2 error O(h) for s = 1/2 on quasi-uniform meshes; grid spacing ~ mesh height
    s = 0.5
    errs, hs = [], []
    for nb, sp_, n in ((50, 0.116, 32), (100, 0.058, 64), (200, 0.029, 128)):
        mesh = disk_mesh(seed=21, n_boundary=nb, spacing=sp_)
        g = grid_for_box(2, n, R=1.0)
        tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
        T = fw.filon_richardson(s, 2, 2 * g.N, 1024)
        b = operator.rhs_grid(tr, s, np.ones((g.W, g.W)))
        uJ, _, _ = solve.pcg(lambda v: operator.apply_K(tr, T, v, "fft"), b, tol=1e-12, maxiter=5000)
        u = np.zeros(mesh.nv)
        u[tr.J] = uJ
        errs.append(exact.l2_error(mesh.X, mesh.elems, u - exact.u_ball_unit_rhs(mesh.X, s, 2)))
        hs.append(mesh.ne ** -0.5)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 0.75 < slope < 1.4, (errs, slope)
    assert errs[-1] < errs[0]
