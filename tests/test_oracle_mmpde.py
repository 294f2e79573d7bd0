"""Pins of the oracle's mesh adaptation (Section 4): Hessian recovery, the metric of eq. MK-1 and its
regularisation parameter, the energy of eq. I-h and its gradient, and the moving mesh equations."""

import math

import numpy as np
import pytest

from oracle import mmpde
from workloads import disk_mesh


def _lattice(n=8, a=0.2):
    """Equilateral triangle lattice (a rhombus of n x n points)."""
    pts = np.array([[i * a + 0.5 * j * a, j * a * math.sqrt(3) / 2] for j in range(n) for i in range(n)])
    tris = []
    for j in range(n - 1):
        for i in range(n - 1):
            v = j * n + i
            tris += [(v, v + 1, v + n), (v + 1, v + n + 1, v + n)]
    return pts, np.array(tris)


def test_hessian_recovery_is_exact_for_quadratics():
    m = disk_mesh(seed=3, n_boundary=30, spacing=0.15)
    x, y = m.X[:, 0], m.X[:, 1]
    u = 1 + 2 * x - y + 3 * x ** 2 - 2 * x * y + 0.5 * y ** 2
    H = mmpde.vertex_hessians(m.X, m.elems, u)
    assert np.allclose(H, np.array([[6.0, -2.0], [-2.0, 1.0]]), rtol=0, atol=1e-8)
    # linear data: zero Hessian
    assert np.max(np.abs(mmpde.vertex_hessians(m.X, m.elems, 3 * x - y))) < 1e-9


def test_abs_sym_and_metric_closed_form():
    H = np.array([[[-2.0, 0.0], [0.0, 3.0]], [[0.0, 1.0], [1.0, 0.0]]])
    A = mmpde.abs_sym(H)
    assert np.allclose(A[0], np.diag([2.0, 3.0]))
    assert np.allclose(A[1], np.eye(2))                 # eigenvalues +-1 of [[0,1],[1,0]]
    assert np.allclose(A @ A, H @ H)
    alpha = 0.7
    M = mmpde.metric(A, alpha)
    b0 = np.array([1 + 2 / alpha, 1 + 3 / alpha])
    assert np.allclose(M[0], np.diag(b0) * (b0[0] * b0[1]) ** (-1 / 6), rtol=1e-14)
    assert np.allclose(mmpde.metric(A, math.inf), np.eye(2))


def test_alpha_solves_its_equation():
    m = disk_mesh(seed=4, n_boundary=30, spacing=0.15)
    r2 = np.sum(m.X ** 2, axis=1)
    u = np.maximum(1 - r2, 0) ** 0.5
    Hk = mmpde.element_hessians(m.elems, mmpde.vertex_hessians(m.X, m.elems, u))
    A = mmpde.abs_sym(Hk)
    area = mmpde.element_areas(m.X, m.elems)
    alpha = mmpde.alpha_h(A, area)
    lam = np.linalg.eigvalsh(A)
    lhs = np.sum(area * np.prod(1 + lam / alpha, axis=1) ** (1 / 3))
    assert lhs == pytest.approx(2 * np.sum(area), rel=1e-12)
    assert mmpde.alpha_h(np.zeros_like(A), area) == math.inf


def test_energy_of_the_reference_element_and_gradient_by_central_differences():
    # the reference element itself with M = I: J = I, t = 2, both terms (1/3) 2^{3/2} |K|, |K| = 1
    Er = mmpde.reference_edges(2)
    X = np.array([[0.0, 0.0], Er[:, 0], Er[:, 1]])
    assert mmpde.energy(X, np.array([[0, 1, 2]]), np.eye(2)[None]) == pytest.approx(2 / 3 * 2 ** 1.5, rel=1e-14)
    rng = np.random.default_rng(5)
    m = disk_mesh(seed=5, n_boundary=16, spacing=0.35)
    Mk = []
    for _ in range(m.ne):
        Q = rng.standard_normal((2, 2))
        Mk.append(Q @ Q.T + 0.5 * np.eye(2))
    Mk = np.array(Mk)
    G = mmpde.energy_gradient(m.X, m.elems, Mk)
    eps = 1e-6
    for i in rng.choice(m.nv, 8, replace=False):
        for a in range(2):
            Xp, Xm = m.X.copy(), m.X.copy()
            Xp[i, a] += eps
            Xm[i, a] -= eps
            fd = (mmpde.energy(Xp, m.elems, Mk) - mmpde.energy(Xm, m.elems, Mk)) / (2 * eps)
            assert G[i, a] == pytest.approx(fd, rel=1e-6, abs=1e-8 * np.abs(G).max())


def test_uniform_equilateral_mesh_is_an_equilibrium():
    # equal equilateral elements satisfy eqs. C-1 and C-2 for a constant metric: by the six-fold symmetry
    # of the star of an interior vertex its energy gradient vanishes
    X, T = _lattice()
    G = mmpde.energy_gradient(X, T, np.broadcast_to(np.eye(2), (len(T), 2, 2)))
    bnd = mmpde.boundary_mask(T, len(X))
    assert np.max(np.abs(G[~bnd])) < 1e-12 * np.abs(G).max() + 1e-13
    Mc = np.broadcast_to(np.diag([3.0, 3.0]), (len(T), 2, 2))
    G3 = mmpde.energy_gradient(X, T, Mc)
    assert np.max(np.abs(G3[~bnd])) < 1e-12 * np.abs(G3).max() + 1e-13


def _disk_metric(seed, nb, spc):
    m = disk_mesh(seed=seed, n_boundary=nb, spacing=spc)
    r2 = np.sum(m.X ** 2, axis=1)
    u = np.maximum(1 - r2, 0) ** 0.5                 # steep near the boundary
    Hk = mmpde.element_hessians(m.elems, mmpde.vertex_hessians(m.X, m.elems, u))
    A = mmpde.abs_sym(Hk)
    area = mmpde.element_areas(m.X, m.elems)
    return m, mmpde.metric(A, mmpde.alpha_h(A, area)), area


def test_hessian_times_vector_is_the_derivative_of_the_gradient():
    # the assembled element Hessians (differences per element, relative steps) against a central difference
    # of the whole gradient along one random direction with one absolute step
    m, M, _ = _disk_metric(7, 30, 0.15)
    J = mmpde.assemble_hessian(m.elems, mmpde.element_hessians_fd(m.X, m.elems, M), m.nv)
    assert abs(J - J.T).max() <= 1e-15 * abs(J).max()      # symmetric up to the order of the sums
    rng = np.random.default_rng(8)
    v = rng.standard_normal((m.nv, 2))
    eps = 1e-6
    d = (mmpde.energy_gradient(m.X + eps * v, m.elems, M) - mmpde.energy_gradient(m.X - eps * v, m.elems, M)) / (2 * eps)
    Jv = (J @ v.ravel()).reshape(-1, 2)
    assert np.max(np.abs(Jv - d)) <= 1e-6 * np.max(np.abs(d))


def test_short_implicit_step_is_the_explicit_one():
    # for h -> 0 the linearly implicit step tends to h times the right side of eq. x-1
    m, M, _ = _disk_metric(9, 30, 0.15)
    bnd = mmpde.boundary_mask(m.elems, m.nv)
    qv = np.random.default_rng(1).uniform(1.0, 3.0, m.nv)
    G = mmpde.energy_gradient(m.X, m.elems, M)
    J = mmpde.assemble_hessian(m.elems, mmpde.element_hessians_fd(m.X, m.elems, M), m.nv)
    v = mmpde.velocity(m.X, m.elems, M, bnd, qv, 1e-2)
    err = []
    for h in (1e-10, 1e-12):
        Y = mmpde.implicit_step(m.X, bnd, qv, h, G, J)
        err.append(np.max(np.abs((Y - m.X) / h - v)) / np.max(np.abs(v)))
    assert err[1] <= 2e-5 and 50 < err[0] / err[1] < 200          # first order in h


def test_metric_derivatives_by_central_differences():
    m, M, _ = _disk_metric(11, 30, 0.15)
    D = mmpde.metric_derivatives(m.X, m.elems, M)
    el = m.elems
    for k in (0, m.ne // 3, m.ne - 1):
        for c, (i, j) in enumerate(((0, 0), (0, 1), (1, 1))):
            eps = 1e-6 * np.abs(M[k]).max()
            Mp, Mm = M[k:k + 1].copy(), M[k:k + 1].copy()
            Mp[0, i, j] += eps
            Mm[0, i, j] -= eps
            if i != j:
                Mp[0, j, i] += eps
                Mm[0, j, i] -= eps
            fd = (mmpde.energy(m.X, el[k:k + 1], Mp) - mmpde.energy(m.X, el[k:k + 1], Mm)) / (2 * eps)
            assert D[k, c] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(D[k]).max())


def test_metric_field_is_exact_for_linear_fields():
    m = disk_mesh(seed=12, n_boundary=30, spacing=0.15)
    A0, A1, A2 = np.array([[3.0, 0.5], [0.5, 2.0]]), np.array([[0.4, 0.1], [0.1, -0.3]]), np.array([[-0.2, 0.0], [0.0, 0.5]])
    Mv = A0[None] + m.X[:, 0, None, None] * A1[None] + m.X[:, 1, None, None] * A2[None]
    field = mmpde.MetricField(m.X, m.elems, Mv)
    # move every vertex a little: the centroids land in other elements, found by the walks
    rng = np.random.default_rng(13)
    bnd = mmpde.boundary_mask(m.elems, m.nv)
    Y = m.X + np.where(bnd[:, None], 0.0, rng.uniform(-0.06, 0.06, m.X.shape))
    Y = np.where(mmpde.element_areas(Y, m.elems)[:, None].min() > 0, Y, m.X)
    M, G, loc = field.at_centroids(Y, np.arange(m.ne))
    C = Y[m.elems].mean(axis=1)
    expect = A0[None] + C[:, 0, None, None] * A1[None] + C[:, 1, None, None] * A2[None]
    assert np.allclose(M, expect, rtol=0, atol=1e-13)
    assert np.allclose(G[:, 0], [A1[0, 0], A2[0, 0]], atol=1e-12) and np.allclose(G[:, 1], [A1[0, 1], A2[0, 1]], atol=1e-12)
    for k in range(m.ne):          # each centroid lies in the element the walk returned
        assert np.all(mmpde.barycentric(m.X, m.elems, loc[k], C[k]) >= -1e-12)
    assert np.any(loc != np.arange(m.ne))


def test_field_energy_gradient_by_central_differences():
    m = disk_mesh(seed=14, n_boundary=30, spacing=0.15)
    r2 = np.sum(m.X ** 2, axis=1)
    Mv, _ = mmpde.level_metric(m.X, m.elems, np.maximum(1 - r2, 0) ** 0.5)
    field = mmpde.MetricField(m.X, m.elems, Mv)
    rng = np.random.default_rng(15)
    X = m.X + 0.02 * rng.standard_normal(m.X.shape)        # off the starting mesh: centroids inside elements
    loc0 = field.at_centroids(X, np.arange(m.ne))[2]
    _, G, _, _ = mmpde.energy_field(X, m.elems, field, loc0)
    eps = 1e-7
    for i in rng.choice(m.nv, 8, replace=False):
        for a in range(2):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, a] += eps
            Xm[i, a] -= eps
            Ip, _, _, lp = mmpde.energy_field(Xp, m.elems, field, loc0)
            Im, _, _, lm = mmpde.energy_field(Xm, m.elems, field, loc0)
            assert np.array_equal(lp, loc0) and np.array_equal(lm, loc0)
            assert G[i, a] == pytest.approx((Ip - Im) / (2 * eps), rel=1e-5, abs=1e-7 * np.abs(G).max())


def test_moving_the_mesh_equidistributes_the_metric():
    m = disk_mesh(seed=6, n_boundary=40, spacing=0.1)
    r2 = np.sum(m.X ** 2, axis=1)
    Mv, _ = mmpde.level_metric(m.X, m.elems, np.maximum(1 - r2, 0) ** 0.5)     # steep near the boundary
    bnd = mmpde.boundary_mask(m.elems, m.nv)
    Y, steps, info = mmpde.move_mesh(m.X, m.elems, Mv, bnd)
    assert steps > 5
    assert info["grad"] <= 1e-3 * info["grad0"]
    assert np.all(mmpde.element_areas(Y, m.elems) > 0)
    assert np.allclose(np.linalg.norm(Y[bnd], axis=1), 1.0, atol=1e-14)
    assert info["energy_end"] < info["energy_start"]
    # sqrt(det M_K) |K| evens out (eq. C-1) and elements near the boundary shrink, those in the middle grow
    field = mmpde.MetricField(m.X, m.elems, Mv)
    spread = []
    for Z in (m.X, Y):
        M, _, _ = field.at_centroids(Z, np.arange(m.ne))
        w = np.sqrt(np.linalg.det(M)) * mmpde.element_areas(Z, m.elems)
        spread.append(w.std() / w.mean())
    assert spread[1] < 0.6 * spread[0]
    cen0 = m.X[m.elems].mean(axis=1)
    near = np.linalg.norm(cen0, axis=1) > 0.85
    a0, a1 = mmpde.element_areas(m.X, m.elems), mmpde.element_areas(Y, m.elems)
    assert a1[near].mean() < 0.7 * a0[near].mean() and a1[~near].mean() > a0[~near].mean()


def test_fixed_boundary_stays():
    m = disk_mesh(seed=10, n_boundary=30, spacing=0.15)
    r2 = np.sum(m.X ** 2, axis=1)
    Mv, _ = mmpde.level_metric(m.X, m.elems, np.maximum(1 - r2, 0) ** 0.5)
    bnd = mmpde.boundary_mask(m.elems, m.nv)
    Y, steps, info = mmpde.move_mesh(m.X, m.elems, Mv, bnd, max_steps=5, boundary="fixed")
    assert steps == 5 and np.array_equal(Y[bnd], m.X[bnd]) and not np.array_equal(Y, m.X)
    assert info["energy_end"] < info["energy_start"]
