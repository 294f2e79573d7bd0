"""MMPDE mesh adaptation on the GPU (Section 4, Algorithm amGoFD) against the oracle: the recovered
Hessians, the metric of eq. MK-1 and alpha_h, the energy of eq. I-h and its gradient, fixed explicit
steps and the step-controlled integration of eq. x-1; then Algorithm amGoFD itself on the unit disk
(Example 1, k = 0, s = 0.5), where the L2 error on adaptive meshes falls faster than on fixed ones."""

import math

import numpy as np
import pytest

from oracle import exact, grid as ogrid, mmpde
from workloads import disk_mesh, grid_for_box

pytestmark = pytest.mark.gpu


def _dev(a, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def _mm(gctx, m):
    import torch
    import paper_2307_14437_amd as gofd
    return gofd.Mmpde(gctx, m.nv, _dev(m.elems, torch.int32))


def _sym3(H):
    """N x 2 x 2 -> N x 3 (h11, h12, h22)."""
    return np.stack([H[:, 0, 0], H[:, 0, 1], H[:, 1, 1]], axis=1)


def _u(X):
    r2 = np.sum(X ** 2, axis=1)
    return np.maximum(1 - r2, 0) ** 0.5 + 0.3 * np.sin(3 * X[:, 0]) * X[:, 1]


def _mat(M3):
    """N x 3 (m11, m12, m22) -> N x 2 x 2."""
    return np.stack([np.stack([M3[:, 0], M3[:, 1]], 1), np.stack([M3[:, 1], M3[:, 2]], 1)], 1)


@pytest.mark.parametrize("seed,nb,spc", [(6, 40, 0.1), (7, 200, 0.029)])
def test_hessian_metric_alpha_match_oracle(gctx, seed, nb, spc):
    m = disk_mesh(seed=seed, n_boundary=nb, spacing=spc)
    u = _u(m.X)
    mm = _mm(gctx, m)
    Mv, alpha, H = mm.metric(_dev(m.X), _dev(u), with_hessian=True)
    Hv = mmpde.vertex_hessians(m.X, m.elems, u)
    Mv_o, alpha_o = mmpde.level_metric(m.X, m.elems, u)
    H, Mv = H.cpu().numpy(), Mv.cpu().numpy()
    print(f"nv={m.nv} ne={m.ne} alpha gpu={alpha:.15g} oracle={alpha_o:.15g}", flush=True)
    # normal equations on the GPU, an SVD least-squares solve in the oracle: equal up to rounding
    assert np.max(np.abs(H - _sym3(Hv))) <= 1e-9 * np.max(np.abs(Hv))
    assert alpha == pytest.approx(alpha_o, rel=1e-9)
    assert np.max(np.abs(Mv - _sym3(Mv_o))) <= 1e-9 * np.max(np.abs(Mv_o))
    # det M = det(I + |H|/alpha)^{2/3} >= 1
    assert np.all(Mv[:, 0] * Mv[:, 2] - Mv[:, 1] ** 2 >= 1.0 - 1e-12)


def test_hessian_exact_for_quadratics_at_size(gctx):
    m = disk_mesh(seed=8, n_boundary=400, spacing=0.0145)
    x, y = m.X[:, 0], m.X[:, 1]
    u = 1 + 2 * x - y + 3 * x ** 2 - 2 * x * y + 0.5 * y ** 2
    mm = _mm(gctx, m)
    _, _, H = mm.metric(_dev(m.X), _dev(u), with_hessian=True)
    H = H.cpu().numpy()
    print(f"nv={m.nv}: max Hessian error {np.max(np.abs(H - [6.0, -2.0, 1.0])):.2e}", flush=True)
    assert np.allclose(H, [6.0, -2.0, 1.0], rtol=0, atol=1e-7)


def test_zero_solution_gives_identity_metric(gctx):
    m = disk_mesh(seed=9, n_boundary=30, spacing=0.15)
    mm = _mm(gctx, m)
    M, alpha = mm.metric(_dev(m.X), _dev(np.zeros(m.nv)))
    assert math.isinf(alpha)
    assert np.array_equal(M.cpu().numpy(), np.tile([1.0, 0.0, 1.0], (m.nv, 1)))


def _random_metric(n, seed):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, 2, 2))
    return Q @ np.transpose(Q, (0, 2, 1)) + 0.5 * np.eye(2)


def _perturbed(m, seed, amp):
    """Interior vertices moved by up to amp (no element inverted)."""
    rng = np.random.default_rng(seed)
    bnd = mmpde.boundary_mask(m.elems, m.nv)
    X = m.X + np.where(bnd[:, None], 0.0, rng.uniform(-amp, amp, m.X.shape))
    assert np.all(mmpde.element_areas(X, m.elems) > 0)
    return X


def test_field_energy_and_gradient_match_oracle(gctx):
    m = disk_mesh(seed=10, n_boundary=60, spacing=0.07)
    Mv = _random_metric(m.nv, 11)
    X = _perturbed(m, 12, 0.02)
    mm = _mm(gctx, m)
    e, G, MK = mm.energy(_dev(m.X), _dev(_sym3(Mv)), _dev(X))
    field = mmpde.MetricField(m.X, m.elems, Mv)
    e_o, G_o, M_o, loc = mmpde.energy_field(X, m.elems, field, np.arange(m.ne))
    print(f"ne={m.ne}: {np.sum(loc != np.arange(m.ne))} centroids left their element", flush=True)
    assert np.any(loc != np.arange(m.ne))
    assert np.max(np.abs(MK.cpu().numpy() - _sym3(M_o))) <= 1e-13 * np.max(np.abs(M_o))
    assert e == pytest.approx(e_o, rel=1e-12)
    assert np.max(np.abs(G.cpu().numpy() - G_o)) <= 1e-11 * np.max(np.abs(G_o))
    # an inverted element gives an infinite energy
    Xb = X.copy()
    k = m.elems[m.ne // 2]
    Xb[k[0]], Xb[k[1]] = X[k[1]], X[k[0]]
    e_bad, _, _ = mm.energy(_dev(m.X), _dev(_sym3(Mv)), _dev(Xb), grad=False)
    assert math.isinf(e_bad)


def test_element_hessians_match_oracle(gctx):
    m = disk_mesh(seed=16, n_boundary=60, spacing=0.07)
    Mk = _random_metric(m.ne, 17)
    H = _mm(gctx, m).element_hessians(_dev(m.X), _dev(_sym3(Mk))).cpu().numpy()
    H_o = mmpde.element_hessians_fd(m.X, m.elems, Mk)
    err = np.max(np.abs(H - H_o), axis=(1, 2)) / np.max(np.abs(H_o), axis=(1, 2))
    print(f"ne={m.ne}: max relative element Hessian difference {err.max():.2e}", flush=True)
    assert err.max() <= 1e-8


def test_fixed_steps_match_oracle(gctx):
    m = disk_mesh(seed=12, n_boundary=50, spacing=0.08)
    Mv_o, _ = mmpde.level_metric(m.X, m.elems, _u(m.X))
    bnd = mmpde.boundary_mask(m.elems, m.nv)
    # 2e-8: the step systems stay positive definite on this mesh
    X_o, _, oi = mmpde.move_mesh(m.X, m.elems, Mv_o, bnd, max_steps=5, fixed_dt=2e-8)
    mm = _mm(gctx, m)
    X = _dev(m.X)
    info = mm.move(X, _dev(_sym3(Mv_o)), max_steps=5, fixed_dt=2e-8, cg_tol=1e-13)
    d = np.max(np.abs(X.cpu().numpy() - X_o))
    print(f"nv={m.nv}: 5 steps of 2e-8, {info['cg_iterations']} CG iterations, max |X - X_oracle| {d:.2e}, "
          f"displacement {np.max(np.abs(X_o - m.X)):.2e}", flush=True)
    assert info["steps"] == 5
    assert d <= 1e-10
    assert info["energy_end"] == pytest.approx(oi["energy_end"], rel=1e-12)


@pytest.mark.parametrize("seed,nb,spc", [(13, 40, 0.1), (14, 70, 0.07)])
def test_move_matches_oracle(gctx, seed, nb, spc):
    m = disk_mesh(seed=seed, n_boundary=nb, spacing=spc)
    u = _u(m.X)
    mm = _mm(gctx, m)
    Xd = _dev(m.X)
    Mv, _ = mm.metric(Xd, _dev(u))
    info = mm.move(Xd, Mv)
    X = Xd.cpu().numpy()
    # the oracle moves the mesh with the GPU's vertex metrics, so that only the moving differs
    bnd = mmpde.boundary_mask(m.elems, m.nv)
    Y, steps, oi = mmpde.move_mesh(m.X, m.elems, _mat(Mv.cpu().numpy()), bnd)
    print(f"nv={m.nv}: steps gpu={info['steps']} (rejected {info['rejected']}, {info['cg_iterations']} CG) "
          f"oracle={steps} (rejected {oi['rejected']}); I {info['energy_start']:.10e} -> {info['energy_end']:.10e} "
          f"(oracle {oi['energy_end']:.10e}); |Pg| {info['grad_start']:.3e} -> {info['grad_end']:.3e} "
          f"(oracle {oi['grad']:.3e}); max |X - Y| {np.max(np.abs(X - Y)):.2e}", flush=True)
    assert info["steps"] == steps and info["rejected"] == oi["rejected"]
    assert info["energy_end"] == pytest.approx(oi["energy_end"], rel=1e-9)
    assert np.max(np.abs(X - Y)) <= 1e-8
    assert info["grad_end"] <= 1e-3 * info["grad_start"]
    assert np.all(mmpde.element_areas(X, m.elems) > 0)
    assert np.allclose(np.linalg.norm(X[bnd], axis=1), 1.0, rtol=0, atol=1e-14)


def test_fixed_boundary_mode(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    m = disk_mesh(seed=18, n_boundary=40, spacing=0.1)
    mm = gofd.Mmpde(gctx, m.nv, _dev(m.elems, torch.int32), boundary=gofd.MMPDE_BOUNDARY_FIXED)
    Xd = _dev(m.X)
    M, _ = mm.metric(Xd, _dev(_u(m.X)))
    info = mm.move(Xd, M, max_steps=5)
    X = Xd.cpu().numpy()
    bnd = mmpde.boundary_mask(m.elems, m.nv)
    assert info["steps"] == 5 and np.array_equal(X[bnd], m.X[bnd]) and not np.array_equal(X, m.X)
    assert info["energy_end"] < info["energy_start"]


def test_results_are_reproducible_bit_for_bit(gctx):
    m = disk_mesh(seed=15, n_boundary=100, spacing=0.045)
    u = _u(m.X)
    mm = _mm(gctx, m)
    out = []
    for _ in range(2):
        Xd = _dev(m.X)
        M, a = mm.metric(Xd, _dev(u))
        info = mm.move(Xd, M, max_steps=10)
        out.append((Xd.cpu().numpy(), M.cpu().numpy(), a, info["energy_end"]))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2] and out[0][3] == out[1][3]


def _min_height(X, elems):
    P = X[elems]
    e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    edge = np.max(np.stack([np.linalg.norm(P[:, a] - P[:, (a + 1) % 3], axis=1) for a in range(3)], 1), 1)
    return float(np.min(2 * area / edge))


def _amgofd(gctx, mesh, s, levels, n_max=1024):
    """Algorithm amGoFD on the GPU: solve, metric, move; returns the relative L2 error of every level.
    The overlay grid follows the paper's choice: R = 1.1, h_FD = R / N <= a_h (the smallest element
    height), N capped at n_max."""
    import torch
    import paper_2307_14437_amd as gofd
    mm = _mm(gctx, mesh)
    X = _dev(mesh.X)
    errs = []
    for lvl in range(levels + 1):
        Xh = X.cpu().numpy()
        N = min(n_max, int(math.ceil(1.1 / _min_height(Xh, mesh.elems))))
        g = grid_for_box(2, 2 * N, R=1.1)
        f = exact.f_ball(ogrid.node_coords(2, g.N, g.R, g.center), s, 2, 0).reshape(g.W, g.W)
        tr = gofd.Transfer(gctx, X, _dev(mesh.elems, torch.int32), g)
        op = gofd.FdOp(gctx, s, g)
        u, info = gofd.solve(gctx, tr, op, _dev(f), tol=1e-10, pc=gofd.Precond(gctx, tr, op, "DIAG"))
        ue = exact.u_ball(Xh, s, 2, 0)
        un = u.cpu().numpy()
        errs.append(exact.l2_error(Xh, mesh.elems, un - ue) / exact.l2_error(Xh, mesh.elems, ue))
        print(f"  level {lvl}: N={N} it={info[0]['iterations']} rel L2 err={errs[-1]:.3e}", flush=True)
        if lvl < levels:
            M, _ = mm.metric(X, u)
            mi = mm.move(X, M)
            print(f"    moved: {mi['steps']} steps ({mi['rejected']} rejected, {mi['cg_iterations']} CG), "
                  f"|Pg| {mi['grad_start']:.2e} -> {mi['grad_end']:.2e}", flush=True)
            assert mi["energy_end"] < mi["energy_start"]
    return errs


def test_adaptive_gofd_on_the_disk(gctx):
    # Example 1 with k = 0, s = 0.5: O(h) in L2 on fixed meshes, about O(hbar^2) on adaptive ones
    s = 0.5
    fixed, adaptive, hbar = [], [], []
    for seed, nb, spc in ((20, 50, 0.116), (21, 100, 0.058), (22, 200, 0.029)):
        mesh = disk_mesh(seed=seed, n_boundary=nb, spacing=spc)
        print(f"disk nv={mesh.nv} ne={mesh.ne}", flush=True)
        errs = _amgofd(gctx, mesh, s, levels=5)
        fixed.append(errs[0])
        adaptive.append(errs[-1])
        hbar.append(mesh.ne ** -0.5)
    rf = np.polyfit(np.log(hbar), np.log(fixed), 1)[0]
    ra = np.polyfit(np.log(hbar), np.log(adaptive), 1)[0]
    print(f"L2 rate fixed {rf:.2f} adaptive {ra:.2f}", flush=True)
    assert all(a < f for a, f in zip(adaptive, fixed))
    assert ra > rf + 0.4
