"""Solves at the large workloads' sizes, checked by what holds at any size:

* 3D unit ball, f = 1, s = 1/2, 64^3 grid (a mid-size copy of the 256^3
  workload): the oracle's residual of eq. GoFD-2 for the FP64 and FP32-grid
  solutions, and the L2 error against the closed-form solution
  u = Gamma(d/2) / (2^{2s} Gamma(1+s) Gamma(d/2+s)) (1-|x|^2)^s (Section 5).
* 2D star domain, 250k vertices, 2048^2 grid (FFT length 4096), s = 0.6:
  the solve by the oracle's residual, then the adjoint gradients of
  L = 1/2 ||u - u_t||^2: the adjoint solution by the oracle's residual of
  K lambda = dL/du, dL/df = h^{2s} I lambda, and dL/df against central
  differences of GPU solves (L is quadratic in f, so they are exact up to
  rounding)."""

import numpy as np
import pytest

from oracle import exact, operator, transfer
from workloads import ball_mesh, config_inputs, grid_for_box

pytestmark = pytest.mark.gpu


def _dev(a, dtype=None):
    import torch
    return torch.tensor(a, device="cuda", dtype=dtype)


def test_ball_64_solve_oracle_residual_and_closed_form(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    s = 0.5
    mesh = ball_mesh(seed=1003, spacing=0.057)
    g = grid_for_box(3, 64, R=1.0)
    print(f"ball 64^3: nv={mesh.nv} ne={mesh.ne}", flush=True)
    tr = gofd.Transfer(gctx, _dev(mesh.X), _dev(mesh.elems, torch.int32), g)
    op = gofd.FdOp(gctx, s, g)
    T = op.table()
    f = np.ones((g.W,) * 3)
    pc = gofd.Precond(gctx, tr, op, "DIAG")
    otr = transfer.Transfer(mesh.X, mesh.elems, 3, g.N, g.R, g.center)
    b = operator.rhs_grid(otr, s, f)
    ue = exact.u_ball_unit_rhs(mesh.X, s, 3)
    for mode in (gofd.MODE_FP64, gofd.MODE_FP32_RELIABLE):
        u, info = gofd.solve(gctx, tr, op, _dev(f), tol=1e-10, pc=pc, mode=mode)
        u = u.cpu().numpy()
        r = operator.apply_K(otr, T, u[otr.J], "fft") - b
        res = np.linalg.norm(r) / np.linalg.norm(b)
        err = exact.l2_error(mesh.X, mesh.elems, u - ue) / exact.l2_error(mesh.X, mesh.elems, ue)
        print(mode, info[0], f"oracle residual {res:.2e}, L2 error vs closed form {err:.3e}", flush=True)
        assert res < 2e-10
        assert err < 0.03
        assert np.all(u[otr.bnd] == 0.0)


def test_star_2048_solve_and_adjoint(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    cfg = config_inputs("c5")
    m, g, f = cfg["mesh"], cfg["grid"], cfg["f"][0]
    s = cfg["s"][0]
    print(f"star 2048^2: nv={m.nv}", flush=True)
    tr = gofd.Transfer(gctx, _dev(m.X), _dev(m.elems, torch.int32), g)
    op = gofd.FdOp(gctx, s, g)
    T = op.table()
    pc = gofd.Precond(gctx, tr, op, "DIAG")
    fd = _dev(f)
    u, info = gofd.solve(gctx, tr, op, fd, tol=1e-11, pc=pc)
    otr = transfer.Transfer(m.X, m.elems, 2, g.N, g.R, g.center)
    b = operator.rhs_grid(otr, s, f)
    uh = u.cpu().numpy()
    res = np.linalg.norm(operator.apply_K(otr, T, uh[otr.J], "fft") - b) / np.linalg.norm(b)
    print("solve", info[0], f"oracle residual {res:.2e}", flush=True)
    assert res < 5e-11
    ut = np.zeros(m.nv)
    ut[otr.J] = 0.9 * uh[otr.J] + 0.05 * np.random.default_rng(3).standard_normal(otr.J.size) * np.abs(uh).max()
    dLdu = _dev(uh - ut)
    gf, gX, lam, ainfo = gofd.solve_adjoint(gctx, tr, op, dLdu, u, fd, tol=1e-11, pc=pc)
    lam = lam.cpu().numpy()
    g_int = (uh - ut)[otr.J]
    lres = np.linalg.norm(operator.apply_K(otr, T, lam[otr.J], "fft") - g_int) / np.linalg.norm(g_int)
    print("adjoint", ainfo, f"oracle residual of K lambda = dL/du: {lres:.2e}", flush=True)
    assert lres < 5e-11
    h2s = otr.h ** (2 * s)
    gf = gf.cpu().numpy()
    ref = h2s * (otr.IJ @ lam[otr.J])
    assert np.linalg.norm(gf - ref) <= 1e-12 * np.linalg.norm(ref)
    assert gX.shape == (m.nv, 2) and np.all(np.isfinite(gX.cpu().numpy()))

    def loss(fv):
        uu, _ = gofd.solve(gctx, tr, op, _dev(fv), tol=1e-12, pc=pc)
        return 0.5 * float(np.sum((uu.cpu().numpy() - ut)[otr.J] ** 2))

    rng = np.random.default_rng(4)
    eps = 0.1 * np.abs(f).max()        # L is quadratic in f: central differences are exact for any step
    for k in rng.choice(otr.inside, 4, replace=False):
        iy, ix = divmod(int(k), g.W)
        fp, fm = f.copy(), f.copy()
        fp[iy, ix] += eps
        fm[iy, ix] -= eps
        fdv = (loss(fp) - loss(fm)) / (2 * eps)
        print("dL/df", k, gf.reshape(g.W, g.W)[iy, ix], fdv, flush=True)
        assert abs(gf.reshape(g.W, g.W)[iy, ix] - fdv) <= 1e-6 * np.abs(gf).max()
