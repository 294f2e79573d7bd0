"""Truncated CG with checkpointed iterates and its unrolled (reverse-mode)
gradient, against the oracle: the checkpoints equal the oracle's textbook CG
iterates, the gradients equal central differences of the oracle's truncated
solve (in f, in the vertex coordinates and in x0), and a converged truncated
solve gives the adjoint of eq. GoFD-2 (Section 3.2)."""

import numpy as np
import pytest

from oracle import fdweights as fw, operator, solve, transfer
from workloads import disk_mesh, grid_for_box

pytestmark = pytest.mark.gpu

S = 0.6


def _dev(a, dtype=None):
    import torch
    return torch.tensor(a, device="cuda", dtype=dtype)


@pytest.fixture(scope="module")
def small(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    mesh = disk_mesh(seed=31, n_boundary=40, spacing=0.16)
    g = grid_for_box(2, 32, R=1.1)
    T = fw.filon_richardson(S, 2, 2 * g.N, 256)
    op = gofd.FdOp(gctx, S, g, T=T)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((g.W, g.W))
    x0 = 0.1 * rng.standard_normal(mesh.nv)
    target = rng.standard_normal(mesh.nv)
    return mesh, g, T, op, f, x0, target


def _oracle_run(mesh, X, g, T, f, x0, iters):
    otr = transfer.Transfer(X, mesh.elems, 2, g.N, g.R, g.center)
    K = operator.dense_K(otr, T)
    b = operator.rhs_grid(otr, S, f)
    its, sc = solve.cg_iterates(lambda v: K @ v, b, iters, None if x0 is None else x0[otr.J])
    return otr, its, sc


def _full(otr, v):
    u = np.zeros(otr.nv)
    u[otr.J] = v
    return u


def test_checkpoints_are_the_oracle_iterates(gctx, small):
    import torch
    import paper_2307_14437_amd as gofd
    mesh, g, T, op, f, x0, _ = small
    tr = gofd.Transfer(gctx, _dev(mesh.X), _dev(mesh.elems, torch.int32), g)
    k, c = 21, 4
    tape = gofd.CgTape(gctx, tr, op, _dev(f), x0=_dev(x0), max_iter=k, ckpt_every=c)
    assert tape.info["iterations"] == k and tape.info["checkpoints"] == k // c + 1
    otr, its, sc = _oracle_run(mesh, mesh.X, g, T, f, x0, k)
    # the residual and direction shrink with the iterations: each is compared on the scale of its
    # iteration-0 value (and x on that of the final iterate)
    scale = [np.linalg.norm(its[k][0]), np.linalg.norm(its[0][1]), np.linalg.norm(its[0][2])]
    for j in range(k // c + 1):
        x, r, p, scal = tape.checkpoint(j)
        for q, (got, want) in enumerate(zip((x, r, p), its[j * c])):
            want = _full(otr, want)
            assert np.linalg.norm(got.cpu().numpy() - want) <= 1e-11 * scale[q], (j, q)
    assert np.allclose(scal[0, :k + 1], sc["gamma"], rtol=1e-10, atol=0)
    assert np.allclose(scal[2, :k], sc["alpha"], rtol=1e-10, atol=0)
    assert np.allclose(scal[3, :k], sc["beta"], rtol=1e-10, atol=0)
    xk = _full(otr, its[k][0])
    assert np.linalg.norm(tape.x.cpu().numpy() - xk) <= 1e-11 * np.linalg.norm(xk)
    tape.close()


@pytest.mark.parametrize("with_x0", [False, True])
def test_unrolled_gradients_match_central_differences(gctx, small, with_x0):
    import torch
    import paper_2307_14437_amd as gofd
    mesh, g, T, op, f, x0, target = small
    x0 = x0 if with_x0 else None
    k, c = 7, 3
    tr = gofd.Transfer(gctx, _dev(mesh.X), _dev(mesh.elems, torch.int32), g)
    tape = gofd.CgTape(gctx, tr, op, _dev(f), x0=None if x0 is None else _dev(x0), max_iter=k, ckpt_every=c)
    otr, its, _ = _oracle_run(mesh, mesh.X, g, T, f, x0, k)
    xk = _full(otr, its[k][0])
    assert np.linalg.norm(tape.x.cpu().numpy() - xk) <= 1e-11 * np.linalg.norm(xk)
    xbar = xk - target                          # L = 1/2 ||x_k - target||^2 over the interior vertices
    xbar[otr.bnd] = 0.0
    gf, gX, g0 = tape.grad(_dev(xbar), want_x0=True)
    gf, gX, g0 = gf.cpu().numpy().reshape(g.W, g.W), gX.cpu().numpy(), g0.cpu().numpy()

    def loss(X=mesh.X, ff=f, xx0=x0):
        o, it_, _ = _oracle_run(mesh, X, g, T, ff, xx0, k)
        return 0.5 * np.sum((_full(o, it_[k][0]) - target)[o.J] ** 2), o

    rng = np.random.default_rng(9)
    # f: nodes inside the mesh
    nodes = rng.choice(otr.inside, 10, replace=False)
    ef = 1e-4
    for kk in nodes:
        iy, ix = divmod(int(kk), g.W)
        fp, fm = f.copy(), f.copy()
        fp[iy, ix] += ef
        fm[iy, ix] -= ef
        fd = (loss(ff=fp)[0] - loss(ff=fm)[0]) / (2 * ef)
        assert abs(gf[iy, ix] - fd) <= 1e-6 * np.max(np.abs(gf)), (kk, gf[iy, ix], fd)
    # X: interior vertex coordinates, skipping steps that change the node -> element map
    eX, checked = 1e-6, 0
    for j in rng.choice(otr.J, 12, replace=False):
        for a in range(2):
            Xp, Xm = mesh.X.copy(), mesh.X.copy()
            Xp[j, a] += eX
            Xm[j, a] -= eX
            lp, op_ = loss(X=Xp)
            lm, om = loss(X=Xm)
            if not (np.array_equal(op_.elem, otr.elem) and np.array_equal(om.elem, otr.elem)):
                continue
            fd = (lp - lm) / (2 * eX)
            assert abs(gX[j, a] - fd) <= 2e-6 * np.max(np.abs(gX)), (j, a, gX[j, a], fd)
            checked += 1
    assert checked >= 12
    # x0 (the starting guess; at x0 = 0 this is the sensitivity to the start)
    base = np.zeros(mesh.nv) if x0 is None else x0
    for j in rng.choice(otr.J, 8, replace=False):
        xp, xm = base.copy(), base.copy()
        xp[j] += 1e-5
        xm[j] -= 1e-5
        fd = (loss(xx0=xp)[0] - loss(xx0=xm)[0]) / 2e-5
        assert abs(g0[j] - fd) <= 1e-6 * np.max(np.abs(g0)), (j, g0[j], fd)
    tape.close()


def test_converged_unrolled_gradient_is_the_adjoint(gctx, small):
    import torch
    import paper_2307_14437_amd as gofd
    mesh, g, T, op, f, _, target = small
    tr = gofd.Transfer(gctx, _dev(mesh.X), _dev(mesh.elems, torch.int32), g)
    tape = gofd.CgTape(gctx, tr, op, _dev(f), max_iter=400, tol=1e-14, ckpt_every=16)
    assert tape.info["converged"] == 1
    x = tape.x
    xbar = (x.cpu().numpy() - target) * tr_interior(tr)
    gf, gX, _ = tape.grad(_dev(xbar))
    af, aX, _, _ = gofd.solve_adjoint(gctx, tr, op, _dev(xbar), x, _dev(f), tol=1e-14)
    print(tape.info, flush=True)
    assert np.linalg.norm(gf.cpu().numpy() - af.cpu().numpy()) <= 1e-8 * np.linalg.norm(af.cpu().numpy())
    assert np.linalg.norm(gX.cpu().numpy() - aX.cpu().numpy()) <= 1e-8 * np.linalg.norm(aX.cpu().numpy())
    tape.close()


def tr_interior(tr):
    import paper_2307_14437_amd as gofd
    return 1.0 - tr.export(gofd.TR_BOUNDARY).cpu().numpy().astype(np.float64)


def test_autograd_unrolled_mode(gctx, small):
    import torch
    from paper_2307_14437_amd.autograd import GoFDProblem, gofd_solve_unrolled
    mesh, g, T, op, f, x0, target = small
    prob = GoFDProblem(gctx, torch.tensor(mesh.elems, dtype=torch.int32), g, S, M=256)
    fd = _dev(f).requires_grad_(True)
    Xd = _dev(mesh.X).requires_grad_(True)
    x0d = _dev(x0).requires_grad_(True)
    x = gofd_solve_unrolled(prob, fd, Xd, x0d, iters=9, ckpt_every=4)
    loss = 0.5 * torch.sum((x - _dev(target)) ** 2)       # the library masks dL/dx to the interior
    loss.backward()
    assert fd.grad.shape == fd.shape and Xd.grad.shape == Xd.shape and x0d.grad.shape == x0d.shape
    # the same gradients through the tape directly
    import paper_2307_14437_amd as gofd
    tr = gofd.Transfer(gctx, Xd.detach(), prob.elems, g)
    tape = gofd.CgTape(gctx, tr, prob.op, fd.detach(), x0=x0d.detach(), max_iter=9, ckpt_every=4)
    gf, gX, g0 = tape.grad(_dev(tape.x.cpu().numpy() - target), want_x0=True)
    assert torch.allclose(fd.grad.view(-1), gf, rtol=1e-12, atol=1e-14)
    assert torch.allclose(Xd.grad, gX, rtol=1e-12, atol=1e-14)
    assert torch.allclose(x0d.grad, g0, rtol=1e-12, atol=1e-14)

