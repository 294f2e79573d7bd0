"""3D parity: the five-pass A_FD product (eq. AU-1 in three dimensions), A_h, solves and adjoint
gradients on small tetrahedral meshes against the oracle."""

import numpy as np
import pytest

from oracle import adjoint, afd, fdweights as fw, operator, solve, transfer
from workloads import ball_mesh, grid_for_box, structured_box_mesh_3d

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(a, dtype=None):
    import torch
    return torch.tensor(a, device="cuda", dtype=dtype)


@pytest.mark.parametrize("n,s", [(4, 0.5), (8, 0.3), (12, 0.7), (32, 0.5)])
def test_afd3_matches_oracle(gctx, n, s):
    import paper_2307_14437_amd as gofd
    g = grid_for_box(3, n, R=1.0)
    print(f"afd3 parity n={n} s={s} L={1 << (4 * g.N - 1).bit_length()}", flush=True)
    T = fw.filon_richardson(s, 3, 2 * g.N, 256 if n > 16 else 128)
    op = gofd.FdOp(gctx, s, g, T=T)
    rng = np.random.default_rng(n)
    v = rng.standard_normal((2, g.W, g.W, g.W))
    y = gofd.apply_afd(gctx, op, _dev(v)).cpu().numpy()
    for r in range(2):
        ref = afd.apply_direct(T, v[r]) if n <= 12 else afd.apply_fft(T, v[r])
        assert _rel(y[r], ref) < 1e-12
    y32 = gofd.apply_afd(gctx, op, _dev(v), gofd.FP32_GRID).cpu().numpy()
    assert _rel(y32[0], afd.apply_fft(T, v[0])) < 3e-6


@pytest.fixture(scope="module")
def ball_small():
    m = ball_mesh(seed=5, spacing=0.22)
    g = grid_for_box(3, 16, R=1.0)
    otr = transfer.Transfer(m.X, m.elems, 3, g.N, g.R, g.center)
    T = fw.filon_richardson(0.5, 3, 2 * g.N, 128)
    return m, g, otr, T


def test_apply_Ah3_matches_oracle(gctx, ball_small):
    import torch
    import paper_2307_14437_amd as gofd
    m, g, otr, T = ball_small
    tr = gofd.Transfer(gctx, _dev(m.X), _dev(m.elems, torch.int32), g)
    op = gofd.FdOp(gctx, 0.5, g, T=T)
    u = np.random.default_rng(4).standard_normal((2, m.nv))
    y = gofd.apply_Ah(gctx, tr, op, _dev(u)).cpu().numpy()
    for r in range(2):
        assert _rel(y[r], operator.apply_Ah(otr, T, u[r], "fft")) < 1e-12
    yk = gofd.apply_Ah(gctx, tr, op, _dev(u), gofd.UNSCALED | gofd.INTERIOR).cpu().numpy()
    ref = np.zeros(m.nv)
    ref[otr.J] = operator.apply_K(otr, T, u[0][otr.J], "fft")
    assert _rel(yk[0], ref) < 1e-12


def test_grid_coincident_mesh_reduces_to_fd_3d(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    g = grid_for_box(3, 8, R=1.0)
    lo = -1.0 + 2 * g.h
    mesh = structured_box_mesh_3d((lo, lo, lo), g.h, 4, 3, 5)
    tr = gofd.Transfer(gctx, _dev(mesh.X), _dev(mesh.elems, torch.int32), g)
    T = fw.filon_richardson(0.4, 3, 2 * g.N, 64)
    op = gofd.FdOp(gctx, 0.4, g, T=T)
    u = np.random.default_rng(2).standard_normal(mesh.nv)
    y = gofd.apply_Ah(gctx, tr, op, _dev(u), gofd.UNSCALED).cpu().numpy()
    # every vertex is a grid node with weight 1 (D = 1): A_h restricted to the vertices is A_FD's rows
    otr = transfer.Transfer(mesh.X, mesh.elems, 3, g.N, g.R, g.center)
    assert _rel(y, operator.apply_Ah(otr, T, u, "fft")) < 1e-12


@pytest.mark.parametrize("pcn", ["NONE", "DIAG", "IC1_27", "IC1_27_MC", "IC1_27_LAP_MC", "IC1_27_BMC"])
def test_solve3_matches_dense(gctx, ball_small, pcn):
    import torch
    import paper_2307_14437_amd as gofd
    m, g, otr, T = ball_small
    tr = gofd.Transfer(gctx, _dev(m.X), _dev(m.elems, torch.int32), g)
    op = gofd.FdOp(gctx, 0.5, g, T=T)
    K = operator.dense_K(otr, T)
    f = np.ones((g.W,) * 3)
    b = operator.rhs_grid(otr, 0.5, f)
    uref = np.zeros(m.nv)
    uref[otr.J] = solve.solve_dense(K, b)
    pc = gofd.Precond(gctx, tr, op, pcn)
    for mode in (gofd.MODE_FP64, gofd.MODE_FP32_RELIABLE):
        u, info = gofd.solve(gctx, tr, op, _dev(f), tol=1e-12, pc=pc, mode=mode)
        print(pcn, mode, info[0], flush=True)
        u = u.cpu().numpy()
        assert np.all(u[otr.bnd] == 0.0)
        assert _rel(u, uref) < (1e-10 if mode == gofd.MODE_FP64 else 1e-9)
        assert info[0]["rel_residual"] <= 1e-12


def test_adjoint3_matches_oracle(gctx):
    import torch
    from paper_2307_14437_amd.autograd import GoFDProblem, gofd_solve
    m = ball_mesh(seed=6, spacing=0.3)
    g = grid_for_box(3, 12, R=1.0)
    s = 0.5
    prob = GoFDProblem(gctx, torch.tensor(m.elems, dtype=torch.int32), g, s, precond="DIAG", tol=1e-13, M=64)
    T = prob.op.table()
    otr = transfer.Transfer(m.X, m.elems, 3, g.N, g.R, g.center)
    f = np.random.default_rng(7).standard_normal((g.W,) * 3)
    ut = np.zeros(m.nv)
    ut[otr.J] = np.random.default_rng(8).standard_normal(otr.J.size) * 0.1
    fd = _dev(f).requires_grad_(True)
    Xd = _dev(m.X).requires_grad_(True)
    u = gofd_solve(prob, fd, Xd)
    loss = 0.5 * torch.sum((u - _dev(ut)) ** 2)
    loss.backward()
    uJ, _ = adjoint.forward_dense(otr, T, s, f)
    gfo, gXo = adjoint.gradients(otr, T, s, f, uJ, uJ - ut[otr.J])
    assert np.max(np.abs(fd.grad.cpu().numpy() - gfo)) <= 1e-9 * np.max(np.abs(gfo))
    assert np.max(np.abs(Xd.grad.cpu().numpy() - gXo)) <= 1e-8 * np.max(np.abs(gXo))


@pytest.mark.parametrize("n,s,M", [(4, 0.3, 64), (8, 0.5, 128), (16, 0.7, 128), (32, 0.5, 256)])
def test_fd_weights3_match_oracle_filon(gctx, n, s, M):
    """The device's 3D T table (Filon's rule along every axis, eq. Tp-1D-2, Richardson over M and M/2,
    Section 2.3) against the oracle's at the same level, with and without the extrapolation."""
    import paper_2307_14437_amd as gofd
    g = grid_for_box(3, n, R=1.0)
    print(f"fd_weights 3D n={n} s={s} M={M}", flush=True)
    Mused = M
    while Mused // 2 < 2 * (2 * g.N) + 1:
        Mused *= 2
    Tg = gofd.FdOp(gctx, s, g, M=M).table()
    To = fw.filon_richardson(s, 3, 2 * g.N, Mused)
    assert Tg.shape == To.shape
    assert np.max(np.abs(Tg - To)) < 1e-13 * abs(To[0, 0, 0])
    T1 = gofd.FdOp(gctx, s, g, M=M, richardson=False).table()
    assert np.max(np.abs(T1 - fw.filon(s, 3, 2 * g.N, Mused))) < 1e-13 * abs(To[0, 0, 0])
    # the table is symmetric under axis permutations (psi~ is), which an index mix-up would break
    assert np.max(np.abs(Tg - Tg.transpose(1, 0, 2))) < 1e-15 * abs(To[0, 0, 0])
    assert np.max(np.abs(Tg - Tg.transpose(2, 1, 0))) < 1e-15 * abs(To[0, 0, 0])


def test_fd_weights3_default_level_against_bessel(gctx):
    """At the paper's 3D level (M = 2^11 with Richardson) the table agrees with the independent
    subordination/Bessel route within the quadrature's remaining error ~C M^{-2-2s}."""
    import paper_2307_14437_amd as gofd
    g = grid_for_box(3, 16, R=1.0)
    for s in (0.3, 0.7):
        print(f"fd_weights 3D default level s={s}", flush=True)
        T = gofd.FdOp(gctx, s, g).table()
        for p in [(0, 0, 0), (0, 0, 1), (0, 1, 1), (1, 1, 1), (1, 2, 3), (0, 5, 9), (16, 16, 16)]:
            assert abs(T[p] - fw.bessel_route(s, p)) < 2e-9 * abs(T[0, 0, 0]), p
