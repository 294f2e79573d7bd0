"""Parity of the A_FD product (eq. AU-1 / AFD-1), of A_h (eq. Ah-1) and of fd_weights with the oracle."""

import numpy as np
import pytest

from oracle import afd, fdweights as fw, operator, transfer
from workloads import config_inputs, disk_mesh, grid_for_box

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,s", [(2, 0.5), (4, 0.4), (8, 0.3), (42, 0.5), (64, 0.75), (128, 0.25)])
def test_afd_matches_direct_sums(gctx, n, s):
    import torch
    import paper_2307_14437_amd as gofd
    g = grid_for_box(2, n, R=1.0)
    print(f"afd parity n={n} s={s}", flush=True)
    T = fw.filon_richardson(s, 2, 2 * g.N, 1024 if n <= 64 else 2048)
    op = gofd.FdOp(gctx, s, g, T=T)
    rng = np.random.default_rng(n)
    v = rng.standard_normal((3, g.W, g.W))
    y = gofd.apply_afd(gctx, op, torch.tensor(v, device="cuda")).cpu().numpy()
    for r in range(3):
        ref = afd.apply_direct(T, v[r]) if n <= 64 else afd.apply_fft(T, v[r])
        assert _rel(y[r], ref) < 1e-12
    y32 = gofd.apply_afd(gctx, op, torch.tensor(v, device="cuda"), gofd.FP32_GRID).cpu().numpy()
    assert _rel(y32[0], afd.apply_fft(T, v[0])) < 2e-6


def test_afd_full_size_sampled(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    g = grid_for_box(2, 1024, R=1.0)
    T = fw.filon(0.75, 2, 2 * g.N, 4096)        # any valid table serves the product check
    op = gofd.FdOp(gctx, 0.75, g, T=T)
    rng = np.random.default_rng(5)
    v = rng.standard_normal((g.W, g.W))
    y = gofd.apply_afd(gctx, op, torch.tensor(v, device="cuda")).cpu().numpy()
    nodes = [(0, 0), (1024, 1024), (0, 1024), (512, 3), (777, 1001), (5, 640)]
    ref = afd.apply_rows(T, v, nodes)
    got = np.array([y[k] for k in nodes])
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(y))
    assert _rel(y, afd.apply_fft(T, v)) < 1e-12


def _synthetic_table(d, W):
    """A symmetric, decaying table: any T serves the product check (the product is linear in T)."""
    idx = np.indices((W,) * d).astype(np.float64)
    r = np.sqrt(np.sum(idx ** 2, axis=0))
    T = -1.0 / (1.0 + r) ** 2.5
    T.flat[0] = 0.0
    T.flat[0] = -T.sum() * 1.01
    return T


@pytest.mark.parametrize("d,n", [(2, 2048), (3, 256)])
def test_afd_largest_grids_sampled(gctx, d, n):
    """The largest workloads' grids (C5: 2048^2, FFT length 4096; C3: 256^3, length 512) against direct
    sums of sampled rows, in both precisions."""
    import torch
    import paper_2307_14437_amd as gofd
    g = grid_for_box(d, n, R=1.0)
    T = _synthetic_table(d, g.W)
    op = gofd.FdOp(gctx, 0.5, g, T=T)
    v = np.random.default_rng(d).standard_normal((g.W,) * d)
    print(f"afd largest d={d} n={n}", flush=True)
    vd = torch.tensor(v, device="cuda")
    y = gofd.apply_afd(gctx, op, vd).cpu().numpy()
    y32 = gofd.apply_afd(gctx, op, vd, gofd.FP32_GRID).cpu().numpy()
    W = g.W
    nodes = [(0,) * d, (W - 1,) * d, tuple([W // 2] * d), tuple(np.random.default_rng(9).integers(0, W, size=d)),
             tuple([1] + [W - 2] * (d - 1))]
    ref = afd.apply_rows(T, v, nodes)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(np.array([y[k] for k in nodes]) - ref)) < 1e-12 * scale
    assert np.max(np.abs(np.array([y32[k] for k in nodes]) - ref)) < 1e-5 * scale


@pytest.fixture(scope="module")
def c1_pair(c1):
    m, g = c1["mesh"], c1["grid"]
    otr = transfer.Transfer(m.X, m.elems, 2, g.N, g.R, g.center)
    T = fw.filon_richardson(0.5, 2, 2 * g.N, 1024)
    return m, g, otr, T


def test_apply_Ah_variants_c1(gctx, c1_pair):
    import torch
    import paper_2307_14437_amd as gofd
    m, g, otr, T = c1_pair
    X = torch.tensor(m.X, device="cuda")
    E = torch.tensor(m.elems, dtype=torch.int32, device="cuda")
    tr = gofd.Transfer(gctx, X, E, g)
    op = gofd.FdOp(gctx, 0.5, g, T=T)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((2, m.nv))
    ud = torch.tensor(u, device="cuda")
    y = gofd.apply_Ah(gctx, tr, op, ud).cpu().numpy()
    for r in range(2):
        assert _rel(y[r], operator.apply_Ah(otr, T, u[r], "direct")) < 1e-12
    ys = gofd.apply_Ah(gctx, tr, op, ud, gofd.SYMMETRIC).cpu().numpy()
    assert _rel(ys[0], operator.apply_Ah_sym(otr, T, u[0], "direct")) < 1e-12
    yk = gofd.apply_Ah(gctx, tr, op, ud, gofd.UNSCALED | gofd.INTERIOR).cpu().numpy()
    ref = np.zeros(m.nv)
    ref[otr.J] = operator.apply_K(otr, T, u[0][otr.J], "direct")
    assert _rel(yk[0], ref) < 1e-12
    yh = gofd.apply_Ah(gctx, tr, op, ud, gofd.SCALE_H2S).cpu().numpy()
    assert _rel(yh[0], operator.apply_Ah(otr, T, u[0], "direct") / g.h ** 1.0) < 1e-12
    y32 = gofd.apply_Ah(gctx, tr, op, ud, gofd.FP32_GRID).cpu().numpy()
    assert _rel(y32[0], y[0]) < 1e-5


def test_apply_Ah_lshape_full_size(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    cfg = config_inputs("c2")
    m, g = cfg["mesh"], cfg["grid"]
    otr = transfer.Transfer(m.X, m.elems, 2, g.N, g.R, g.center)
    T = fw.filon(0.25, 2, 2 * g.N, 4096)
    tr = gofd.Transfer(gctx, torch.tensor(m.X, device="cuda"), torch.tensor(m.elems, dtype=torch.int32,
                                                                            device="cuda"), g)
    op = gofd.FdOp(gctx, 0.25, g, T=T)
    u = np.random.default_rng(2).standard_normal(m.nv)
    y = gofd.apply_Ah(gctx, tr, op, torch.tensor(u, device="cuda")).cpu().numpy()
    assert _rel(y, operator.apply_Ah(otr, T, u, "fft")) < 1e-12


@pytest.mark.parametrize("n,s,M", [(16, 0.4, 256), (64, 0.5, 1024), (64, 0.8, 512)])
def test_fd_weights_match_oracle_filon(gctx, n, s, M):
    import paper_2307_14437_amd as gofd
    g = grid_for_box(2, n, R=1.0)
    op = gofd.FdOp(gctx, s, g, M=M)
    Tg = op.table()
    Mused = M
    while Mused // 2 < 2 * (2 * g.N) + 1:
        Mused *= 2
    To = fw.filon_richardson(s, 2, 2 * g.N, Mused)
    assert np.max(np.abs(Tg - To)) < 1e-13
    op1 = gofd.FdOp(gctx, s, g, M=M, richardson=False)
    assert np.max(np.abs(op1.table() - fw.filon(s, 2, 2 * g.N, Mused))) < 1e-13


def test_fd_weights_default_level_against_bessel(gctx):
    import paper_2307_14437_amd as gofd
    g = grid_for_box(2, 1024, R=1.0)
    for s in (0.25, 0.75):
        T = gofd.FdOp(gctx, s, g).table()      # paper's level M = 2^14 with Richardson
        for p in [(0, 0), (0, 1), (1, 1), (3, 7), (40, 2), (300, 511), (1024, 1024)]:
            assert abs(T[p] - fw.bessel_route(s, p)) < 2e-10 * max(1.0, abs(T[0, 0]))
