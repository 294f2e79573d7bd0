"""Column-pass schedules and their tuner: every schedule gives the oracle's product, the tuner installs
the fastest it measured, and the cached choice is reused."""

import json

import numpy as np
import pytest

from oracle import afd, fdweights as fw, operator, transfer
from workloads import disk_mesh, grid_for_box

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(a, dtype=None):
    import torch
    return torch.tensor(a, device="cuda", dtype=dtype)


@pytest.mark.parametrize("n", [32, 256])
def test_every_schedule_matches_the_oracle(gctx, n):
    import torch
    import paper_2307_14437_amd as gofd
    g = grid_for_box(2, n, R=1.0)
    M = 1
    while M < 8 * g.N + 2:      # Richardson's coarse rule needs M/2 >= 2P + 1 (P = 2N)
        M *= 2
    T = fw.filon_richardson(0.6, 2, 2 * g.N, M)
    op = gofd.FdOp(gctx, 0.6, g, T=T)
    rng = np.random.default_rng(n)
    v = rng.standard_normal((2, g.W, g.W))
    ref = [afd.apply_direct(T, v[r]) if n <= 32 else afd.apply_fft(T, v[r]) for r in range(2)]
    try:
        for s in range(gofd.N_COL_SCHED):
            print(f"schedule {s} n={n}", flush=True)
            for fp32 in (False, True):
                gofd.set_schedule(gctx, g, s, fp32=fp32)
                y = gofd.apply_afd(gctx, op, torch.tensor(v, device="cuda"), gofd.FP32_GRID if fp32 else 0)
                y = y.cpu().numpy()
                for r in range(2):
                    assert _rel(y[r], ref[r]) < (2e-6 if fp32 else 1e-12)
    finally:
        for fp32 in (False, True):
            gofd.set_schedule(gctx, g, 0, fp32=fp32)


def test_schedules_in_cg_match(gctx):
    # the column pass of CG also carries the delta partials: every schedule gives the same solve to rounding
    import torch
    import paper_2307_14437_amd as gofd
    m = disk_mesh(seed=41, n_boundary=40, spacing=0.1)
    g = grid_for_box(2, 64, R=1.0)
    tr = gofd.Transfer(gctx, torch.tensor(m.X, device="cuda"), torch.tensor(m.elems, dtype=torch.int32,
                                                                           device="cuda"), g)
    op = gofd.FdOp(gctx, 0.5, g, M=512)
    f = torch.tensor(np.ones((g.W, g.W)), device="cuda")
    out = []
    try:
        for s in range(gofd.N_COL_SCHED):
            gofd.set_schedule(gctx, g, s, fp32=False)
            u, info = gofd.solve(gctx, tr, op, f, tol=1e-10)
            out.append((u.cpu().numpy(), info[0]["iterations"]))
    finally:
        gofd.set_schedule(gctx, g, 0, fp32=False)
    for u, it in out[1:]:
        assert abs(it - out[0][1]) <= 1
        assert _rel(u, out[0][0]) < 1e-9


def test_autotune_picks_its_fastest_and_caches(gctx, tmp_path):
    import paper_2307_14437_amd as gofd
    g = grid_for_box(2, 512, R=1.0)
    cache = str(tmp_path / "tune.json")
    try:
        s, times = gofd.autotune(gctx, g, fp32=True, cache=cache)
        print(s, times, flush=True)
        assert 0 <= s < gofd.N_COL_SCHED and len(times) == gofd.N_COL_SCHED
        assert all(t > 0 for t in times)
        assert times[s] == min(times) or (s == 0 and min(times) >= 0.95 * times[0])
        data = json.load(open(cache))
        assert len(data) == 1 and list(data.values())[0]["schedule"] == s
        s2, t2 = gofd.autotune(gctx, g, fp32=True, cache=cache)      # served from the cache
        assert s2 == s and t2 is None
    finally:
        gofd.set_schedule(gctx, g, 0, fp32=True)


def test_row_pass_and_3d_schedules_tune_and_agree(gctx):
    """The first row pass of the products at 8 and 16 values per thread (2D, L >= 1024) and the 3D y/z/y
    passes at four and two slots per block give the same product to rounding; the tuner times both of
    each and installs what it measured."""
    import paper_2307_14437_amd as gofd
    g2 = grid_for_box(2, 512, R=1.0)                     # L = 1024: both row-pass widths exist
    T2 = fw.filon_richardson(0.4, 2, 2 * g2.N, 4096)
    op2 = gofd.FdOp(gctx, 0.4, g2, T=T2)
    v2 = np.random.default_rng(3).standard_normal((1, g2.W, g2.W))
    ref2 = afd.apply_fft(T2, v2[0])
    g3 = grid_for_box(3, 32, R=1.0)                      # L = 128
    T3 = fw.filon_richardson(0.6, 3, 2 * g3.N, 256)
    op3 = gofd.FdOp(gctx, 0.6, g3, T=T3)
    v3 = np.random.default_rng(4).standard_normal((1, g3.W, g3.W, g3.W))
    ref3 = afd.apply_fft(T3, v3[0])
    try:
        for fp32 in (False, True):
            tol = 3e-6 if fp32 else 1e-12
            flags = gofd.FP32_GRID if fp32 else 0
            for width in (8, 16):
                gofd.set_schedule(gctx, g2, width, fp32=fp32, rows=True)
                y = gofd.apply_afd(gctx, op2, _dev(v2), flags).cpu().numpy()
                assert _rel(y[0], ref2) < tol, (fp32, width)
            for sch in (0, 1):
                gofd.set_schedule(gctx, g3, sch, fp32=fp32)
                y = gofd.apply_afd(gctx, op3, _dev(v3), flags).cpu().numpy()
                assert _rel(y[0], ref3) < tol, (fp32, sch)
            r2 = gofd.autotune_all(gctx, g2, fp32=fp32)
            print("2D", fp32, r2, flush=True)
            t = r2["times"]
            assert r2["row"] in (8, 16) and t[4] > 0 and t[5] > 0
            assert r2["row"] == (16 if t[5] < 0.95 * t[4] else 8)
            r3 = gofd.autotune_all(gctx, g3, fp32=fp32)
            print("3D", fp32, r3, flush=True)
            t = r3["times"]
            assert t[0] > 0 and t[1] > 0 and r3["yzy"] == (1 if t[1] < 0.95 * t[0] else 0)
    finally:
        for fp32 in (False, True):
            gofd.set_schedule(gctx, g2, 0, fp32=fp32, rows=True)
            gofd.set_schedule(gctx, g3, 0, fp32=fp32)

