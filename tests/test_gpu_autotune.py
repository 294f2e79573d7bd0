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
