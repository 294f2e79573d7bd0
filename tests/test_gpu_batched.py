"""Batched solves: problems of one grid shape advance together (one launch per stage for the group);
every item must match its own solve and, for a small case, the oracle's dense solution."""

import numpy as np
import pytest

from oracle import fdweights as fw, operator, solve as osolve, transfer
from workloads import disk_mesh, fourier_rhs, grid_for_box, star_mesh

pytestmark = pytest.mark.gpu


def _dev(a, dtype=None):
    import torch
    return torch.tensor(a, device="cuda", dtype=dtype)


def _problems(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    specs = [  # (mesh, n, R, s, precond, nrhs)
        (disk_mesh(seed=21, n_boundary=30, spacing=0.14), 32, 1.0, 0.3, "DIAG", 2),
        (star_mesh(22, 300), 32, 1.6, 0.7, "NONE", 1),
        (disk_mesh(seed=23, n_boundary=40, spacing=0.09), 64, 1.05, 0.5, "IC1_9", 2),
        (disk_mesh(seed=24, n_boundary=28, spacing=0.15), 32, 1.1, 0.55, "IC1_9", 1),
    ]
    out = []
    for k, (m, n, R, s, pcn, nr) in enumerate(specs):
        g = grid_for_box(2, n, R=R)
        tr = gofd.Transfer(gctx, _dev(m.X), _dev(m.elems, torch.int32), g)
        op = gofd.FdOp(gctx, s, g, M=512)
        pc = gofd.Precond(gctx, tr, op, pcn)
        f = np.stack([fourier_rhs(100 + 10 * k + r, g) for r in range(nr)])
        out.append(dict(m=m, g=g, s=s, tr=tr, op=op, pc=pc, f=f))
    return out


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
def test_batched_matches_individual_solves(gctx, mode):
    import paper_2307_14437_amd as gofd
    md = gofd.MODE_FP64 if mode == "fp64" else gofd.MODE_FP32_RELIABLE
    P = _problems(gctx)
    us, infos = gofd.solve_batched(gctx, [p["tr"] for p in P], [p["op"] for p in P], [p["pc"] for p in P],
                                   [_dev(p["f"]) for p in P], tol=1e-12, mode=md)
    k = 0
    for p, u in zip(P, us):
        u = u.cpu().numpy().reshape(len(p["f"]), -1)
        for r in range(len(p["f"])):
            ui, ii = gofd.solve(gctx, p["tr"], p["op"], _dev(p["f"][r]), tol=1e-12, pc=p["pc"], mode=md)
            ui = ui.cpu().numpy()
            print(mode, k, infos[k], ii[0], flush=True)
            assert infos[k]["rel_residual"] <= 1e-12 and infos[k]["status"] == 0
            assert np.linalg.norm(u[r] - ui) <= 1e-9 * np.linalg.norm(ui)
            # FP32: the replacement points follow the checks, which differ between a batch and one item
            slack = 2 if mode == "fp64" else 3 + ii[0]["iterations"] // 10
            assert abs(infos[k]["iterations"] - ii[0]["iterations"]) <= slack
            k += 1


def test_batched_item_matches_oracle(gctx):
    import paper_2307_14437_amd as gofd
    P = _problems(gctx)
    us, infos = gofd.solve_batched(gctx, [p["tr"] for p in P], [p["op"] for p in P], [p["pc"] for p in P],
                                   [_dev(p["f"]) for p in P], tol=1e-12)
    p = P[1]
    g = p["g"]
    otr = transfer.Transfer(p["m"].X, p["m"].elems, 2, g.N, g.R, g.center)
    T = fw.filon_richardson(p["s"], 2, 2 * p["g"].N, 512)      # the oracle's table (the GPU's matches it, 1e-13)
    K = operator.dense_K(otr, T)
    uref = np.zeros(p["m"].nv)
    uref[otr.J] = osolve.solve_dense(K, operator.rhs_grid(otr, p["s"], p["f"][0]))
    u = us[1].cpu().numpy()
    assert np.linalg.norm(u - uref) <= 1e-10 * np.linalg.norm(uref)


def test_batched_fp32_replacement_count(gctx):
    # residual replacements are per item (only the items whose residual has
    # dropped, or that stopped, are replaced); an item whose stop a replacement
    # has confirmed has no more of them while the others continue
    import torch
    import paper_2307_14437_amd as gofd
    m = star_mesh(31, 900)
    g = grid_for_box(2, 64, R=1.6)
    tr = gofd.Transfer(gctx, _dev(m.X), _dev(m.elems, torch.int32), g)
    ops = [gofd.FdOp(gctx, s, g, M=512) for s in (0.2, 0.8)]
    pcs = [gofd.Precond(gctx, tr, op, "NONE") for op in ops]
    f = _dev(fourier_rhs(7, g)[None, :])
    tol, drop = 1e-10, 0.1
    us, infos = gofd.solve_batched(gctx, [tr, tr], ops, pcs, [f, f], tol=tol, mode=gofd.MODE_FP32_RELIABLE,
                                   inner_tol=drop)
    print(infos, flush=True)
    it = sorted(i["iterations"] for i in infos)
    assert it[1] >= it[0] + 20                  # the fast item stops well before the slow one
    for i in infos:
        assert i["status"] == 0 and i["rel_residual"] <= tol
        # (r, r) falls by tol^2 overall, drop^2 per replacement, plus one at each item's stop
        assert i["refinements"] <= round(np.log(tol) / np.log(drop)) + 4


def test_batched_direct_launches_match_graph_replay(gctx):
    # per-item arithmetic does not depend on the launch path, the check interval
    # or the narrowing of the launches to the items still iterating
    import paper_2307_14437_amd as gofd
    P = _problems(gctx)
    args = ([p["tr"] for p in P], [p["op"] for p in P], [p["pc"] for p in P], [_dev(p["f"]) for p in P])
    ref, iref = gofd.solve_batched(gctx, *args, tol=1e-12, use_graph=1)
    for ug, ce in ((0, 8), (0, 1), (1, 2)):
        us, infos = gofd.solve_batched(gctx, *args, tol=1e-12, use_graph=ug, check_every=ce)
        assert [i["iterations"] for i in infos] == [i["iterations"] for i in iref], (ug, ce)
        for a, b in zip(us, ref):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), (ug, ce)


def test_shape_groups_run_concurrently_with_the_same_results(gctx):
    """Problems of different grid shapes form groups that run concurrently (a host thread and streams
    each); every item's FP64 iterates are those of the groups solved one after another (stage timing
    forces that path)."""
    import paper_2307_14437_amd as gofd
    P = _problems(gctx)
    args = ([p["tr"] for p in P], [p["op"] for p in P], [p["pc"] for p in P], [_dev(p["f"]) for p in P])
    conc, ic = gofd.solve_batched(gctx, *args, tol=1e-12)
    seq, iseq = gofd.solve_batched(gctx, *args, tol=1e-12, stage_ms=np.zeros(len(gofd.STAGES)))
    assert [i["iterations"] for i in ic] == [i["iterations"] for i in iseq]
    for a, b in zip(conc, seq):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_c4_members_of_three_grid_sizes_match_the_oracle(gctx):
    """Members of the 64-mesh star workload with 128^2, 256^2 and 512^2 grids, 16 Fourier right-hand sides
    each, solved in one batched FP32-grid call (three concurrent shape groups) to 1e-11; items checked
    against the oracle's FFT-product CG solution (same T level on both sides: M = 2048, raised to
    4096 for the 512^2 grid)."""
    import torch
    import paper_2307_14437_amd as gofd
    from workloads.configs import c4_plan, c4_problem
    plan = c4_plan()
    picks = []
    for n in (128, 256, 512):
        cand = [m for m in plan if 2 * m["grid"].N == n]
        picks.append(min(cand, key=lambda m: m["nv"]))
    probs = [c4_problem(m) for m in picks]
    trs, ops, fs = [], [], []
    for pr in probs:
        g = pr["grid"]
        print(f"c4 member: nv={pr['mesh'].nv} grid {2 * g.N} s={pr['s']:.3f}", flush=True)
        trs.append(gofd.Transfer(gctx, _dev(pr["mesh"].X), _dev(pr["mesh"].elems, torch.int32), g))
        ops.append(gofd.FdOp(gctx, pr["s"], g, M=2048))
        fs.append(_dev(np.stack(pr["f"])))
    us, infos = gofd.solve_batched(gctx, trs, ops, [None] * 3, fs, tol=1e-11, mode=gofd.MODE_FP32_RELIABLE,
                                   inner_tol=0.1)
    assert all(i["status"] == 0 and i["rel_residual"] <= 1e-11 for i in infos)
    for q, pr in enumerate(probs):
        m, g, s = pr["mesh"], pr["grid"], pr["s"]
        otr = transfer.Transfer(m.X, m.elems, 2, g.N, g.R, g.center)
        M = 2048
        while M // 2 < 2 * (2 * g.N) + 1:          # the level both sides raise M to
            M *= 2
        T = fw.filon_richardson(s, 2, 2 * g.N, M)
        u = us[q].cpu().numpy().reshape(16, -1)
        for r in ((0, 15) if q == 0 else (q * 7,)):
            b = operator.rhs_grid(otr, s, pr["f"][r])
            uJ, it, _ = osolve.pcg(lambda v: operator.apply_K(otr, T, v, "fft"), b, tol=1e-13, maxiter=5000)
            uref = np.zeros(m.nv)
            uref[otr.J] = uJ
            err = np.linalg.norm(u[r] - uref) / np.linalg.norm(uref)
            print(f"  rhs {r}: oracle iterations {it}, rel error {err:.2e}", flush=True)
            assert err <= 1e-8


def test_block_multicolour_items_of_several_problems_in_one_launch(gctx):
    """Problems preconditioned by IC(1) of the Laplacian in block multicolour order, mixed with unpreconditioned
    ones, in one shape group: their triangular solves run as one launch per colour and direction over all their
    items (each item reaching its last colour in its own launch).  Every item matches its problem solved alone
    (whose launches take the problem's arrays as arguments) and, for the smallest mesh, the oracle's dense
    solution."""
    import torch
    import paper_2307_14437_amd as gofd
    specs = [  # (mesh, R, s, precond, nrhs): one grid shape (n = 64)
        (disk_mesh(seed=31, n_boundary=30, spacing=0.14), 1.0, 0.8, "IC1_9_LAP_BMC", 2),
        (star_mesh(32, 900), 1.6, 0.3, "NONE", 1),
        (disk_mesh(seed=33, n_boundary=50, spacing=0.07), 1.05, 0.7, "IC1_9_LAP_BMC", 3),
        (star_mesh(34, 800), 1.6, 0.9, "IC1_5_LAP_BMC", 1),
    ]
    P = []
    for k, (m, R, s, pcn, nr) in enumerate(specs):
        g = grid_for_box(2, 64, R=R)
        tr = gofd.Transfer(gctx, _dev(m.X), _dev(m.elems, torch.int32), g)
        op = gofd.FdOp(gctx, s, g, M=512)
        pc = gofd.Precond(gctx, tr, op, pcn)
        f = np.stack([fourier_rhs(300 + 10 * k + r, g) for r in range(nr)])
        P.append(dict(m=m, g=g, s=s, tr=tr, op=op, pc=pc, f=f))
    colours = [p["pc"].info["colours"] for p in P if p["pc"].info["colours"]]
    print("colours", colours, flush=True)
    assert len(set(colours)) > 1 or len(colours) > 2
    for mode in (gofd.MODE_FP64, gofd.MODE_FP32_RELIABLE):
        us, infos = gofd.solve_batched(gctx, [p["tr"] for p in P], [p["op"] for p in P], [p["pc"] for p in P],
                                       [_dev(p["f"]) for p in P], tol=1e-11, mode=mode, inner_tol=0.1)
        k = 0
        for p, u in zip(P, us):
            ua, ia = gofd.solve(gctx, p["tr"], p["op"], _dev(p["f"]), tol=1e-11, pc=p["pc"], mode=mode,
                                inner_tol=0.1)
            u, ua = u.cpu().numpy().reshape(len(p["f"]), -1), ua.cpu().numpy().reshape(len(p["f"]), -1)
            for r in range(len(p["f"])):
                assert abs(infos[k]["iterations"] - ia[r]["iterations"]) <= 2, (infos[k], ia[r])
                assert infos[k]["rel_residual"] <= 1e-11
                assert np.linalg.norm(u[r] - ua[r]) <= 1e-9 * np.linalg.norm(ua[r])
                k += 1
    # the smallest preconditioned problem against the oracle's dense solve
    p = P[0]
    otr = transfer.Transfer(p["m"].X, p["m"].elems, 2, p["g"].N, p["g"].R, p["g"].center)
    T = fw.filon_richardson(p["s"], 2, 2 * p["g"].N, 512)      # the oracle's table (the GPU's matches it, 1e-13)
    K = operator.dense_K(otr, T)
    for r in range(len(p["f"])):
        uref = np.zeros(otr.nv)
        uref[otr.J] = osolve.solve_dense(K, operator.rhs_grid(otr, p["s"], p["f"][r]))
        ug = us[0].cpu().numpy().reshape(len(p["f"]), -1)[r]
        assert np.linalg.norm(ug - uref) <= 1e-9 * np.linalg.norm(uref)


def test_block_multicolour_problem_finishing_first_in_a_batch(gctx):
    """One problem preconditioned in block multicolour order (its solves take its arrays as launch arguments),
    two right-hand sides, batched with a slower unpreconditioned problem: the preconditioned items finish first
    and the later launches of their solves store nothing for them.  Every item matches its problem solved
    alone, and the finished items keep the iterates at which they stopped."""
    import torch
    import paper_2307_14437_amd as gofd
    specs = [  # (mesh, R, s, precond, nrhs): one grid shape (n = 64)
        (disk_mesh(seed=35, n_boundary=40, spacing=0.09), 1.05, 0.9, "IC1_9_LAP_BMC", 2),
        (star_mesh(36, 900), 1.6, 0.3, "NONE", 1),
    ]
    P = []
    for k, (m, R, s, pcn, nr) in enumerate(specs):
        g = grid_for_box(2, 64, R=R)
        tr = gofd.Transfer(gctx, _dev(m.X), _dev(m.elems, torch.int32), g)
        op = gofd.FdOp(gctx, s, g, M=512)
        pc = gofd.Precond(gctx, tr, op, pcn)
        f = np.stack([fourier_rhs(500 + 10 * k + r, g) for r in range(nr)])
        P.append(dict(tr=tr, op=op, pc=pc, f=f))
    for mode in (gofd.MODE_FP64, gofd.MODE_FP32_RELIABLE):
        us, infos = gofd.solve_batched(gctx, [p["tr"] for p in P], [p["op"] for p in P], [p["pc"] for p in P],
                                       [_dev(p["f"]) for p in P], tol=1e-11, mode=mode, inner_tol=0.1)
        print(mode, [i["iterations"] for i in infos], flush=True)
        assert max(i["iterations"] for i in infos[:2]) < infos[2]["iterations"]   # the BMC items stop first
        k = 0
        for p, u in zip(P, us):
            ua, ia = gofd.solve(gctx, p["tr"], p["op"], _dev(p["f"]), tol=1e-11, pc=p["pc"], mode=mode,
                                inner_tol=0.1)
            u, ua = u.cpu().numpy().reshape(len(p["f"]), -1), ua.cpu().numpy().reshape(len(p["f"]), -1)
            for r in range(len(p["f"])):
                assert infos[k]["status"] == 0
                assert abs(infos[k]["iterations"] - ia[r]["iterations"]) <= 2, (infos[k], ia[r])
                assert infos[k]["rel_residual"] <= 1e-11
                assert np.linalg.norm(u[r] - ua[r]) <= 1e-9 * np.linalg.norm(ua[r])
                k += 1
