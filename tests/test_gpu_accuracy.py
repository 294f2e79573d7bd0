"""Accuracy of the GPU solves of the 2D L-shape workload (1024^2 grid, 67k
vertices, s in {0.25, 0.75}, tolerance 1e-8) against the oracle's solution of
eq. GoFD-2, solved to a relative residual of 1e-13 and stored by
tests/golden/make_c2_oracle_solution.py (a script that calls only the oracle).

The GPU side uses its own T table (Filon + Richardson on the device at the
paper's levels, pinned to the oracle's at equal M), so the comparison covers
every step of the path: location, weights, the FFT product, the transposed
transfer and CG."""

import hashlib
import os

import numpy as np
import pytest

from workloads import config_inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_oracle_solution.npz")


def _dev(a, dtype=None):
    import torch
    return torch.tensor(a, device="cuda", dtype=dtype)


@pytest.fixture(scope="module")
def c2_gpu(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    cfg = config_inputs("c2")
    m, g, f = cfg["mesh"], cfg["grid"], cfg["f"][0]
    z = np.load(GOLDEN)
    h = hashlib.sha256()
    for a in (m.X, m.elems, f):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(repr((g.d, g.N, g.R, tuple(g.center))).encode())
    if str(z["input_hash"]) != h.hexdigest()[:16]:
        pytest.fail("the stored oracle solution was made from other inputs: run "
                    "tests/golden/make_c2_oracle_solution.py again")
    tr = gofd.Transfer(gctx, _dev(m.X), _dev(m.elems, torch.int32), g)
    ops = [gofd.FdOp(gctx, s, g) for s in cfg["s"]]
    refs = [z[f"u_{s:g}"] for s in cfg["s"]]
    for s in cfg["s"]:
        assert float(z[f"true_residual_{s:g}"]) < 1e-12
    return cfg, tr, ops, refs, _dev(f)


def _errors(us, refs):
    return [float(np.linalg.norm(u.cpu().numpy() - r) / np.linalg.norm(r)) for u, r in zip(us, refs)]


@pytest.mark.parametrize("mode_name", ["MODE_FP32_RELIABLE", "MODE_FP64", "MODE_FP32_REFINE"])
def test_c2_solutions_within_1e8_of_oracle(gctx, c2_gpu, mode_name):
    """The benchmark's step (both orders in one batched call, plain CG, tolerance 1e-8) in each
    precision mode: relative L2 error against the oracle's solution at most 1e-8."""
    import paper_2307_14437_amd as gofd
    cfg, tr, ops, refs, fd = c2_gpu
    mode = getattr(gofd, mode_name)
    inner = 0.1 if mode == gofd.MODE_FP32_RELIABLE else 1e-4
    print(f"c2 batched solve {mode_name}", flush=True)
    us, infos = gofd.solve_batched(gctx, [tr] * 2, ops, [None, None], [fd, fd], tol=cfg["tol"], mode=mode,
                                   inner_tol=inner)
    errs = _errors(us, refs)
    print(mode_name, [i["iterations"] for i in infos], errs, flush=True)
    for e in errs:
        assert e <= 1e-8


@pytest.mark.parametrize("pc_name", ["IC1_9_MC", "IC1_9_LAP_BMC", "IC1_9_BMC"])
def test_c2_multicolour_ic1_solutions_within_1e8_of_oracle(gctx, c2_gpu, pc_name):
    """The same step preconditioned by IC(1) of A_h^(9) (Section 3.3) in multicolour order, in block
    multicolour order, and with the Laplacian on the 9-point pattern in place of A_FD."""
    import paper_2307_14437_amd as gofd
    cfg, tr, ops, refs, fd = c2_gpu
    pcs = [gofd.Precond(gctx, tr, op, pc_name) for op in ops]
    print(pc_name, pcs[1].info, flush=True)
    if pc_name.endswith("_MC"):
        assert pcs[1].info["levels"] <= pcs[1].info["colours"] <= 32
    else:
        assert pcs[1].info["colours"] <= 12
    for mode in (gofd.MODE_FP32_RELIABLE, gofd.MODE_FP64):
        us, infos = gofd.solve_batched(gctx, [tr] * 2, ops, pcs, [fd, fd], tol=cfg["tol"], mode=mode, inner_tol=0.1)
        errs = _errors(us, refs)
        print(mode, [i["iterations"] for i in infos], errs, flush=True)
        for e in errs:
            assert e <= 1e-8


def test_c2_tight_fp64_solve_matches_oracle(gctx, c2_gpu):
    """FP64 GPU solves driven to a relative residual of 1e-12: what remains is the difference of the two
    T tables (<= 1e-13 relative) times the condition number (~1.3e3 at s = 0.75)."""
    import paper_2307_14437_amd as gofd
    cfg, tr, ops, refs, fd = c2_gpu
    for k, s in enumerate(cfg["s"]):
        u, info = gofd.solve(gctx, tr, ops[k], fd, tol=1e-12, mode=gofd.MODE_FP64)
        e = _errors([u], [refs[k]])[0]
        print(s, info[0]["iterations"], e, flush=True)
        assert e <= 1e-9
