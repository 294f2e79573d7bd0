"""The allocation-free product entry point (gofd_apply_Ah_noalloc) against gofd_apply_Ah.

Two calls in a row on different problems (the second smaller), every flag
combination of the product, a request beyond the static workspace (rejected
on the host before any kernel runs), and an operator's own workspaces still
unreserved after the allocation-free call."""

import numpy as np
import pytest

from workloads import disk_mesh, grid_for_box

pytestmark = pytest.mark.gpu


def _dev(a, dtype=None):
    import torch
    return torch.tensor(a, device="cuda", dtype=dtype)


def _problem(gctx, n, spacing, nb, seed, s):
    import torch
    import paper_2307_14437_amd as gofd
    mesh = disk_mesh(seed=seed, n_boundary=nb, spacing=spacing)
    g = grid_for_box(2, n, R=1.1)
    tr = gofd.Transfer(gctx, _dev(mesh.X), _dev(mesh.elems, torch.int32), g)
    op = gofd.FdOp(gctx, s, g, M=max(512, 8 * n))
    return mesh, g, tr, op


FLAG_SETS = ["0", "FP32_GRID", "SYMMETRIC|INTERIOR", "UNSCALED|INTERIOR|FP32_GRID", "SCALE_H2S"]


def _flags(gofd, spec):
    f = 0
    for name in spec.split("|"):
        f |= 0 if name == "0" else getattr(gofd, name)
    return f


def _check(gofd, gctx, tr, op, u, spec):
    import torch
    flags = _flags(gofd, spec)
    ref = gofd.apply_Ah(gctx, tr, op, u, flags)
    y = torch.full_like(u, float("nan"))
    gofd.apply_Ah_noalloc(gctx, tr, op, u, y, flags)
    torch.cuda.synchronize()
    scale = float(ref.abs().max())
    err = float((y - ref).abs().max()) / scale
    print(f"noalloc W={tr.W} nrhs={u.numel() // tr.nv} flags={spec}: max rel diff {err:.2e}", flush=True)
    assert err <= (1e-6 if flags & gofd.FP32_GRID else 1e-13)


def test_noalloc_matches_apply_on_two_calls_in_a_row(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    _, _, tr1, op1 = _problem(gctx, 64, 0.06, 100, 11, 0.5)
    _, _, tr2, op2 = _problem(gctx, 32, 0.12, 50, 12, 0.3)
    rng = np.random.default_rng(5)
    u1 = _dev(rng.standard_normal(3 * tr1.nv))
    u2 = _dev(rng.standard_normal(tr2.nv))
    for spec in FLAG_SETS:
        _check(gofd, gctx, tr1, op1, u1, spec)     # first call: W = 65, three fields
        _check(gofd, gctx, tr2, op2, u2, spec)     # second call: smaller grid, one field


def test_noalloc_rejects_more_than_the_static_workspace_and_allocates_nothing(gctx):
    import torch
    import paper_2307_14437_amd as gofd
    mesh, g, tr, op = _problem(gctx, 1024, 0.1, 60, 13, 0.6)        # W = 1025, FFT length 2048
    rng = np.random.default_rng(6)
    u2 = _dev(rng.standard_normal(2 * tr.nv))
    y2 = torch.empty_like(u2)
    torch.cuda.synchronize()
    # two double-precision fields of this grid need 2 * 33.6 MB > 64 MiB
    with pytest.raises(gofd.GofdError) as e:
        gofd.apply_Ah_noalloc(gctx, tr, op, u2, y2, 0)
    assert e.value.code == gofd.E_ARG and "need" in str(e.value)
    # one field fits; this operator has never reserved its own workspaces
    u1 = u2[:tr.nv].contiguous()
    y1 = torch.empty_like(u1)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    gofd.apply_Ah_noalloc(gctx, tr, op, u1, y1, 0)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    ref = gofd.apply_Ah(gctx, tr, op, u1, 0)                       # reserves the operator's buffers
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    print(f"free bytes: before {free0}, after noalloc {free1}, after apply_Ah {free2}", flush=True)
    # gofd_apply_Ah now reserves the operator's grid result, gathered field and spectra (8.4 + 8.4 +
    # 16.8 MB): had the allocation-free call reserved them, they would already exist
    assert free1 - free2 >= 30e6
    assert float((y1 - ref).abs().max()) <= 1e-13 * float(ref.abs().max())
