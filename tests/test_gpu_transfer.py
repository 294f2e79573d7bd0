"""Parity of point location, weights, the transposed structure and D (Section 3.1) with the oracle."""

import numpy as np
import pytest

from conftest import oracle_csc
from oracle import grid as ogrid, transfer
from workloads import config_inputs, disk_mesh, grid_for_box, structured_box_mesh, structured_box_mesh_3d

pytestmark = pytest.mark.gpu


def _build(gctx, mesh, grid):
    import torch
    import paper_2307_14437_amd as gofd
    X = torch.tensor(mesh.X, dtype=torch.float64, device="cuda")
    E = torch.tensor(mesh.elems, dtype=torch.int32, device="cuda")
    return gofd.Transfer(gctx, X, E, grid)


def _check_all(gctx, mesh, grid):
    import paper_2307_14437_amd as gofd
    print(f"transfer parity: {mesh.name} nv={mesh.nv} W={grid.W} d={grid.d}", flush=True)
    tr = _build(gctx, mesh, grid)
    otr = transfer.Transfer(mesh.X, mesh.elems, grid.d, grid.N, grid.R, grid.center)
    el = tr.export(gofd.TR_ELEM).cpu().numpy()
    assert np.array_equal(el, otr.elem)                                   # bit-exact location
    d1 = grid.d + 1
    vv = tr.export(gofd.TR_ELL_VERTS).cpu().numpy().reshape(-1, d1)
    ww = tr.export(gofd.TR_ELL_WEIGHTS).cpu().numpy().reshape(-1, d1)
    assert np.array_equal(vv[otr.inside], otr.verts)                      # bit-exact sparsity
    assert np.all(vv[otr.elem < 0] == -1)
    assert np.max(np.abs(ww[otr.inside] - otr.lam)) < 1e-13
    off, nodes, w = oracle_csc(otr)
    assert np.array_equal(tr.export(gofd.TR_CSC_OFFSETS).cpu().numpy(), off)
    assert np.array_equal(tr.export(gofd.TR_CSC_NODES).cpu().numpy(), nodes)
    assert np.max(np.abs(tr.export(gofd.TR_CSC_WEIGHTS).cpu().numpy() - w)) < 1e-13
    D = tr.export(gofd.TR_D).cpu().numpy()
    assert np.max(np.abs(D - otr.D) / np.maximum(otr.D, 1)) < 1e-13
    assert np.array_equal(tr.export(gofd.TR_BOUNDARY).cpu().numpy().astype(bool), otr.bnd)
    assert tr.info["n_inside"] == otr.inside.size
    assert tr.info["n_interior"] == otr.J.size
    assert tr.info["a_h"] == pytest.approx(otr.min_height(), rel=1e-12)
    return tr, otr


def test_disk_c1(gctx, c1):
    _check_all(gctx, c1["mesh"], c1["grid"])


def test_grid_coincident_2d(gctx):
    g = grid_for_box(2, 32, R=1.0)
    lo = ogrid.axis_coords(0.0, g.R, g.N)[5]
    mesh = structured_box_mesh((lo, lo), g.h, 17, 13)
    tr, otr = _check_all(gctx, mesh, g)
    assert tr.info["exact_tests"] > 0          # nodes on edges and vertices went through exact arithmetic


def test_ragged_grid_not_power_of_two(gctx):
    mesh = disk_mesh(seed=4, n_boundary=60, spacing=0.1)
    _check_all(gctx, mesh, grid_for_box(2, 42, R=1.05, center=(0.01, -0.02)))


def test_grid_coincident_3d(gctx):
    g = grid_for_box(3, 12, R=1.0)
    lo = ogrid.axis_coords(0.0, g.R, g.N)[3]
    mesh = structured_box_mesh_3d((lo, lo, lo), g.h, 5, 4, 3)
    _check_all(gctx, mesh, g)


def test_lshape_c2_full_size(gctx):
    cfg = config_inputs("c2")
    _check_all(gctx, cfg["mesh"], cfg["grid"])


def test_errors_rank_and_colsum(gctx):
    import paper_2307_14437_amd as gofd
    mesh = disk_mesh(seed=1, n_boundary=60, spacing=0.08)
    with pytest.raises(gofd.GofdError) as e:
        _build(gctx, mesh, grid_for_box(2, 8, R=1.0))        # 81 nodes < N_v
    assert e.value.code == gofd.E_RANK
    # split an element that holds no grid node at its centroid: the new interior
    # vertex has an empty patch, hence D_j = 0 (Thm IhFD needs a fine enough grid)
    g = grid_for_box(2, 26, R=1.0)
    otr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    empty = np.setdiff1d(np.arange(mesh.ne), otr.elem[otr.elem >= 0])
    e0 = int(empty[len(empty) // 2])
    a, b, c = mesh.elems[e0]
    nvtx = mesh.nv
    X2 = np.vstack([mesh.X, mesh.X[[a, b, c]].mean(axis=0)])
    E2 = np.vstack([np.delete(mesh.elems, e0, axis=0), [[a, b, nvtx], [b, c, nvtx], [c, a, nvtx]]]).astype(np.int32)
    from workloads.meshes import Mesh
    o2 = transfer.Transfer(X2, E2, 2, g.N, g.R, g.center)
    assert o2.D[nvtx] == 0 and not o2.bnd[nvtx]
    with pytest.raises(gofd.GofdError) as e:
        _build(gctx, Mesh(X2, E2), g)
    assert e.value.code == gofd.E_ZERO_COLSUM


def test_degenerate_element_rejected(gctx):
    import paper_2307_14437_amd as gofd
    from workloads.meshes import Mesh
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [0.5, 0.5], [1.0, 1.0]])
    E = np.array([[0, 1, 2], [1, 3, 2], [1, 4, 2]], dtype=np.int32)     # (1,3,2) is flat
    with pytest.raises(gofd.GofdError) as e:
        _build(gctx, Mesh(X, E), grid_for_box(2, 8, R=1.0))
    assert e.value.code == gofd.E_DEGENERATE
