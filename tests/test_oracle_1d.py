"""Pins of the oracle in one dimension (the 1D example of Section 5): the transfer on grid-coincident meshes,
location ties and nodes outside the mesh, and the fixed-mesh L2 rate of eq. GoFD-2 against the closed-form
solution (eq. exam-2 with k = 0)."""

import math

import numpy as np
import pytest

from oracle import exact, fdweights as fw, grid as ogrid, operator, solve, transfer
from workloads import interval_mesh


def _tr(m, N, R=1.1):
    return transfer.Transfer(m.X, m.elems, 1, N, R, (0.0,))


def test_grid_coincident_mesh():
    # vertices on every other grid node of (-1, 1): a node on a vertex has weight 1 there, a midpoint 1/2 each
    N, R = 8, 1.0
    m = interval_mesh(N, a=-1.0, b=1.0)           # spacing 2/8 = 2 h with h = R/N = 1/8
    tr = _tr(m, N, R)
    z = ogrid.node_coords(1, N, R, (0.0,))[:, 0]
    I = tr.I.toarray()
    assert np.allclose(I.sum(axis=1), 1.0)        # every node of [-1, 1] is inside
    assert np.allclose(tr.D[1:-1], 2.0) and np.allclose(tr.D[[0, -1]], 1.5)
    assert np.allclose(I @ m.X[:, 0], z)          # linear reproduction
    # a node on vertex j (0 < j < n) belongs to element j - 1 (the smaller id), with lambda_1 = 1
    on = np.nonzero(np.isclose(z[:, None], m.X[None, :, 0]).any(axis=1))[0]
    for k in on:
        j = int(np.argmin(np.abs(m.X[:, 0] - z[k])))
        assert tr.elem[k] == max(j - 1, 0)


def test_nodes_outside_the_mesh_have_zero_rows():
    m = interval_mesh(10, seed=1, jitter=0.3)
    tr = _tr(m, 12, 1.1)
    z = ogrid.node_coords(1, 12, 1.1, (0.0,))[:, 0]
    out = (z < -1.0) | (z > 1.0)
    assert np.all(tr.elem[out] == -1) and np.all(tr.I.toarray()[out] == 0.0)
    assert np.allclose(tr.I.toarray()[~out].sum(axis=1), 1.0)


def _l2(x, e):
    hx = np.diff(x)
    return np.sqrt(np.sum(hx / 3 * (e[:-1] ** 2 + e[:-1] * e[1:] + e[1:] ** 2)))


def _solve_example(n, s, ratio=2):
    """Example 5 with k = 0 on a uniform mesh of n elements, R = 1.1, h_FD = a_h / ratio (eq. hFD-1 in 1D is
    h_FD <= a_h / 2)."""
    m = interval_mesh(n)
    N = int(np.ceil(1.1 / (2.0 / n / ratio)))
    tr = _tr(m, N)
    T = fw.closed_form_1d(s, 2 * N)
    f = exact.f_ball(ogrid.node_coords(1, N, 1.1, (0.0,)), s, 1, 0)
    u = np.zeros(tr.nv)
    u[tr.J] = solve.solve_dense(operator.dense_K(tr, T), operator.rhs_grid(tr, s, f))
    ue = exact.u_ball(m.X, s, 1, 0)
    x = m.X[:, 0]
    return _l2(x, u - ue) / _l2(x, ue)


@pytest.mark.parametrize("s,rate", [(0.5, 1.0), (0.25, 0.75)])
def test_fixed_mesh_l2_rate(s, rate):
    # fixed meshes: O(h^{min(1, s + 1/2)}) in L2
    ns = (32, 64, 128, 256)
    errs = [_solve_example(n, s) for n in ns]
    slope = np.polyfit(np.log(2.0 / np.array(ns)), np.log(errs), 1)[0]
    assert errs[-1] < errs[0] / 4
    assert slope > rate - 0.25


@pytest.mark.parametrize("s", [0.1, 0.5, 0.9])
def test_closed_form_T_against_exact_ratios(s):
    # eq. T-1D-0 gives T_{p+1} / T_p = (p - s) / (p + s + 1): the log-gamma evaluation against rational arithmetic,
    # within its expected loss of |ln Gamma(p + s + 1)| eps
    from fractions import Fraction
    P = 2000
    T = fw.closed_form_1d(s, P)
    q = Fraction(str(s))
    r, ratio = Fraction(1), [1.0]
    for p in range(P):
        r = r * (p - q) / (p + q + 1)
        ratio.append(float(r))
    ratio = np.array(ratio)
    rel = np.abs(T / T[0] - ratio) / np.abs(ratio)
    loss = 8 * np.finfo(float).eps * (1 + np.abs([math.lgamma(p + s + 1) for p in range(P + 1)]))
    assert np.all(rel <= loss)
    assert T[0] == pytest.approx(math.gamma(2 * s + 1) / math.gamma(s + 1) ** 2, rel=1e-14)
