"""Transfer matrix I_h^FD, column sums D_h and the interior vertex set (Section 3.1).

(I_h^FD)_{k,j} = phi_j(x_k^FD), the P1 (barycentric) basis functions of the
mesh evaluated at the grid nodes (eqs. interp-1, I_h_FD-1, IhFD-1).  Basis
functions vanish outside the closed mesh, so a node that lies in no closed
element gets a zero row (the homogeneous Dirichlet conformity discussed after
eq. IhFD-1).

Location (which element holds node k) is stated but not specified by the
paper; the reading used here: elem(k) = the smallest element id e whose
closed simplex contains x_k, decided by exact orientation signs, or -1.
Weights solve E lambda = [x; 1] with E = [[x_0 ... x_d], [1 ... 1]] (the
relation used in the proof of the simplex interpolation lemma).

D_{h,j} = sum_k (I_h^FD)_{k,j} (definition after eq. Ah-1; Lemma IhFD-1(iv)).
Dirichlet vertices are those on a boundary facet (a facet owned by one
element); the system is solved for the interior block only (remark after
eq. GoFD-2).
"""

from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp

from . import grid as ogrid
from .predicates import orient_signs


def _element_signs(X, elems):
    return orient_signs(X[elems])


def _contains(X, elems, eids, pts, esign):
    """Closed-simplex test for (element, point) pairs: all d+1 sub-orientations
    agree with the element's orientation or vanish."""
    d = X.shape[1]
    P = X[elems[eids]]                                # (n, d+1, d)
    ok = np.ones(len(eids), dtype=bool)
    for r in range(d + 1):
        Q = P.copy()
        Q[:, r, :] = pts
        sg = orient_signs(Q)
        ok &= (sg.astype(np.int32) * esign[eids].astype(np.int32)) >= 0
    return ok


def locate_bruteforce(X, elems, d, N, R, center) -> np.ndarray:
    """elem(k) by testing every (node, element) pair (tiny inputs only)."""
    nodes = ogrid.node_coords(d, N, R, center)
    esign = _element_signs(X, elems)
    if np.any(esign == 0):
        raise ValueError("degenerate element")
    out = -np.ones(nodes.shape[0], dtype=np.int64)
    ne = elems.shape[0]
    for k in range(nodes.shape[0]):
        eids = np.arange(ne)
        pts = np.repeat(nodes[k][None, :], ne, axis=0)
        ok = _contains(X, elems, eids, pts, esign)
        hit = np.nonzero(ok)[0]
        if hit.size:
            out[k] = hit.min()
    return out


def candidate_pairs(X, elems, d, N, R, center):
    """(element, node) pairs whose node lies in a conservative index box of the element."""
    W = 2 * N + 1
    h = ogrid.spacing(R, N)
    lo = np.array([np.float64(c) - np.float64(R) for c in center])
    P = X[elems]
    pmin = P.min(axis=1)
    pmax = P.max(axis=1)
    ilo = np.clip(np.floor((pmin - lo) / h).astype(np.int64) - 1, 0, W - 1)
    ihi = np.clip(np.ceil((pmax - lo) / h).astype(np.int64) + 1, 0, W - 1)
    ext = ihi - ilo + 1
    cnt = np.prod(ext, axis=1)
    eid = np.repeat(np.arange(elems.shape[0]), cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(eid.size) - start
    multi = np.empty((eid.size, d), dtype=np.int64)
    rem = local.copy()
    for a in range(d):
        e = ext[eid, a]
        multi[:, a] = ilo[eid, a] + rem % e
        rem //= e
    node = ogrid.node_index(multi, W)
    return eid, node


def locate(X, elems, d, N, R, center, chunk=2_000_000) -> np.ndarray:
    """elem(k) = min{e : x_k in closed K_e}, or -1 (all nodes, bucketed search)."""
    X = np.asarray(X, dtype=np.float64)
    elems = np.asarray(elems, dtype=np.int64)
    W = 2 * N + 1
    esign = _element_signs(X, elems)
    if np.any(esign == 0):
        raise ValueError("degenerate element")
    axes = [ogrid.axis_coords(center[a], R, N) for a in range(d)]
    eid, node = candidate_pairs(X, elems, d, N, R, center)
    out = np.full(W ** d, np.iinfo(np.int64).max, dtype=np.int64)
    for s0 in range(0, eid.size, chunk):
        e = eid[s0:s0 + chunk]
        k = node[s0:s0 + chunk]
        pts = np.empty((k.size, d))
        rem = k.copy()
        for a in range(d):
            pts[:, a] = axes[a][rem % W]
            rem //= W
        ok = _contains(X, elems, e, pts, esign)
        np.minimum.at(out, k[ok], e[ok])
    out[out == np.iinfo(np.int64).max] = -1
    return out


def barycentric(X, elems, elem_of_node, node_pts) -> np.ndarray:
    """lambda = E^{-1} [x; 1] for located nodes; rows (n, d+1) in element-vertex order."""
    d = X.shape[1]
    P = X[elems[elem_of_node]]                        # (n, d+1, d)
    E = np.ones((P.shape[0], d + 1, d + 1))
    E[:, :d, :] = np.transpose(P, (0, 2, 1))
    rhs = np.ones((P.shape[0], d + 1))
    rhs[:, :d] = node_pts
    return np.linalg.solve(E, rhs[:, :, None])[:, :, 0]


def boundary_vertices(elems, nv) -> np.ndarray:
    """Vertices on a facet owned by exactly one element (boolean mask)."""
    elems = np.asarray(elems, dtype=np.int64)
    d = elems.shape[1] - 1
    facets = []
    for r in range(d + 1):
        cols = [c for c in range(d + 1) if c != r]
        facets.append(elems[:, cols])
    F = np.sort(np.concatenate(facets), axis=1)
    uniq, cnt = np.unique(F, axis=0, return_counts=True)
    mask = np.zeros(nv, dtype=bool)
    mask[uniq[cnt == 1].ravel()] = True
    return mask


class Transfer:
    """I_h^FD (scipy CSR, rows = grid nodes), D_h, interior set J, and the pieces."""

    def __init__(self, X, elems, d, N, R, center, elem_of_node=None):
        X = np.asarray(X, dtype=np.float64)
        elems = np.asarray(elems, dtype=np.int64)
        self.d, self.N, self.R, self.center = d, N, float(R), tuple(center)
        self.W = 2 * N + 1
        self.h = ogrid.spacing(R, N)
        self.nv = X.shape[0]
        self.X, self.elems = X, elems
        if elem_of_node is None:
            elem_of_node = locate(X, elems, d, N, R, center)
        self.elem = elem_of_node
        inside = np.nonzero(self.elem >= 0)[0]
        nodes = ogrid.node_coords(d, N, R, center)
        self.node_pts = nodes
        lam = barycentric(X, elems, self.elem[inside], nodes[inside]) if inside.size else np.zeros((0, d + 1))
        self.inside = inside
        self.lam = lam
        self.verts = elems[self.elem[inside]] if inside.size else np.zeros((0, d + 1), dtype=np.int64)
        rows = np.repeat(inside, d + 1)
        self.I = sp.csr_matrix((lam.ravel(), (rows, self.verts.ravel())), shape=(self.W ** d, self.nv))
        self.D = np.asarray(self.I.sum(axis=0)).ravel()
        self.bnd = boundary_vertices(elems, self.nv)
        self.J = np.nonzero(~self.bnd)[0]
        self.IJ = self.I[:, self.J].tocsr()

    # ---- derived quantities used by tests (Lemma IhFD-1, Thm IhFD) ----
    def min_height(self) -> float:
        """a_h: the minimum element height (Section 3.1)."""
        d = self.d
        P = self.X[self.elems]
        vol = np.abs(np.linalg.det(P[:, 1:] - P[:, :1])) / math.factorial(d)
        a = np.inf
        for j in range(d + 1):
            oth = [k for k in range(d + 1) if k != j]
            if d == 2:
                fac = np.linalg.norm(P[:, oth[1]] - P[:, oth[0]], axis=1)
            elif d == 3:
                fac = np.linalg.norm(np.cross(P[:, oth[1]] - P[:, oth[0]], P[:, oth[2]] - P[:, oth[0]]), axis=1) / 2
            else:
                fac = np.ones(P.shape[0])
            a = min(a, float(np.min(d * vol / fac)))
        return a

    def max_diameter(self) -> float:
        P = self.X[self.elems]
        best = 0.0
        for i, j in itertools.combinations(range(self.d + 1), 2):
            best = max(best, float(np.max(np.linalg.norm(P[:, i] - P[:, j], axis=1))))
        return best
