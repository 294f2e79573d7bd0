"""Sparse preconditioner for GoFD-2 (Section 3.3, "Preconditioning with sparse matrices").

1. Take the entries of A_FD on a Laplacian-like pattern: 5-point or 9-point
   in 2D (the paper), 27-point in 3D (Example 4).  This is the matrix
   A_FD^(p) whose entry for nodes j, m is T_{j-m} when j - m lies in the
   pattern and 0 otherwise.
2. A_h^(p) = I^T A_FD^(p) I  (eq. Ah-4), restricted to the interior block.
3. Incomplete Cholesky of A_h^(p) with level-1 fill-in.

The paper does not define the level-of-fill rule, the ordering, or what
happens on a non-positive pivot.  Readings: the classical level-of-fill rule
(lev = 0 on the pattern of the matrix, lev(i,j) = min over k < min(i,j) of
lev(i,k) + lev(k,j) + 1, keep lev <= 1), the vertex numbering given with the
mesh, and on a pivot <= 0 a restart on A + alpha diag(A) with alpha = 1e-3,
doubled until the factorisation succeeds.

Counts of iterations that the preconditioner saves are shown in the paper
only in figures, so the iteration counts themselves are "parity unpinned".

Multicolour variant (a reading for data-parallel triangular solves; the
paper fixes no ordering): colour the graph of A greedily (vertices in index
order, each taking the smallest colour that no already coloured neighbour
has), order the vertices by (colour, index), and factor P A P^T with the
level-1 fill kept only between vertices of different colours.  Vertices of
one colour are then never coupled in the factor, so a triangular solve has at
most as many dependency levels as there are colours.

Block multicolour variant (the same reading with blocks of at most 16
vertices grown breadth first, the blocks coloured in smallest-last order
instead of the vertices; ic1_block_multicolour): far fewer colours, each
block's own rows solved together.

Laplacian variant: the discrete Laplacian on the pattern in place of A_FD's
entries (laplacian_table), the alternative Section 3.3 names.
"""

from __future__ import annotations

import heapq
import math

import numpy as np
import scipy.sparse as sp

PATTERNS = {"IC1_5": 5, "IC1_9": 9, "IC1_27": 27}


def stencil_offsets(d: int, npts: int):
    """Offsets of the 5-, 9- or 27-point pattern."""
    if d == 2 and npts == 5:
        return [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    if d == 2 and npts == 9:
        return [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    if d == 3 and npts == 7:
        return [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    if d == 3 and npts == 27:
        return [(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    raise ValueError("unsupported pattern")


def afd_pattern_matrix(T, d, W, npts) -> sp.csr_matrix:
    """A_FD^(p): the entries of A_FD on the stencil pattern (step 1)."""
    n = W ** d
    idx = np.indices((W,) * d).reshape(d, -1)    # idx[0] slowest = coordinate axis d-1
    rows, cols, vals = [], [], []
    k = np.arange(n)
    for off in stencil_offsets(d, npts):
        ok = np.ones(n, dtype=bool)
        nb = np.zeros(n, dtype=np.int64)
        mult = 1
        for a in range(d):                        # coordinate axis a
            ia = idx[d - 1 - a] + off[a]
            ok &= (ia >= 0) & (ia < W)
            nb += np.clip(ia, 0, W - 1) * mult
            mult *= W
        rows.append(k[ok])
        cols.append(nb[ok])
        tv = T[tuple(abs(off[a]) for a in reversed(range(d)))]
        vals.append(np.full(int(ok.sum()), tv))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def Ah_pattern(tr, T, npts) -> sp.csr_matrix:
    """A_h^(p) = I_J^T A_FD^(p) I_J on the interior block (eq. Ah-4).  T is indexed by the absolute offsets
    (|o_{d-1}|, ..., |o_0|): the table of A_FD, or laplacian_table(d, npts)."""
    Ap = afd_pattern_matrix(T, tr.d, tr.W, npts)
    return (tr.IJ.T @ Ap @ tr.IJ).tocsr()


def laplacian_table(d: int, npts: int) -> np.ndarray:
    """The discrete Laplacian on the p-point pattern, to take the place of A_FD in the stiffness matrix
    (Section 3.3 names the direct use of the Laplacian as a preconditioner): p - 1 at the centre and -1 at each
    of the other p - 1 points, i.e. h^2 (-Delta_h) for the standard 5-point stencil and a multiple of it for the
    isotropic 9-point (factor 3) and compact 27-point stencils.  The factor does not change preconditioned CG.
    Indexed like T, by absolute offsets (all at most 1)."""
    stencil_offsets(d, npts)                        # only the supported patterns
    t = np.full((2,) * d, -1.0)
    t[(0,) * d] = npts - 1
    return t


def ic1_pattern(A: sp.csr_matrix, level: int = 1):
    """Lower-triangular pattern of incomplete factorisation with level-of-fill <= level.

    Row by row (Gaussian-elimination order): start from the structural
    pattern of row i (level 0); for each k < i in the row, in increasing
    order, propagate lev(i,j) = min(lev(i,j), lev(i,k) + lev(k,j) + 1) for the
    upper part j > k of the already-final row k.  Symmetric A: the lower
    pattern is the transpose of the upper pattern.
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    upper_levels = [None] * n   # row k: dict j -> lev for j > k (the part of U used later)
    lower_rows = []
    for i in range(n):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        lev = {int(j): 0 for j in cols}
        lev[i] = 0
        k_list = sorted(j for j in lev if j < i)
        heap = list(k_list)
        heapq.heapify(heap)
        seen = set(k_list)
        while heap:
            k = heapq.heappop(heap)
            lik = lev[k]
            if lik > level:
                continue
            for j, lkj in upper_levels[k].items():
                nl = lik + lkj + 1
                if nl <= level and nl < lev.get(j, level + 1):
                    lev[j] = nl
                    if j < i and j not in seen:
                        heapq.heappush(heap, j)
                        seen.add(j)
        kept = {j: l for j, l in lev.items() if l <= level}
        upper_levels[i] = {j: l for j, l in kept.items() if j > i}
        lower_rows.append(sorted(j for j in kept if j <= i))
    return lower_rows


def ic_numeric(A: sp.csr_matrix, lower_rows):
    """Incomplete Cholesky on a given lower pattern: (L L^T)_ij = a_ij on the pattern.

    Row-oriented: for j < i in the pattern of row i,
      L_ij = (a_ij - sum_{k<j} L_ik L_jk) / L_jj,
      L_ii = sqrt(a_ii - sum_{k<i} L_ik^2);
    contributions outside the pattern are dropped.  Returns (L as CSR, ok).
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    rows = []
    for i in range(n):
        a_row = {int(j): float(v) for j, v in zip(A.indices[A.indptr[i]:A.indptr[i + 1]],
                                                  A.data[A.indptr[i]:A.indptr[i + 1]])}
        Li = {}
        for j in lower_rows[i]:
            if j == i:
                continue
            acc = a_row.get(j, 0.0)
            Lj = rows[j]
            for k, v in Li.items():
                if k < j and k in Lj:
                    acc -= v * Lj[k]
            Li[j] = acc / Lj[j]
        diag = a_row.get(i, 0.0) - sum(v * v for v in Li.values())
        if not diag > 0.0:
            return None, False
        Li[i] = math.sqrt(diag)
        rows.append(Li)
    indptr = [0]
    ind, val = [], []
    for i in range(n):
        for j in sorted(rows[i]):
            ind.append(j)
            val.append(rows[i][j])
        indptr.append(len(ind))
    return sp.csr_matrix((np.array(val), np.array(ind), np.array(indptr)), shape=(n, n)), True


def ic1(A: sp.csr_matrix, level: int = 1):
    """IC(level) with the diagonal-shift restart; returns (L, alpha)."""
    A = sp.csr_matrix(A)
    pattern = ic1_pattern(A, level)
    alpha = 0.0
    while True:
        As = A if alpha == 0.0 else (A + alpha * sp.diags(A.diagonal())).tocsr()
        L, ok = ic_numeric(As, pattern)
        if ok:
            return L, alpha
        alpha = 1e-3 if alpha == 0.0 else 2 * alpha


def apply_ic(L: sp.csr_matrix, r: np.ndarray) -> np.ndarray:
    """z = (L L^T)^{-1} r by a forward then a backward triangular solve."""
    from scipy.sparse.linalg import spsolve_triangular
    y = spsolve_triangular(L, r, lower=True)
    return spsolve_triangular(L.T.tocsr(), y, lower=False)


def greedy_colouring(A: sp.csr_matrix) -> np.ndarray:
    """Colour of each vertex: in index order, the smallest colour not used by an already coloured
    neighbour in the graph of A."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    colour = -np.ones(n, dtype=np.int64)
    for i in range(n):
        taken = {int(colour[j]) for j in A.indices[A.indptr[i]:A.indptr[i + 1]] if colour[j] >= 0}
        c = 0
        while c in taken:
            c += 1
        colour[i] = c
    return colour


def ic1_multicolour(A: sp.csr_matrix, level: int = 1):
    """Multicolour IC(level): returns (L for P A P^T, perm, colour of each factor row, alpha), where
    row i of L is vertex perm[i] and the fill between equal colours is dropped."""
    A = sp.csr_matrix(A)
    colour = greedy_colouring(A)
    perm = np.lexsort((np.arange(A.shape[0]), colour))
    Ap = A[perm][:, perm].tocsr()
    cp = colour[perm]
    pattern = [[j for j in row if j == i or cp[j] != cp[i]] for i, row in enumerate(ic1_pattern(Ap, level))]
    alpha = 0.0
    while True:
        As = Ap if alpha == 0.0 else (Ap + alpha * sp.diags(Ap.diagonal())).tocsr()
        L, ok = ic_numeric(As, pattern)
        if ok:
            return L, perm, cp, alpha
        alpha = 1e-3 if alpha == 0.0 else 2 * alpha


def smallest_last_colouring(A: sp.csr_matrix) -> np.ndarray:
    """Colour of each vertex in Matula and Beck's smallest-last order: vertices are removed one at a time, each
    time one of least degree among those left (ties: the smallest index), and coloured in the reverse of that
    order, each the smallest colour not used by an already coloured neighbour.  It uses at most one colour more
    than the graph's degeneracy."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    nbrs = [[int(j) for j in A.indices[A.indptr[v]:A.indptr[v + 1]] if j != v] for v in range(n)]
    deg = [len(x) for x in nbrs]
    heap = [(deg[v], v) for v in range(n)]
    heapq.heapify(heap)
    removed = [False] * n
    order = []
    while heap:
        d, v = heapq.heappop(heap)
        if removed[v] or d != deg[v]:
            continue
        removed[v] = True
        order.append(v)
        for j in nbrs[v]:
            if not removed[j]:
                deg[j] -= 1
                heapq.heappush(heap, (deg[j], j))
    colour = -np.ones(n, dtype=np.int64)
    for v in reversed(order):
        taken = {int(colour[j]) for j in nbrs[v] if colour[j] >= 0}
        c = 0
        while c in taken:
            c += 1
        colour[v] = c
    return colour


def grow_blocks(A: sp.csr_matrix, size: int) -> np.ndarray:
    """Block of each vertex: vertices in index order, each not yet in a block starts one, which then takes
    not yet placed vertices breadth first (a vertex's neighbours in increasing index) until it has `size`."""
    A = sp.csr_matrix(A, copy=True)
    A.sort_indices()
    n = A.shape[0]
    blk = -np.ones(n, dtype=np.int64)
    nb = 0
    for v in range(n):
        if blk[v] >= 0:
            continue
        blk[v] = nb
        queue, head, count = [v], 0, 1
        while head < len(queue) and count < size:
            u = queue[head]
            head += 1
            for j in A.indices[A.indptr[u]:A.indptr[u + 1]]:
                if count == size:
                    break
                if blk[j] < 0:
                    blk[j] = nb
                    queue.append(int(j))
                    count += 1
        nb += 1
    return blk


def ic1_block_multicolour(A: sp.csr_matrix, size: int = 16, level: int = 1):
    """Block multicolour IC(level), a reading for triangular solves with few device-wide steps: vertices are
    grouped into blocks of at most `size` (grow_blocks), the graph of the blocks (two blocks adjacent when A
    couples a vertex of one to a vertex of the other) is coloured in smallest-last order, the vertices are
    ordered by (colour of their block, block, index) and P A P^T is factored keeping the level-`level` fill
    inside a block and between blocks of different colours (blocks of one colour are never coupled, so a
    triangular solve takes one step per colour, each block solved on its own).  Returns (L, perm, block of
    each factor row, colour of each factor row, alpha)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    blk = grow_blocks(A, size)
    nb = int(blk.max()) + 1 if n else 0
    Ac = A.tocoo()
    off = blk[Ac.row] != blk[Ac.col]
    G = sp.csr_matrix((np.ones(int(off.sum())), (blk[Ac.row[off]], blk[Ac.col[off]])), shape=(nb, nb))
    bcol = smallest_last_colouring(G)
    perm = np.lexsort((np.arange(n), blk, bcol[blk]))
    Ap = A[perm][:, perm].tocsr()
    pb = blk[perm]
    pc = bcol[pb]
    pattern = [[j for j in row if pb[j] == pb[i] or pc[j] != pc[i]] for i, row in enumerate(ic1_pattern(Ap, level))]
    alpha = 0.0
    while True:
        As = Ap if alpha == 0.0 else (Ap + alpha * sp.diags(Ap.diagonal())).tocsr()
        L, ok = ic_numeric(As, pattern)
        if ok:
            return L, perm, pb, pc, alpha
        alpha = 1e-3 if alpha == 0.0 else 2 * alpha


def apply_ic_ordered(L: sp.csr_matrix, perm: np.ndarray, r: np.ndarray) -> np.ndarray:
    """z = P^T (L L^T)^{-1} P r for a factor in the order perm."""
    z = np.empty_like(r)
    z[perm] = apply_ic(L, r[perm])
    return z


def dependency_levels(L: sp.csr_matrix) -> int:
    """Longest chain of the forward solve: level(i) = 1 + max level of the columns j < i of row i."""
    L = sp.csr_matrix(L)
    lev = np.zeros(L.shape[0], dtype=np.int64)
    for i in range(L.shape[0]):
        cols = L.indices[L.indptr[i]:L.indptr[i + 1]]
        cols = cols[cols < i]
        lev[i] = lev[cols].max() + 1 if cols.size else 0
    return int(lev.max()) + 1 if L.shape[0] else 0

