"""Further pins of the oracle: eq. GoFD-3's right-hand side, the shift restart
of incomplete Cholesky, the exact ball solutions for k > 0 (eqs. exam-0,
exam-2) and the 2D Toeplitz coefficients to 1e-12 by an identity that shares
nothing with the oracle's two routes."""

import math

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

from oracle import exact, fdweights as fw, grid as ogrid, operator, precond, solve, transfer
from workloads import disk_mesh, grid_for_box, structured_box_mesh


# ---------------------------------------------------------------- eq. GoFD-3


def _spacing2_mesh():
    """Vertices on every second node of a 33^2 grid (mesh spacing 2h), squares
    split along alternating diagonals."""
    g = grid_for_box(2, 32, R=1.0)
    lo = ogrid.axis_coords(0.0, g.R, g.N)[4]
    mesh = structured_box_mesh((lo, lo), 2 * g.h, 12, 12)
    return g, mesh


def test_column_sums_on_a_spacing_two_mesh():
    # Hand count of D_j = sum_k phi_j(x_k) with the grid twice as fine as the
    # mesh: phi_j is 1 at its own node and 1/2 at the midpoint of each of its
    # edges (the only other nodes where it is nonzero).  An interior vertex
    # has 8 edges where the diagonals meet (D = 5) and 4 elsewhere (D = 3).
    g, mesh = _spacing2_mesh()
    tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    edges = set()
    for t in mesh.elems:
        for a in range(3):
            i, j = int(t[a]), int(t[(a + 1) % 3])
            edges.add((min(i, j), max(i, j)))
    deg = np.zeros(mesh.nv, dtype=int)
    for i, j in edges:
        deg[i] += 1
        deg[j] += 1
    J = tr.J
    assert set(np.unique(deg[J])) == {4, 8}
    assert np.array_equal(tr.D[J], 1.0 + 0.5 * deg[J])


def test_gofd3_rhs_with_unit_f_equals_gofd1_rhs():
    # f = 1 both at the vertices and at the grid nodes: eq. GoFD-3 multiplied
    # through by D_h has right side h^{2s} D_J, eq. GoFD-2 has h^{2s} I_J^T 1,
    # and I^T 1 = D by definition of the column sums.
    for g, mesh in (_spacing2_mesh(), (grid_for_box(2, 32, R=1.1), disk_mesh(seed=4, n_boundary=30,
                                                                             spacing=0.2))):
        tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
        assert np.ptp(tr.D[tr.J]) > 0.5                   # D is far from constant: a dropped D shows
        for s in (0.3, 0.7):
            bv = operator.rhs_vertex(tr, s, np.ones(mesh.nv))
            bg = operator.rhs_grid(tr, s, np.ones((g.W, g.W)))
            assert np.allclose(bv, bg, rtol=1e-13, atol=0)


def test_gofd3_recovers_a_manufactured_solution():
    # eq. GoFD-3 as printed: h^{-2s} D^{-1} I^T A_FD I u = f_h.  Take f_h from a
    # chosen u0 (zero on Dirichlet vertices) through A_h; solving the
    # simplified system K u_J = rhs_vertex(f_h) must give u0 back.
    mesh = disk_mesh(seed=6, n_boundary=30, spacing=0.2)
    g = grid_for_box(2, 24, R=1.1)
    tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    s = 0.6
    T = fw.filon_richardson(s, 2, 2 * g.N, 256)
    u0 = np.zeros(mesh.nv)
    u0[tr.J] = np.random.default_rng(2).standard_normal(tr.J.size)
    f_h = operator.apply_Ah(tr, T, u0, "direct") / g.h ** (2 * s)
    uJ = solve.solve_dense(operator.dense_K(tr, T), operator.rhs_vertex(tr, s, f_h))
    assert np.max(np.abs(uJ - u0[tr.J])) < 1e-11 * np.max(np.abs(u0))


# ---------------------------------------------------------------- IC shift restart


KERSHAW = np.array([[3.0, -2.0, 0.0, 2.0],
                    [-2.0, 3.0, -2.0, 0.0],
                    [0.0, -2.0, 3.0, -2.0],
                    [2.0, 0.0, -2.0, 3.0]])


def _kershaw_ic0_pivots(alpha):
    """Squared pivots of IC(0) of Kershaw's matrix with diagonal 3(1+alpha),
    worked by hand: the dropped entry is L_42 (a_42 = 0 and level 1)."""
    d = 3.0 * (1.0 + alpha)
    p2 = d - 4.0 / d                  # l22^2 = d - l21^2,          l21 = -2/sqrt(d)
    p3 = d - 4.0 / p2                 # l33^2 = d - l32^2,          l32 = -2/sqrt(p2)
    p4 = d - 4.0 / d - 4.0 / p3       # l44^2 = d - l41^2 - l43^2,  l41 = 2/sqrt(d), l43 = -2/sqrt(p3)
    return d, p2, p3, p4


def test_ic_shift_restart_on_kershaw_matrix():
    # Kershaw (1978): SPD, yet incomplete Cholesky on its own pattern meets a
    # negative pivot (l44^2 = -5 at alpha = 0).  The restart rule shifts by
    # alpha diag(A), alpha = 1e-3, 2e-3, 4e-3, ... until every pivot is positive.
    assert np.all(np.linalg.eigvalsh(KERSHAW) > 0)
    assert _kershaw_ic0_pivots(0.0)[3] == pytest.approx(-5.0, rel=1e-15)
    alpha = 1e-3
    while min(_kershaw_ic0_pivots(alpha)) <= 0.0:
        alpha *= 2
    L, a = precond.ic1(sp.csr_matrix(KERSHAW), level=0)
    assert a == alpha and a > 0.1
    piv = _kershaw_ic0_pivots(a)
    assert np.allclose(np.diag(L.toarray()) ** 2, piv, rtol=1e-13)
    As = KERSHAW + a * np.diag(np.diag(KERSHAW))
    Lc = L.tocoo()
    M = (L @ L.T).toarray()
    assert np.max(np.abs(M[Lc.row, Lc.col] - As[Lc.row, Lc.col])) < 1e-13
    assert set(zip(Lc.row.tolist(), Lc.col.tolist())) == {(0, 0), (1, 0), (1, 1), (2, 1), (2, 2), (3, 0),
                                                         (3, 2), (3, 3)}


def test_ic_level_one_on_kershaw_matrix_is_complete_cholesky():
    # level-1 fill adds (4,2), the only fill of the 4-cycle, so IC(1) is the
    # exact Cholesky factor and needs no shift
    L, a = precond.ic1(sp.csr_matrix(KERSHAW), level=1)
    assert a == 0.0
    assert np.allclose(L.toarray(), np.linalg.cholesky(KERSHAW), rtol=0, atol=1e-14)


# ---------------------------------------------------------------- exact solutions, k > 0


def _jacobi_by_hand(k, a, b, x):
    """P_k^{(a,b)} written out for k = 1, 2 (the standard normalisation)."""
    if k == 1:
        return (a + 1) + (a + b + 2) * (x - 1) / 2
    if k == 2:
        return ((a + 1) * (a + 2) / 2 + (a + 2) * (a + b + 3) * (x - 1) / 2
                + (a + b + 3) * (a + b + 4) * (x - 1) ** 2 / 8)
    raise ValueError(k)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("k", [1, 2])
def test_ball_solution_polynomial_part(d, k):
    s = 0.35
    x = np.random.default_rng(k + d).uniform(-0.6, 0.6, size=(20, d))
    r2 = np.sum(x ** 2, axis=1)
    P = _jacobi_by_hand(k, s, d / 2 - 1, 2 * r2 - 1)
    assert np.allclose(exact.u_ball(x, s, d, k), (1 - r2) ** s * P, rtol=1e-13)
    # f/P is the constant 2^{2s} Gamma(1+s+k) Gamma(d/2+s+k) / (k! Gamma(d/2+k));
    # at s = 1/2, d = 2, k = 1 it is 2 Gamma(5/2)^2 / Gamma(2) = 9 pi / 8
    c = exact.f_ball(x, s, d, k) / P
    assert np.allclose(c, c[0], rtol=1e-13)
    c12 = exact.f_ball(np.array([[0.1, 0.2]]), 0.5, 2, 1) / _jacobi_by_hand(1, 0.5, 0.0, 2 * 0.05 - 1)
    assert c12[0] == pytest.approx(9 * math.pi / 8, rel=1e-14)


@pytest.mark.parametrize("s", [0.3, 0.5, 0.8])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_ball_solution_is_the_limit_of_the_1d_fd_scheme(s, k):
    # In 1D the unit ball is (-1, 1); the uniform-grid FD scheme (closed-form T,
    # eq. T-1D-0) with u = 0 outside converges to the exact solution at the
    # rate O(h^{min(1, s+1/2)}).  A wrong constant or Jacobi normalisation in
    # (f, u) leaves an O(1) error that does not shrink.
    errs = []
    for n in (256, 1024, 4096):
        h = 2.0 / n
        x = -1 + h * np.arange(1, n)
        T = fw.closed_form_1d(s, n)
        u = scipy.linalg.solve_toeplitz(T[:n - 1], h ** (2 * s) * exact.f_ball(x[:, None], s, 1, k))
        ue = exact.u_ball(x[:, None], s, 1, k)
        errs.append(np.linalg.norm(u - ue) / np.linalg.norm(ue))
    rate = math.log(errs[0] / errs[-1]) / math.log(16)
    assert errs[-1] < 5e-3
    assert rate > min(1.0, s + 0.5) - 0.1


def test_disk_solution_k1_converges():
    # eq. exam-0 with k = 1 on the unit disk (d = 2): non-constant f, sign change of u
    s, k = 0.5, 1
    errs = []
    for nb, sp_, n in ((50, 0.116, 32), (100, 0.058, 64)):
        mesh = disk_mesh(seed=22, n_boundary=nb, spacing=sp_)
        g = grid_for_box(2, n, R=1.0)
        tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
        T = fw.filon_richardson(s, 2, 2 * g.N, 1024)
        nodes = ogrid.node_coords(2, g.N, g.R, g.center)
        b = operator.rhs_grid(tr, s, exact.f_ball(nodes, s, 2, k))
        uJ, _, _ = solve.pcg(lambda v: operator.apply_K(tr, T, v, "fft"), b, tol=1e-12, maxiter=5000)
        u = np.zeros(mesh.nv)
        u[tr.J] = uJ
        ue = exact.u_ball(mesh.X, s, 2, k)
        errs.append(exact.l2_error(mesh.X, mesh.elems, u - ue) / exact.l2_error(mesh.X, mesh.elems, ue))
    assert errs[1] < 0.05
    assert errs[0] / errs[1] > 1.6


# ---------------------------------------------------------------- 2D T to 1e-12


def _t2d_hypergeometric(s, p):
    """T_{(p,0)} in 2D from the inner integral in closed form.

    T_{(p,0)} = pi^{-2} int_0^pi cos(p x) int_0^pi (a(x) + 2 - 2 cos y)^s dy dx with
    a(x) = 4 sin^2(x/2) (eqs. FL-6, T-1), and for B < A
    int_0^pi (A - B cos y)^s dy = pi A^s 2F1(-s/2, (1-s)/2; 1; B^2/A^2)
    (binomial series of (1 - (B/A) cos y)^s, odd powers integrate to zero).
    """
    with mp.workdps(25):
        s = mp.mpf(s)

        def inner(x):
            A = 4 * mp.sin(x / 2) ** 2 + 2
            return mp.pi * A ** s * mp.hyp2f1(-s / 2, (1 - s) / 2, 1, 4 / A ** 2)

        v = mp.quad(lambda x: inner(x) * mp.cos(p * x), [0, mp.pi / 4, mp.pi / 2, mp.pi]) / mp.pi ** 2
        return float(v)


@pytest.mark.parametrize("s", [0.25, 0.5, 0.75])
def test_2d_coefficients_to_1e12(s):
    for p in (0, 1, 3):
        truth = _t2d_hypergeometric(s, p)
        assert abs(fw.bessel_route(s, (p, 0)) - truth) < 1e-12 * max(1.0, abs(truth))
    # s = 1/2 also has the elliptic form pi^{-2} int_0^pi 2 sqrt(a+4) E(4/(a+4)) dx for T_00
    if s == 0.5:
        with mp.workdps(25):
            ell = mp.quad(lambda x: 2 * mp.sqrt(4 * mp.sin(x / 2) ** 2 + 4)
                          * mp.ellipe(4 / (4 * mp.sin(x / 2) ** 2 + 4)), [0, mp.pi]) / mp.pi ** 2
        assert abs(float(ell) - _t2d_hypergeometric(0.5, 0)) < 1e-14
        assert abs(float(ell) - 1.91618279737) < 5e-12      # the value quoted with the method's survey


@pytest.mark.parametrize("s", [0.25, 0.75])
def test_filon_richardson_within_its_error_model(s):
    # after Richardson over M and M/2 the remaining error is ~C M^{-2-2s} (here M = 2^12)
    F = fw.filon_richardson(s, 2, 3, 2 ** 12)
    for p in (0, 1, 3):
        assert abs(F[0, p] - _t2d_hypergeometric(s, p)) < 50 * 4096.0 ** (-2 - 2 * s)


# ---------------------------------------------------------------- multicolour IC(1)


def test_multicolour_ic1_on_the_c1_mesh(c1):
    m, g = c1["mesh"], c1["grid"]
    tr = transfer.Transfer(m.X, m.elems, 2, g.N, g.R, g.center)
    T = fw.filon_richardson(0.5, 2, 2 * g.N, 1024)
    A = precond.Ah_pattern(tr, T, 9)
    L, perm, cp, alpha = precond.ic1_multicolour(A)
    assert alpha == 0.0
    n = A.shape[0]
    assert np.array_equal(np.sort(perm), np.arange(n))
    # a proper colouring of A's graph, colours in non-decreasing order along the factor
    Ac = A.tocoo()
    colour = np.empty(n, dtype=int)
    colour[perm] = cp
    off = Ac.row != Ac.col
    assert np.all(colour[Ac.row[off]] != colour[Ac.col[off]])
    assert np.all(np.diff(cp) >= 0)
    # greedy: every vertex of colour c > 0 has a lower-numbered neighbour of each colour below c
    Acsr = A.tocsr()
    for v in range(n):
        nb = Acsr.indices[Acsr.indptr[v]:Acsr.indptr[v + 1]]
        lower = {int(colour[j]) for j in nb if j < v}
        assert set(range(colour[v])) <= lower
    # no factor entry joins two vertices of one colour, so the levels are at most the colours
    Lc = L.tocoo()
    offl = Lc.row != Lc.col
    assert np.all(cp[Lc.row[offl]] != cp[Lc.col[offl]])
    assert precond.dependency_levels(L) <= cp.max() + 1 < 20
    # (L L^T)_ij = (P A P^T)_ij on the kept pattern, which contains the lower pattern of P A P^T
    Ap = A.tocsr()[perm][:, perm].toarray()
    M = (L @ L.T).toarray()
    assert np.max(np.abs(M[Lc.row, Lc.col] - Ap[Lc.row, Lc.col])) < 1e-12 * np.abs(Ap).max()
    lowA = np.argwhere(np.tril(Ap) != 0)
    Lmask = L.toarray() != 0
    assert np.all(Lmask[lowA[:, 0], lowA[:, 1]])
    # as a preconditioner of eq. GoFD-2 it leaves the solution unchanged and cuts iterations
    K = operator.dense_K(tr, T)
    b = operator.rhs_grid(tr, 0.5, np.ones((g.W, g.W)))
    x = solve.solve_dense(K, b)
    xm, itm, _ = solve.pcg(lambda v: K @ v, b, tol=1e-13, precond=lambda r: precond.apply_ic_ordered(L, perm, r))
    _, it0, _ = solve.pcg(lambda v: K @ v, b, tol=1e-13)
    assert np.max(np.abs(xm - x)) < 1e-11 * np.max(np.abs(x))
    assert itm < it0


# ---------------------------------------------------------------- the Laplacian in place of A_FD (Section 3.3)


def _coincident_2d(nx=9, ny=7, N=16, at=3):
    g = grid_for_box(2, N, R=1.0)
    lo = ogrid.axis_coords(0.0, g.R, g.N)[at]
    m = structured_box_mesh((lo, lo), g.h, nx, ny)
    return m, transfer.Transfer(m.X, m.elems, 2, g.N, g.R, g.center)


def test_laplacian_5_point_on_a_grid_coincident_mesh():
    # with the vertices on grid nodes I_J selects the interior vertices, so I_J^T (-Delta_h) I_J is the 5-point
    # Laplacian (times h^2) on them: 4 on the diagonal, -1 between vertices one grid step apart on an axis,
    # written out by brute force over vertex pairs
    m, tr = _coincident_2d()
    A = precond.Ah_pattern(tr, precond.laplacian_table(2, 5), 5).toarray()
    J = tr.J
    h = tr.h
    P = np.rint(m.X[J] / h).astype(int)
    ref = np.zeros((len(J), len(J)))
    for a in range(len(J)):
        for b in range(len(J)):
            dx, dy = P[b] - P[a]
            if dx == 0 and dy == 0:
                ref[a, b] = 4.0
            elif abs(dx) + abs(dy) == 1:
                ref[a, b] = -1.0
    assert np.array_equal(A, ref)


@pytest.mark.parametrize("npts", [9, 5])
def test_laplacian_pattern_is_consistent(npts):
    # interior rows far from the boundary: the stencil sums to zero on constants and gives -c h^2 Delta on x^2
    # and y^2 (c = 1 for the 5-point, 3 for the isotropic 9-point: -2 h^2 and -6 h^2)
    m, tr = _coincident_2d(nx=12, ny=12, N=16, at=1)
    A = precond.Ah_pattern(tr, precond.laplacian_table(2, npts), npts)
    X = m.X[tr.J]
    h = tr.h
    lo, hi = X.min(axis=0) + 1.5 * h, X.max(axis=0) - 1.5 * h
    deep = np.all((X > lo) & (X < hi), axis=1)
    assert deep.sum() > 20
    c = {5: 1.0, 9: 3.0}[npts]
    assert np.allclose((A @ np.ones(len(X)))[deep], 0.0, atol=1e-12)
    for a in range(2):
        q = (A @ X[:, a] ** 2)[deep]
        assert np.allclose(q, -2.0 * c * h * h, rtol=1e-10, atol=1e-14)
    # a mixed term: only the diagonal neighbours of the 9-point stencil see xy, and they cancel
    assert np.allclose((A @ (X[:, 0] * X[:, 1]))[deep], 0.0, atol=1e-12)


def test_laplacian_27_point_is_consistent():
    from workloads import structured_box_mesh_3d
    g = grid_for_box(3, 8, R=1.0)
    lo = ogrid.axis_coords(0.0, g.R, g.N)[1]
    m = structured_box_mesh_3d((lo, lo, lo), g.h, 7, 7, 7)
    tr = transfer.Transfer(m.X, m.elems, 3, g.N, g.R, g.center)
    A = precond.Ah_pattern(tr, precond.laplacian_table(3, 27), 27)
    X = m.X[tr.J]
    h = g.h
    lo3, hi3 = X.min(axis=0) + 1.5 * h, X.max(axis=0) - 1.5 * h
    deep = np.all((X > lo3) & (X < hi3), axis=1)
    assert deep.sum() >= 8
    assert np.allclose((A @ np.ones(len(X)))[deep], 0.0, atol=1e-12)
    # 18 of the 26 neighbours are one step off along a given axis: -18 h^2 on x_a^2 (a multiple of -Delta)
    for a in range(3):
        assert np.allclose((A @ X[:, a] ** 2)[deep], -18.0 * h * h, rtol=1e-10, atol=1e-14)
    assert precond.laplacian_table(3, 27)[0, 0, 0] == 26 and np.all(precond.laplacian_table(3, 27).ravel()[1:] == -1)


# ---------------------------------------------------------------- block multicolour IC(1)


def test_block_multicolour_ic1_on_the_c1_mesh(c1):
    m, g = c1["mesh"], c1["grid"]
    tr = transfer.Transfer(m.X, m.elems, 2, g.N, g.R, g.center)
    A = precond.Ah_pattern(tr, precond.laplacian_table(2, 9), 9).tocsr()
    n = A.shape[0]
    L, perm, pb, pc, alpha = precond.ic1_block_multicolour(A, 16)
    assert alpha == 0.0 and np.array_equal(np.sort(perm), np.arange(n))
    # blocks: at most 16 vertices, each connected in A's graph (grown breadth first), contiguous in the order
    starts = np.r_[0, np.nonzero(np.diff(pb))[0] + 1, n]
    assert len(np.unique(pb)) == len(starts) - 1                      # every block is one contiguous run
    assert np.max(np.diff(starts)) <= 16
    Ap = A[perm][:, perm].tocsr()
    for a, b in zip(starts[:-1], starts[1:]):
        sub = Ap[a:b, a:b]
        ncomp, _ = sp.csgraph.connected_components(sub, directed=False)
        assert ncomp == 1
    # block colours: blocks of one colour are never adjacent in A, colours non-decreasing along the order
    assert np.all(np.diff(pc) >= 0)
    Ac = Ap.tocoo()
    cross = pb[Ac.row] != pb[Ac.col]
    assert np.all(pc[Ac.row[cross]] != pc[Ac.col[cross]])
    # a block of colour c > 0 touches blocks of every colour below c (each took the smallest free colour)
    for b in np.unique(pb):
        rows = np.nonzero(pb == b)[0]
        nbrs = {int(pb[j]) for i in rows for j in Ap.indices[Ap.indptr[i]:Ap.indptr[i + 1]] if pb[j] != b}
        assert set(range(pc[rows[0]])) <= {int(pc[np.nonzero(pb == q)[0][0]]) for q in nbrs}
    # factor: no entry between two blocks of one colour; L L^T = P A P^T on the kept pattern
    Lc = L.tocoo()
    offb = pb[Lc.row] != pb[Lc.col]
    assert np.all(pc[Lc.row[offb]] != pc[Lc.col[offb]])
    M = (L @ L.T).toarray()
    Ad = Ap.toarray()
    assert np.max(np.abs(M[Lc.row, Lc.col] - Ad[Lc.row, Lc.col])) < 1e-12 * np.abs(Ad).max()
    # few colours: a triangular solve takes one step per colour
    assert pc.max() + 1 <= 8 < precond.dependency_levels(L)


def test_grow_blocks_by_hand():
    # a path 0-1-2-3-4-5 and an isolated vertex 6: blocks of 4 grow from 0 (0,1,2,3), then 4 (4,5), then 6;
    # in a star centred on 2 with leaves 0,1,3,4, blocks of 3 from 0 take 0, then 2 (its neighbour), then 1
    # (2's smallest unplaced neighbour); leaves 3 and 4 only touch the placed centre, so each is alone
    n = 7
    e = [(i, i + 1) for i in range(5)]
    A = sp.csr_matrix((np.ones(2 * len(e)), ([a for a, b in e] + [b for a, b in e], [b for a, b in e] + [a for a, b in e])),
                      shape=(n, n))
    assert precond.grow_blocks(A, 4).tolist() == [0, 0, 0, 0, 1, 1, 2]
    e = [(2, 0), (2, 1), (2, 3), (2, 4)]
    S = sp.csr_matrix((np.ones(8), ([a for a, b in e] + [b for a, b in e], [b for a, b in e] + [a for a, b in e])),
                      shape=(5, 5))
    assert precond.grow_blocks(S, 3).tolist() == [0, 0, 0, 1, 2]


def test_smallest_last_colouring_by_hand():
    # the path 0 - 2 - 3 - 1: colouring in index order needs three colours (0, 1 -> 0; 2 -> 1; 3 -> 2); smallest
    # last removes 0, 1 (degree 1), then 2 (degree 1, the smaller index of 2 and 3), then 3, and colours 3, 2, 1, 0
    e = [(0, 2), (2, 3), (3, 1)]
    A = sp.csr_matrix((np.ones(6), ([a for a, b in e] + [b for a, b in e], [b for a, b in e] + [a for a, b in e])),
                      shape=(4, 4))
    assert precond.greedy_colouring(A).tolist() == [0, 0, 1, 2]
    assert precond.smallest_last_colouring(A).tolist() == [0, 1, 1, 0]
    # a wheel: hub 0 and a rim cycle of 5 (odd): three colours for the rim, one for the hub
    rim = [(i, i % 5 + 1) for i in range(1, 6)]
    e = [(0, i) for i in range(1, 6)] + rim
    W = sp.csr_matrix((np.ones(2 * len(e)), ([a for a, b in e] + [b for a, b in e], [b for a, b in e] + [a for a, b in e])),
                      shape=(6, 6))
    c = precond.smallest_last_colouring(W)
    assert c.max() + 1 == 4 and all(c[a] != c[b] for a, b in e)
