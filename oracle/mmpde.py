"""Mesh adaptation by the MMPDE moving mesh method (Section 4, Algorithm amGoFD), 2D.

Steps of one adaptation level, in the paper's order:

1. A recovered Hessian H_K of u_h on every element (quadratic least-squares
   fitting).  Reading: at every vertex, the quadratic polynomial fitted in
   the least-squares sense to the values of u_h at the vertices of its
   two-ring (the vertex, its neighbours and theirs); its Hessian is the
   vertex Hessian, and H_K is the mean of the vertex Hessians of K.
2. The metric tensor of eq. MK-1,
       M = det(I + |H| / alpha_h)^{-1/(d+4)} (I + |H| / alpha_h),
   |H| = sqrt(H^2), with alpha_h the root of
       sum_K |K| det(I + |H_K| / alpha_h)^{2/(d+4)} = 2 |Omega|
   (the paper prints |H_K(H_K(u))| inside this sum; the reading is |H_K(u)|).
   When every H_K vanishes the sum equals |Omega| for every alpha and there
   is no root: then M = I.  Reading: M is a field of position, the
   piecewise-linear interpolant on the mesh the move starts from of the
   vertex metrics (eq. MK-1 with the vertex Hessians).
3. The mesh energy of eq. I-h,
       I_h = 1/3 sum_K sqrt(det M_K) |K| tr(J_K M_K^{-1} J_K^T)^{3d/4}
           + d^{3d/4}/3 sum_K sqrt(det M_K) |K| (sqrt(det M_K) det F'_K)^{-3d/4},
   J_K = (F'_K)^{-1}, F_K the affine map from the equilateral reference
   simplex of unit volume onto K, and M_K the metric field at the current
   centroid of K.  The centroid is located in the starting mesh by a walk
   (from the element where it was at the last accepted step, across the edge
   opposite the most negative barycentric coordinate, until none is negative
   or the edge is on the boundary, where the value is extrapolated).  Both
   the equidistribution of the mesh and its alignment depend on M_K moving
   with the element: with M_K frozen per element the minimiser of I_h only
   grades element areas like (sqrt(det M_K))^{-1/3}.
4. The moving mesh equations (eqs. x-1, mmpde-1):
       dx_i/dt = -sqrt(det M(x_i)) / tau  dI_h/dx_i,
   with sqrt(det M(x_i)) taken at the vertex metric of the starting mesh,
   the normal component removed on the boundary (vertices slide along it),
   over t in (0, 1], tau = 1e-2, connectivity fixed.  The system is stiff
   (I_h grows like h^-3 as the mesh is refined, so an explicit step must
   shrink like tau h^3), and the paper integrates it with a stiff solver
   (MATLAB's ode15s) whose Jacobian comes from finite differences.  Reading
   of the integrator: linearly implicit (Rosenbrock-Euler) steps
       (tau/h Q^{-1} + J) dx = -dI_h/dx,   Q = diag(sqrt(det M(x_i))),
   restricted to the allowed motions (tangential on the boundary), with J
   the Hessian of I_h for the current M_K held fixed (the stiff shape
   terms; the metric's own variation is left to the right-hand side, as in
   a W-method), assembled from element Hessians taken by central
   differences of the analytic element gradient (step 1e-5 times the
   element's longest edge, then symmetrised).  A trial step is halved until
   the restricted matrix is positive definite, no element inverts and I_h
   decreases; the next trial step is twice the accepted one, or the accepted
   one itself when it had to be halved.  Integration
   stops at t = 1, or earlier once the flow is at rest: the restricted
   gradient has fallen to 1e-6 of its initial norm (the mesh then no longer
   moves, so the mesh at t = 1 is the one reached), or no step of at least
   1e-6 times the longest accepted one (and 1e-14) decreases I_h (the
   gradient of I_h jumps where a centroid crosses an edge of the starting
   mesh, and the flow comes to rest at such a kink).

The derivative dI_h/dx_i is the plain chain rule through eq. I-h (the paper
points to Huang & Kamenski for the same quantity): with E = [x_1 - x_0, ..,
x_d - x_0], V = det E, B = E_ref^T E_ref (the reference simplex's edges),
A = M^{-1}, t = tr(E^{-1} A E^{-T} B):
    dV/dE = V E^{-T},    dt/dE = -2 E^{-T} B E^{-1} A E^{-T},
and column j of dG_K/dE is the derivative with respect to vertex j of K
(j = 1..d), vertex 0 taking minus their sum.  The metric adds, at each
vertex of K, 1/(d+1) sum_c dG_K/dm_c grad m_c, m_c the components (m11, m12,
m22) and grad m_c their gradient on the element of the starting mesh that
holds the centroid; with q = sqrt(det M):
    dq/dM = q A / 2,    dt/dM = -A C A,   C = E^{-T} B E^{-1}.

Test infrastructure: plain numpy, one element or vertex at a time where a
loop is clearer.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------- topology


def vertex_rings(elems: np.ndarray, nv: int, rings: int = 2):
    """Sorted vertex sets within `rings` edges of every vertex (the vertex included)."""
    nb = [set() for _ in range(nv)]
    for t in np.asarray(elems):
        for a in t:
            nb[int(a)].update(int(b) for b in t)
    out = []
    for i in range(nv):
        cur = {i}
        for _ in range(rings):
            nxt = set(cur)
            for j in cur:
                nxt |= nb[j]
            cur = nxt
        out.append(sorted(cur))
    return out


def boundary_mask(elems: np.ndarray, nv: int) -> np.ndarray:
    """Vertices on an edge owned by one element."""
    from collections import Counter
    cnt = Counter()
    for t in np.asarray(elems):
        for a in range(3):
            e = tuple(sorted((int(t[a]), int(t[(a + 1) % 3]))))
            cnt[e] += 1
    bnd = np.zeros(nv, dtype=bool)
    for (a, b), c in cnt.items():
        if c == 1:
            bnd[a] = bnd[b] = True
    return bnd


# ---------------------------------------------------------------- Hessian recovery and metric


def vertex_hessians(X: np.ndarray, elems: np.ndarray, u: np.ndarray, rings=None) -> np.ndarray:
    """H_i (nv x 2 x 2): Hessian of the least-squares quadratic through u at vertex i's two-ring.

    Monomials in coordinates relative to x_i, scaled by the patch radius rho:
    1, dx, dy, dx^2/2, dx dy, dy^2/2 (so that the fitted coefficients of the
    last three are rho^2 times the Hessian entries)."""
    X = np.asarray(X, dtype=np.float64)
    nv = X.shape[0]
    if rings is None:
        rings = vertex_rings(elems, nv, 2)
    H = np.zeros((nv, 2, 2))
    for i in range(nv):
        P = rings[i]
        d = X[P] - X[i]
        rho = np.max(np.abs(d)) or 1.0
        d = d / rho
        Phi = np.stack([np.ones(len(P)), d[:, 0], d[:, 1], 0.5 * d[:, 0] ** 2, d[:, 0] * d[:, 1],
                        0.5 * d[:, 1] ** 2], axis=1)
        c, *_ = np.linalg.lstsq(Phi, u[P], rcond=None)
        H[i] = np.array([[c[3], c[4]], [c[4], c[5]]]) / rho ** 2
    return H


def element_hessians(elems: np.ndarray, Hv: np.ndarray) -> np.ndarray:
    return Hv[np.asarray(elems)].mean(axis=1)


def abs_sym(H: np.ndarray) -> np.ndarray:
    """|H| = sqrt(H^2) = V |Lambda| V^T for symmetric H (batched)."""
    lam, V = np.linalg.eigh(H)
    return np.einsum("...ij,...j,...kj->...ik", V, np.abs(lam), V)


def element_areas(X: np.ndarray, elems: np.ndarray) -> np.ndarray:
    P = np.asarray(X)[np.asarray(elems)]
    e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
    return 0.5 * (e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])


def alpha_h(absH: np.ndarray, areas: np.ndarray, d: int = 2) -> float:
    """Root of sum_K |K| det(I + |H_K|/alpha)^{2/(d+4)} = 2 |Omega| by bisection in log(alpha); inf if
    every |H_K| is zero (no root)."""
    lam = np.linalg.eigvalsh(absH)              # |H| is positive semidefinite
    omega = float(np.sum(areas))

    def f(alpha):
        return float(np.sum(areas * np.prod(1.0 + lam / alpha, axis=1) ** (2.0 / (d + 4)))) - 2.0 * omega

    if not np.any(lam > 0):
        return math.inf
    lo, hi = 1e-300, 1.0
    while f(hi) > 0:
        hi *= 2.0
    lo = hi / 2.0
    while f(lo) <= 0:
        lo /= 2.0
    for _ in range(200):                        # bisection in the logarithm: f decreases in alpha
        mid = math.sqrt(lo * hi)
        if f(mid) > 0:
            lo = mid
        else:
            hi = mid
        if hi / lo - 1.0 < 1e-15:
            break
    return math.sqrt(lo * hi)


def metric(absH: np.ndarray, alpha: float, d: int = 2) -> np.ndarray:
    """M_K of eq. MK-1 (batched); the identity when alpha is infinite."""
    n = absH.shape[0]
    if not math.isfinite(alpha):
        return np.broadcast_to(np.eye(d), (n, d, d)).copy()
    B = np.eye(d)[None] + absH / alpha
    return np.linalg.det(B)[:, None, None] ** (-1.0 / (d + 4)) * B


# ---------------------------------------------------------------- energy and its gradient


def reference_edges(d: int = 2) -> np.ndarray:
    """Edge matrix of the equilateral reference simplex of unit volume (2D: side a, sqrt(3)/4 a^2 = 1)."""
    if d != 2:
        raise ValueError("2D only")
    a = math.sqrt(4.0 / math.sqrt(3.0))
    return a * np.array([[1.0, 0.5], [0.0, math.sqrt(3.0) / 2.0]])


def energy(X: np.ndarray, elems: np.ndarray, M: np.ndarray) -> float:
    """I_h of eq. I-h, the metric held per element."""
    d = 2
    p = 3.0 * d / 4.0
    Er = reference_edges(d)
    Dr = np.linalg.det(Er)
    total = 0.0
    P = np.asarray(X)[np.asarray(elems)]
    for k in range(P.shape[0]):
        E = np.stack([P[k, 1] - P[k, 0], P[k, 2] - P[k, 0]], axis=1)
        V = np.linalg.det(E)
        J = Er @ np.linalg.inv(E)                # (F'_K)^{-1}, F'_K = E Er^{-1}
        q = math.sqrt(np.linalg.det(M[k]))
        area = V / math.factorial(d)
        t = np.trace(J @ np.linalg.inv(M[k]) @ J.T)
        total += q * area * t ** p / 3.0 + d ** p / 3.0 * q * area * (q * V / Dr) ** (-p)
    return total


def element_gradients(X: np.ndarray, elems: np.ndarray, M: np.ndarray) -> np.ndarray:
    """dG_K/dx for the three vertices of every element (N_e x 3 x 2), by the chain rule through eq. I-h
    (see the module docstring); batched over elements."""
    d = 2
    p = 3.0 * d / 4.0
    Er = reference_edges(d)
    Dr = np.linalg.det(Er)
    B = Er.T @ Er
    P = np.asarray(X)[np.asarray(elems)]
    E = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=2)      # columns x_1 - x_0, x_2 - x_0
    V = np.linalg.det(E)
    Ei = np.linalg.inv(E)
    EiT = np.transpose(Ei, (0, 2, 1))
    A = np.linalg.inv(M)
    q = np.sqrt(np.linalg.det(M))
    X1 = Ei @ A @ EiT
    t = np.einsum("kij,ji->k", X1, B)
    dV = V[:, None, None] * EiT
    dt = -2.0 * EiT @ B @ X1
    fac = q / math.factorial(d)
    g1 = (fac / 3.0 * t ** p)[:, None, None] * dV + (fac / 3.0 * V * p * t ** (p - 1.0))[:, None, None] * dt
    g2 = (d ** p / 3.0 * fac * (q / Dr) ** (-p) * (1.0 - p) * V ** (-p))[:, None, None] * dV
    gE = g1 + g2
    g = np.empty(P.shape)
    g[:, 1] = gE[:, :, 0]
    g[:, 2] = gE[:, :, 1]
    g[:, 0] = -(gE[:, :, 0] + gE[:, :, 1])
    return g


def energy_gradient(X: np.ndarray, elems: np.ndarray, M: np.ndarray) -> np.ndarray:
    """dI_h/dx_i (nv x 2): the element gradients summed at the vertices."""
    X = np.asarray(X)
    g = element_gradients(X, elems, M)
    G = np.zeros_like(X)
    for a in range(3):
        np.add.at(G, np.asarray(elems)[:, a], g[:, a])
    return G


def element_hessians_fd(X: np.ndarray, elems: np.ndarray, M: np.ndarray, rel_step: float = 1e-5) -> np.ndarray:
    """Hessian of every element's term of I_h with respect to its six coordinates (N_e x 6 x 6, in the
    order x_0, y_0, x_1, .., y_2), by central differences of element_gradients with the step rel_step
    times the element's longest edge, symmetrised."""
    X = np.asarray(X)
    elems = np.asarray(elems)
    P = X[elems]
    edge = np.max(np.stack([np.linalg.norm(P[:, a] - P[:, (a + 1) % 3], axis=1) for a in range(3)], 1), 1)
    eps = rel_step * edge
    ne = P.shape[0]
    H = np.empty((ne, 6, 6))
    loc = np.arange(3, dtype=np.int64)[None].repeat(ne, 0)
    for c in range(6):
        Pp, Pm = P.copy(), P.copy()
        Pp[:, c // 2, c % 2] += eps
        Pm[:, c // 2, c % 2] -= eps
        Xp, Xm = Pp.reshape(-1, 2), Pm.reshape(-1, 2)             # every element on its own three points
        el = loc + 3 * np.arange(ne)[:, None]
        H[:, :, c] = (element_gradients(Xp, el, M) - element_gradients(Xm, el, M)).reshape(ne, 6) / (2 * eps[:, None])
    return 0.5 * (H + np.transpose(H, (0, 2, 1)))


def assemble_hessian(elems: np.ndarray, H: np.ndarray, nv: int) -> sp.csr_matrix:
    """Sum of the element Hessians into the (2 nv x 2 nv) Hessian of I_h (unknowns x_0, y_0, x_1, ..)."""
    idx = (2 * np.asarray(elems, dtype=np.int64)[:, :, None] + np.arange(2)[None, None]).reshape(-1, 6)
    rows = np.repeat(idx, 6, axis=1).ravel()
    cols = np.tile(idx, (1, 6)).ravel()
    return sp.csr_matrix((H.ravel(), (rows, cols)), shape=(2 * nv, 2 * nv))


# ---------------------------------------------------------------- moving the mesh


def velocity(X, elems, M, bnd, qv, tau=1e-2):
    """Right side of eq. x-1 for per-element metrics M; boundary vertices (on the unit circle) keep their
    tangential component."""
    X = np.asarray(X)
    v = -(np.asarray(qv) / tau)[:, None] * energy_gradient(X, elems, M)
    n = X[bnd] / np.linalg.norm(X[bnd], axis=1)[:, None]
    v[bnd] -= np.sum(v[bnd] * n, axis=1)[:, None] * n
    return v


# ---------------------------------------------------------------- the metric as a field of position


def element_neighbours(elems: np.ndarray) -> np.ndarray:
    """(N_e x 3): the element across the edge opposite corner a of element k, or -1 on the boundary."""
    elems = np.asarray(elems)
    nb = -np.ones((elems.shape[0], 3), dtype=np.int64)
    seen = {}
    for k, t in enumerate(elems):
        for a in range(3):
            e = tuple(sorted((int(t[(a + 1) % 3]), int(t[(a + 2) % 3]))))
            if e in seen:
                k2, a2 = seen.pop(e)
                nb[k, a], nb[k2, a2] = k2, k
            else:
                seen[e] = (k, a)
    return nb


def barycentric(Xb: np.ndarray, elems: np.ndarray, k: int, x: np.ndarray) -> np.ndarray:
    P = Xb[elems[k]]
    T = np.stack([P[1] - P[0], P[2] - P[0]], axis=1)
    l12 = np.linalg.solve(T, np.asarray(x) - P[0])
    return np.array([1.0 - l12[0] - l12[1], l12[0], l12[1]])


def walk(Xb, elems, nb, k, x, max_moves=10000):
    """Element of the starting mesh holding x and x's barycentric coordinates there: from element k, cross
    the edge opposite the most negative coordinate until none is negative or that edge is on the boundary."""
    for _ in range(max_moves):
        lam = barycentric(Xb, elems, k, x)
        a = int(np.argmin(lam))
        if lam[a] >= 0.0 or nb[k, a] < 0:
            return k, lam
        k = int(nb[k, a])
    raise RuntimeError("point location did not end")


class MetricField:
    """Piecewise-linear metric on the starting mesh (Xb, elems) from vertex metrics Mv (N_v x 2 x 2)."""

    def __init__(self, Xb, elems, Mv):
        self.Xb = np.array(Xb, dtype=np.float64)
        self.elems = np.asarray(elems)
        self.m = np.stack([Mv[:, 0, 0], Mv[:, 0, 1], Mv[:, 1, 1]], axis=1)      # components m11, m12, m22
        self.nb = element_neighbours(self.elems)
        # gradient of each component on each element: grad^T [x1 - x0, x2 - x0] = [f1 - f0, f2 - f0]
        P = self.Xb[self.elems]
        T = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=2)
        f = self.m[self.elems]                                                   # ne x 3 corners x 3 comps
        df = np.stack([f[:, 1] - f[:, 0], f[:, 2] - f[:, 0]], axis=1)           # ne x 2 x 3
        self.grad = np.transpose(np.linalg.solve(np.transpose(T, (0, 2, 1)), df), (0, 2, 1))  # ne x 3 x 2

    def at_centroids(self, X, loc):
        """(M_K as N_e x 2 x 2, gradients of the components N_e x 3 x 2, new locations)."""
        C = np.asarray(X)[self.elems].mean(axis=1)
        ne = self.elems.shape[0]
        M3 = np.empty((ne, 3))
        G = np.empty((ne, 3, 2))
        loc = np.array(loc)
        for k in range(ne):
            kb, lam = walk(self.Xb, self.elems, self.nb, int(loc[k]), C[k])
            loc[k] = kb
            M3[k] = lam @ self.m[self.elems[kb]]
            G[k] = self.grad[kb]
        M = np.stack([np.stack([M3[:, 0], M3[:, 1]], 1), np.stack([M3[:, 1], M3[:, 2]], 1)], 1)
        return M, G, loc


def metric_derivatives(X: np.ndarray, elems: np.ndarray, M: np.ndarray) -> np.ndarray:
    """dG_K/dm_c (N_e x 3) for the components m11, m12, m22 of M_K (m12 standing for both off-diagonal
    entries), by the formulas in the module docstring."""
    d = 2
    p = 3.0 * d / 4.0
    Er = reference_edges(d)
    Dr = np.linalg.det(Er)
    B = Er.T @ Er
    P = np.asarray(X)[np.asarray(elems)]
    E = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=2)
    V = np.linalg.det(E)
    Ei = np.linalg.inv(E)
    C = np.transpose(Ei, (0, 2, 1)) @ B @ Ei
    A = np.linalg.inv(M)
    q = np.sqrt(np.linalg.det(M))
    t = np.einsum("kij,kji->k", A, C)
    area = V / math.factorial(d)
    # G = q |K| t^p / 3 + d^p / 3 q |K| (q V / Dr)^{-p}
    dG_dq = area * t ** p / 3.0 + d ** p / 3.0 * area * (1.0 - p) * q ** (-p) * (V / Dr) ** (-p)
    dG_dt = q * area * p * t ** (p - 1.0) / 3.0
    ACA = A @ C @ A
    dq = np.stack([0.5 * q * A[:, 0, 0], q * A[:, 0, 1], 0.5 * q * A[:, 1, 1]], axis=1)
    dt = np.stack([-ACA[:, 0, 0], -2.0 * ACA[:, 0, 1], -ACA[:, 1, 1]], axis=1)
    return dG_dq[:, None] * dq + dG_dt[:, None] * dt


def energy_field(X, elems, field: MetricField, loc):
    """(I_h, dI_h/dx (N_v x 2), M_K, new locations) with M_K the field at the current centroids;
    I_h = inf (and no gradient) when an element has non-positive area."""
    X = np.asarray(X)
    M, GM, loc = field.at_centroids(X, loc)
    if not np.all(element_areas(X, elems) > 0):
        return math.inf, None, M, loc
    g = element_gradients(X, elems, M) + (np.einsum("kc,kcd->kd", metric_derivatives(X, elems, M), GM)
                                          / 3.0)[:, None, :]
    G = np.zeros_like(X)
    for a in range(3):
        np.add.at(G, np.asarray(elems)[:, a], g[:, a])
    return energy(X, elems, M), G, M, loc


def motion_basis(X: np.ndarray, bnd: np.ndarray, boundary: str = "circle") -> sp.csr_matrix:
    """Columns spanning the allowed vertex motions (2 nv x n_dof): x and y for an interior vertex, the
    unit tangent of the circle through a boundary vertex ("circle"), nothing for it ("fixed")."""
    X = np.asarray(X)
    rows, cols, vals = [], [], []
    k = 0
    for i in range(X.shape[0]):
        if not bnd[i]:
            rows += [2 * i, 2 * i + 1]
            cols += [k, k + 1]
            vals += [1.0, 1.0]
            k += 2
        elif boundary == "circle":
            r = math.hypot(X[i, 0], X[i, 1])
            rows += [2 * i, 2 * i + 1]
            cols += [k, k]
            vals += [-X[i, 1] / r, X[i, 0] / r]
            k += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * X.shape[0], k))


def place(Y: np.ndarray, bnd: np.ndarray, boundary: str = "circle") -> np.ndarray:
    """Boundary vertices put back on the unit circle."""
    if boundary == "circle":
        Y[bnd] /= np.linalg.norm(Y[bnd], axis=1)[:, None]
    return Y


def implicit_step(X, bnd, qv, h, G, J, tau=1e-2, boundary="circle"):
    """One linearly implicit step of length h: X + B z with (B^T (tau/h Q^{-1} + J) B) z = -B^T G.
    Returns None when that matrix is not positive definite."""
    X = np.asarray(X)
    Bm = motion_basis(X, bnd, boundary)
    A = (Bm.T @ (J + sp.diags(np.repeat(tau / (h * np.asarray(qv)), 2))) @ Bm).toarray()
    try:
        L = np.linalg.cholesky(A)
    except np.linalg.LinAlgError:
        return None
    z = np.linalg.solve(L.T, np.linalg.solve(L, -(Bm.T @ np.asarray(G).ravel())))
    return place(X + (Bm @ z).reshape(-1, 2), bnd, boundary)


def move_mesh(X, elems, Mv, bnd, tau=1e-2, t_end=1.0, dt0=1e-3, max_steps=400, gtol=1e-6, boundary="circle",
              fixed_dt=0.0):
    """Integrate eq. x-1 over (0, t_end] for the vertex metrics Mv (N_v x 2 x 2) of the mesh X, with the
    linearly implicit steps and the step control of the module docstring.  With fixed_dt > 0: exactly
    max_steps steps of that length, no energy test and no gradient stop.
    Returns (new X, accepted steps, dict with t, rejected, energy and gradient norms)."""
    X = np.array(X, dtype=np.float64)
    elems = np.asarray(elems)
    field = MetricField(X, elems, Mv)
    qv = np.sqrt(np.linalg.det(Mv))
    loc = np.arange(elems.shape[0])
    I0, G, M, loc = energy_field(X, elems, field, loc)
    I_start = I0
    t, dt, steps, rejected, h_max = 0.0, (fixed_dt if fixed_dt > 0 else dt0), 0, 0, 0.0
    g0 = float(np.linalg.norm(motion_basis(X, bnd, boundary).T @ G.ravel()))
    gn = g0
    while steps < max_steps and (fixed_dt > 0 or t < t_end):
        if fixed_dt <= 0 and gn <= gtol * g0:
            break
        J = assemble_hessian(elems, element_hessians_fd(X, elems, M), X.shape[0])
        h = dt if fixed_dt > 0 else min(dt, t_end - t)
        halved = False
        while True:
            Y = implicit_step(X, bnd, qv, h, G, J, tau, boundary)
            if fixed_dt > 0:
                if Y is None:
                    raise np.linalg.LinAlgError("step system not positive definite")
                I1, G1, M1, loc1 = energy_field(Y, elems, field, loc)
                break
            if Y is not None and np.all(element_areas(Y, elems) > 0):
                I1, G1, M1, loc1 = energy_field(Y, elems, field, loc)
                if I1 < I0:
                    break
            h *= 0.5
            rejected += 1
            halved = True
            if h < 1e-14 or h < 1e-6 * h_max:
                return X, steps, dict(t=t, rejected=rejected, energy_start=I_start, energy_end=I0, grad0=g0,
                                      grad=gn)
        X, I0, G, M, loc, t, steps = Y, I1, G1, M1, loc1, t + h, steps + 1
        h_max = max(h_max, h)
        gn = float(np.linalg.norm(motion_basis(X, bnd, boundary).T @ G.ravel())) if G is not None else math.inf
        if fixed_dt <= 0:
            dt = h if halved else 2.0 * h
    return X, steps, dict(t=t, rejected=rejected, energy_start=I_start, energy_end=I0, grad0=g0, grad=gn)


# ---------------------------------------------------------------- Algorithm amGoFD


def level_metric(X, elems, u, rings=None):
    """(vertex metrics N_v x 2 x 2, alpha_h) of one adaptation level: vertex Hessians, alpha_h from the
    element Hessians, eq. MK-1 at the vertices."""
    Hv = vertex_hessians(X, elems, u, rings)
    alpha = alpha_h(abs_sym(element_hessians(elems, Hv)), element_areas(X, elems))
    return metric(abs_sym(Hv), alpha), alpha


def adapt(X, elems, solve_on, levels=5, tau=1e-2, max_steps=400):
    """Algorithm amGoFD: for each level, u = solve_on(X) on the current mesh, then a new mesh from the
    MMPDE method driven by u.  Returns the list of (X, u) of every level; the connectivity never changes."""
    X = np.array(X, dtype=np.float64)
    elems = np.asarray(elems)
    bnd = boundary_mask(elems, X.shape[0])
    rings = vertex_rings(elems, X.shape[0], 2)
    out = []
    for _ in range(levels):
        u = solve_on(X)
        out.append((X.copy(), u))
        Mv, _ = level_metric(X, elems, u, rings)
        X, _, _ = move_mesh(X, elems, Mv, bnd, tau=tau, max_steps=max_steps)
    return out
