"""Mesh adaptation by the MMPDE moving mesh method (Section 4, Algorithm amGoFD), 2D.

Steps of one adaptation level, in the paper's order:

1. A recovered Hessian H_K of u_h on every element (quadratic least-squares
   fitting).  Reading: at every vertex, the quadratic polynomial fitted in
   the least-squares sense to the values of u_h at the vertices of its
   two-ring (the vertex, its neighbours and theirs); its Hessian is the
   vertex Hessian, and H_K is the mean of the vertex Hessians of K.
2. The metric tensor of eq. MK-1,
       M_K = det(I + |H_K| / alpha_h)^{-1/(d+4)} (I + |H_K| / alpha_h),
   |H| = sqrt(H^2), with alpha_h the root of
       sum_K |K| det(I + |H_K| / alpha_h)^{2/(d+4)} = 2 |Omega|
   (the paper prints |H_K(H_K(u))| inside this sum; the reading is |H_K(u)|).
   When every H_K vanishes the sum equals |Omega| for every alpha and there
   is no root: then M_K = I.
3. The mesh energy of eq. I-h for the metric held fixed on every element,
       I_h = 1/3 sum_K sqrt(det M_K) |K| tr(J_K M_K^{-1} J_K^T)^{3d/4}
           + d^{3d/4}/3 sum_K sqrt(det M_K) |K| (sqrt(det M_K) det F'_K)^{-3d/4},
   J_K = (F'_K)^{-1}, F_K the affine map from the equilateral reference
   simplex of unit volume onto K.
4. The moving mesh equations (eqs. x-1, mmpde-1):
       dx_i/dt = -sqrt(det M(x_i)) / tau  dI_h/dx_i,
   with M(x_i) the mean of the metrics of the elements around vertex i, the
   normal component removed on the boundary (vertices slide along it), over
   t in (0, 1], tau = 1e-2, connectivity fixed.  Reading of the integrator
   (the paper uses MATLAB's ode15s): explicit steps of the gradient flow whose
   length is halved until no element inverts and the energy decreases, and
   grown by 1.5 after an accepted step.

The derivative dI_h/dx_i is the plain chain rule through eq. I-h (the paper
points to Huang & Kamenski for the same quantity): with E = [x_1 - x_0, ..,
x_d - x_0], V = det E, B = E_ref^T E_ref (the reference simplex's edges),
A = M^{-1}, t = tr(E^{-1} A E^{-T} B):
    dV/dE = V E^{-T},    dt/dE = -2 E^{-T} B E^{-1} A E^{-T},
and column j of dG_K/dE is the derivative with respect to vertex j of K
(j = 1..d), vertex 0 taking minus their sum.

Test infrastructure: plain numpy, one element or vertex at a time where a
loop is clearer.
"""

from __future__ import annotations

import math

import numpy as np


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


def energy_gradient(X: np.ndarray, elems: np.ndarray, M: np.ndarray) -> np.ndarray:
    """dI_h/dx_i (nv x 2) by the chain rule through eq. I-h (see the module docstring)."""
    d = 2
    p = 3.0 * d / 4.0
    Er = reference_edges(d)
    Dr = np.linalg.det(Er)
    B = Er.T @ Er
    X = np.asarray(X)
    G = np.zeros_like(X)
    for k, t_ in enumerate(np.asarray(elems)):
        P = X[t_]
        E = np.stack([P[1] - P[0], P[2] - P[0]], axis=1)
        V = np.linalg.det(E)
        Ei = np.linalg.inv(E)
        A = np.linalg.inv(M[k])
        q = math.sqrt(np.linalg.det(M[k]))
        t = np.trace(Ei @ A @ Ei.T @ B)
        dV = V * Ei.T
        dt = -2.0 * Ei.T @ B @ Ei @ A @ Ei.T
        fac = q / math.factorial(d)
        g1 = fac / 3.0 * (t ** p * dV + V * p * t ** (p - 1.0) * dt)
        g2 = d ** p / 3.0 * fac * (q / Dr) ** (-p) * (1.0 - p) * V ** (-p) * dV
        gE = g1 + g2
        G[t_[1]] += gE[:, 0]
        G[t_[2]] += gE[:, 1]
        G[t_[0]] -= gE[:, 0] + gE[:, 1]
    return G


# ---------------------------------------------------------------- moving the mesh


def vertex_metric_sqrtdet(elems: np.ndarray, M: np.ndarray, nv: int) -> np.ndarray:
    """sqrt(det M(x_i)) with M(x_i) the mean of the metrics of the elements around vertex i."""
    S = np.zeros((nv, 2, 2))
    c = np.zeros(nv)
    for k, t_ in enumerate(np.asarray(elems)):
        for a in t_:
            S[a] += M[k]
            c[a] += 1
    return np.sqrt(np.linalg.det(S / c[:, None, None]))


def velocity(X, elems, M, bnd, tau=1e-2, qv=None):
    """Right side of eq. x-1; boundary vertices (on the unit circle) keep their tangential component."""
    X = np.asarray(X)
    if qv is None:
        qv = vertex_metric_sqrtdet(elems, M, X.shape[0])
    v = -(qv / tau)[:, None] * energy_gradient(X, elems, M)
    n = X[bnd] / np.linalg.norm(X[bnd], axis=1)[:, None]
    v[bnd] -= np.sum(v[bnd] * n, axis=1)[:, None] * n
    return v


def euler_step(X, v, dt, bnd):
    """x + dt v, boundary vertices put back on the unit circle."""
    Y = np.asarray(X) + dt * v
    Y[bnd] /= np.linalg.norm(Y[bnd], axis=1)[:, None]
    return Y


def move_mesh(X, elems, M, bnd, tau=1e-2, t_end=1.0, dt0=1e-3, max_steps=400):
    """Integrate eq. x-1 over (0, t_end] with the step control described in the module docstring.
    Returns (new X, number of accepted steps)."""
    X = np.array(X, dtype=np.float64)
    qv = vertex_metric_sqrtdet(elems, M, X.shape[0])
    t, dt, steps = 0.0, dt0, 0
    I0 = energy(X, elems, M)
    while t < t_end and steps < max_steps:
        h = min(dt, t_end - t)
        v = velocity(X, elems, M, bnd, tau, qv)
        while True:
            Y = euler_step(X, v, h, bnd)
            if np.all(element_areas(Y, elems) > 0):
                I1 = energy(Y, elems, M)
                if I1 < I0:
                    break
            h *= 0.5
            if h < 1e-14:
                return X, steps
        X, I0, t, steps = Y, I1, t + h, steps + 1
        dt = 1.5 * h
    return X, steps


# ---------------------------------------------------------------- Algorithm amGoFD


def adapt(X, elems, solve_on, levels=5, tau=1e-2, max_steps=400):
    """Algorithm amGoFD: for each level, u = solve_on(X) on the current mesh, then a new mesh from the
    MMPDE method driven by u (the metric of eq. MK-1 from the recovered Hessian).  Returns the list of
    (X, u) of every level; the connectivity never changes."""
    X = np.array(X, dtype=np.float64)
    elems = np.asarray(elems)
    bnd = boundary_mask(elems, X.shape[0])
    rings = vertex_rings(elems, X.shape[0], 2)
    out = []
    for _ in range(levels):
        u = solve_on(X)
        out.append((X.copy(), u))
        A = abs_sym(element_hessians(elems, vertex_hessians(X, elems, u, rings)))
        M = metric(A, alpha_h(A, element_areas(X, elems)))
        X, _ = move_mesh(X, elems, M, bnd, tau=tau, max_steps=max_steps)
    return out
