"""Solving GoFD-2 (Section 3.2): dense LU for tiny systems, (preconditioned) CG otherwise.

The paper solves eq. GoFD-2 with the conjugate gradient method, optionally
preconditioned by the incomplete Cholesky factor of A_h^(5/9/27) (Section
3.3).  It does not state x_0 or the stopping test; the reading used here is
x_0 = 0 and ||b - K x_k||_2 <= tol ||b||_2 on the recursively updated
residual (Hestenes-Stiefel CG).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


def solve_dense(K: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x = K^{-1} b by LU with partial pivoting (LAPACK getrf/getrs)."""
    lu, piv = scipy.linalg.lu_factor(K)
    return scipy.linalg.lu_solve((lu, piv), b)


def pcg(apply_K, b, tol=1e-10, maxiter=10000, precond=None, x0=None):
    """Preconditioned conjugate gradients; returns (x, iterations, residual history)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_K(x) if x0 is not None else b.copy()
    z = precond(r) if precond is not None else r.copy()
    p = z.copy()
    rz = float(r @ z)
    nb = float(np.linalg.norm(b))
    hist = [float(np.linalg.norm(r)) / nb if nb > 0 else 0.0]
    if nb == 0.0:
        return x, 0, hist
    for it in range(1, maxiter + 1):
        q = apply_K(p)
        pq = float(p @ q)
        if not pq > 0.0:
            raise FloatingPointError("CG breakdown: p^T K p <= 0")
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        rn = float(np.linalg.norm(r))
        hist.append(rn / nb)
        if rn <= tol * nb:
            return x, it, hist
        z = precond(r) if precond is not None else r.copy()
        rz_new = float(r @ z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    raise RuntimeError(f"CG did not converge in {maxiter} iterations (rel. residual {hist[-1]:.3e})")


def cg_iterates(apply_K, b, iters, x0=None):
    """Exactly `iters` iterations of textbook CG (the steps of ``pcg`` without a
    preconditioner or a stopping test) from x0 (default 0).  Returns the list of
    iterates (x_i, r_i, p_i) for i = 0..iters and the scalars gamma_i = (r_i, r_i),
    delta_i = (p_i, K p_i), alpha_i, beta_i.  Used as the truncated solve whose
    derivative the unrolled gradient computes (parity of the checkpoints and
    finite-difference pins)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_K(x) if x0 is not None else b.copy()
    p = r.copy()
    g = float(r @ r)
    out = [(x.copy(), r.copy(), p.copy())]
    sc = {"gamma": [g], "delta": [], "alpha": [], "beta": []}
    for _ in range(iters):
        q = apply_K(p)
        d = float(p @ q)
        a = g / d
        x = x + a * p
        r = r - a * q
        g1 = float(r @ r)
        beta = g1 / g
        p = r + beta * p
        g = g1
        out.append((x.copy(), r.copy(), p.copy()))
        for k, v in (("gamma", g1), ("delta", d), ("alpha", a), ("beta", beta)):
            sc[k].append(v)
    return out, sc
