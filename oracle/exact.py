"""Closed-form solutions on the unit ball and error norms (Section 5).

For Omega = B(0,1) and f as in eq. exam-0,
    u = (1 - |x|^2)_+^s P_k^{(s, d/2-1)}(2|x|^2 - 1)           (eq. exam-2),
    f = 2^{2s} Gamma(1+s+k) Gamma(d/2+s+k) / (k! Gamma(d/2+k)) P_k^{(s,d/2-1)}(2|x|^2-1).
For k = 0 the right-hand side is the constant 2^{2s} Gamma(1+s) Gamma(d/2+s) / Gamma(d/2),
so f = 1 gives u = Gamma(d/2) / (2^{2s} Gamma(1+s) Gamma(d/2+s)) (1-|x|^2)_+^s.

Errors are measured in the L2 norm of the P1 interpolant of the nodal error
(the paper does not name the discrete norm; this reading uses the P1 mass
matrix) and in the maximum norm over vertices.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy import special


def f_ball(x, s, d, k=0):
    r2 = np.sum(np.asarray(x) ** 2, axis=-1)
    c = 2 ** (2 * s) * special.gamma(1 + s + k) * special.gamma(d / 2 + s + k) / (
        math.factorial(k) * special.gamma(d / 2 + k))
    return c * special.eval_jacobi(k, s, d / 2 - 1, 2 * r2 - 1)


def u_ball(x, s, d, k=0):
    r2 = np.sum(np.asarray(x) ** 2, axis=-1)
    return np.maximum(1 - r2, 0.0) ** s * special.eval_jacobi(k, s, d / 2 - 1, 2 * r2 - 1)


def u_ball_unit_rhs(x, s, d):
    """Solution for f = 1 on the unit ball."""
    c = special.gamma(d / 2) / (2 ** (2 * s) * special.gamma(1 + s) * special.gamma(d / 2 + s))
    r2 = np.sum(np.asarray(x) ** 2, axis=-1)
    return c * np.maximum(1 - r2, 0.0) ** s


def mass_matrix(X, elems) -> sp.csr_matrix:
    """P1 mass matrix: on each simplex M_ij = |K| (1 + delta_ij) / ((d+1)(d+2))."""
    X = np.asarray(X)
    elems = np.asarray(elems, dtype=np.int64)
    d = X.shape[1]
    P = X[elems]
    vol = np.abs(np.linalg.det(P[:, 1:] - P[:, :1])) / math.factorial(d)
    loc = (np.ones((d + 1, d + 1)) + np.eye(d + 1)) / ((d + 1) * (d + 2))
    rows = np.repeat(elems, d + 1, axis=1).ravel()
    cols = np.tile(elems, (1, d + 1)).ravel()
    vals = (vol[:, None, None] * loc[None]).reshape(-1)
    n = X.shape[0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def l2_error(X, elems, e) -> float:
    M = mass_matrix(X, elems)
    return float(np.sqrt(e @ (M @ e)))
