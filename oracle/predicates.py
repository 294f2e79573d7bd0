"""Exact orientation signs for point location (used by Section 3.1's location step).

orient(q_0, ..., q_d) = det[q_1 - q_0, ..., q_d - q_0] for points in R^d.
The sign is computed exactly: a double-precision evaluation whose magnitude
exceeds a generous rounding bound decides directly; every other case is
recomputed in exact rational arithmetic (``fractions.Fraction`` holds each
double exactly).  The floating-point path is only a shortcut; the answer is
always the sign of the exact determinant.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np

_FILTER = 1e-13   # relative bound, far above the true rounding error of these formulas


def _det_exact(rows):
    """Exact determinant of a small matrix of Fractions (cofactor expansion)."""
    n = len(rows)
    if n == 1:
        return rows[0][0]
    if n == 2:
        return rows[0][0] * rows[1][1] - rows[0][1] * rows[1][0]
    total = Fraction(0)
    for c in range(n):
        minor = [r[:c] + r[c + 1:] for r in rows[1:]]
        term = rows[0][c] * _det_exact(minor)
        total += term if c % 2 == 0 else -term
    return total


def orient_exact(points) -> int:
    """Exact sign of orient(q_0..q_d) for one tuple of points (each a sequence of floats)."""
    q = [[Fraction(float(x)) for x in pt] for pt in points]
    rows = [[q[i][a] - q[0][a] for a in range(len(q[0]))] for i in range(1, len(q))]
    det = _det_exact(rows)
    return (det > 0) - (det < 0)


def orient_signs(P: np.ndarray) -> np.ndarray:
    """Signs of orient for a batch: P has shape (n, d+1, d); returns int8 (n,)."""
    P = np.asarray(P, dtype=np.float64)
    n, dp1, d = P.shape
    E = P[:, 1:, :] - P[:, :1, :]                      # (n, d, d)
    if d == 2:
        t1 = E[:, 0, 0] * E[:, 1, 1]
        t2 = E[:, 0, 1] * E[:, 1, 0]
        det = t1 - t2
        perm = np.abs(t1) + np.abs(t2)
    elif d == 3:
        m0 = E[:, 1, 1] * E[:, 2, 2] - E[:, 1, 2] * E[:, 2, 1]
        m1 = E[:, 1, 0] * E[:, 2, 2] - E[:, 1, 2] * E[:, 2, 0]
        m2 = E[:, 1, 0] * E[:, 2, 1] - E[:, 1, 1] * E[:, 2, 0]
        det = E[:, 0, 0] * m0 - E[:, 0, 1] * m1 + E[:, 0, 2] * m2
        pm0 = np.abs(E[:, 1, 1] * E[:, 2, 2]) + np.abs(E[:, 1, 2] * E[:, 2, 1])
        pm1 = np.abs(E[:, 1, 0] * E[:, 2, 2]) + np.abs(E[:, 1, 2] * E[:, 2, 0])
        pm2 = np.abs(E[:, 1, 0] * E[:, 2, 1]) + np.abs(E[:, 1, 1] * E[:, 2, 0])
        perm = np.abs(E[:, 0, 0]) * pm0 + np.abs(E[:, 0, 1]) * pm1 + np.abs(E[:, 0, 2]) * pm2
    elif d == 1:
        det = E[:, 0, 0]
        perm = np.abs(det)
    else:
        raise ValueError("d must be 1, 2 or 3")
    sign = np.sign(det).astype(np.int8)
    # the coordinate differences themselves are rounded, so scale the bound by
    # the magnitude of the raw coordinates as well
    scale = np.max(np.abs(P), axis=(1, 2))
    bound = _FILTER * (perm + scale ** d)
    unsure = ~(np.abs(det) > bound)
    for r in np.nonzero(unsure)[0]:
        sign[r] = orient_exact(P[r])
    return sign
