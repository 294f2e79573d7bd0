"""Overlay grid T_FD (Section 2.1; Section 3.1).

The cube (c - R, c + R)^d carries 2N+1 nodes per axis, spacing h = R/N.  The
paper indexes nodes -N..N; here they are re-indexed i = 0..2N so node i sits
at (c - R) + i h, each operation rounded separately in double precision.

Grid fields are stored as numpy arrays of shape (W,)*d in C order with the x
index fastest: a 2D field F[j, i] is the value at (x_i, y_j).  The linear
node number is i_0 + W i_1 (+ W^2 i_2), the paper's natural ordering.
"""

from __future__ import annotations

import numpy as np


def spacing(R: float, N: int) -> float:
    """h_FD = R / N (Section 3.1)."""
    return float(np.float64(R) / np.float64(N))


def axis_coords(center: float, R: float, N: int) -> np.ndarray:
    """Node coordinates (c - R) + i h, i = 0..2N, rounded step by step."""
    lo = np.float64(center) - np.float64(R)
    h = np.float64(R) / np.float64(N)
    i = np.arange(2 * N + 1, dtype=np.float64)
    t = i * h          # one rounding
    return lo + t      # one rounding


def node_coords(d: int, N: int, R: float, center) -> np.ndarray:
    """All node coordinates, shape (W^d, d), in linear node order."""
    W = 2 * N + 1
    axes = [axis_coords(center[a], R, N) for a in range(d)]
    idx = np.indices((W,) * d).reshape(d, -1)  # idx[0] slowest
    cols = []
    for a in range(d):
        cols.append(axes[a][idx[d - 1 - a]])
    return np.stack(cols, axis=1)


def node_index(multi, W: int) -> np.ndarray:
    """Linear node number from per-axis indices (i_0 fastest)."""
    multi = np.asarray(multi)
    k = np.zeros(multi.shape[:-1], dtype=np.int64)
    for a in reversed(range(multi.shape[-1])):
        k = k * W + multi[..., a]
    return k
