"""Overlay uniform grid descriptions (inputs only).

A grid is the cube (c - R, c + R)^d covered by 2N+1 nodes per axis with
spacing h = R/N (Section 3.1 of the paper; the node set of Section 2.1 is
-N..N, re-indexed here as i = 0..2N).  Node i along axis a sits at

    x_i = (c_a - R) + i * h,     h = R / N,

with every operation rounded separately in IEEE double (no fused
multiply-add).  This rounding sequence is part of the interface: the oracle
and the HIP library both place nodes by exactly this recipe, which is what
makes point location comparable bit for bit.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Grid:
    d: int
    N: int
    R: float
    center: tuple

    @property
    def W(self) -> int:
        """Nodes per axis, 2N + 1."""
        return 2 * self.N + 1

    @property
    def h(self) -> float:
        return float(np.float64(self.R) / np.float64(self.N))

    @property
    def n_nodes(self) -> int:
        return self.W ** self.d


def grid_for_box(d: int, n: int, R: float = 1.0, center=None) -> Grid:
    """A grid named "n x n" (or n^3): n intervals per axis, so N = n/2."""
    if n % 2:
        raise ValueError("n must be even (n = 2N intervals per axis)")
    if center is None:
        center = (0.0,) * d
    return Grid(d=d, N=n // 2, R=float(R), center=tuple(float(c) for c in center))


def grid_node_coords_1d(grid: Grid, axis: int) -> np.ndarray:
    """Node coordinates along one axis (used to sample right-hand sides)."""
    lo = np.float64(grid.center[axis]) - np.float64(grid.R)
    h = np.float64(grid.R) / np.float64(grid.N)
    i = np.arange(grid.W, dtype=np.float64)
    return lo + i * h
