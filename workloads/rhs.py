"""Seeded right-hand sides sampled on the overlay grid (inputs only)."""

from __future__ import annotations

import numpy as np

from .grids import Grid, grid_node_coords_1d


def fourier_coeffs(seed: int, d: int, modes: int = 4) -> np.ndarray:
    """N(0,1) coefficients c_{a,b(,c)} for a, b, c in 0..modes-1."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=(modes,) * d)


def eval_fourier(coeffs: np.ndarray, pts: np.ndarray, box_lo, box_len) -> np.ndarray:
    """f(x) = sum_a c_a prod_i cos(pi a_i (x_i - lo_i) / len_i) at the given points."""
    d = pts.shape[1]
    modes = coeffs.shape[0]
    basis = []
    for i in range(d):
        t = (pts[:, i] - box_lo[i]) / box_len[i]
        basis.append(np.cos(np.pi * np.arange(modes)[None, :] * t[:, None]))
    if d == 1:
        return basis[0] @ coeffs
    if d == 2:
        return np.einsum("na,nb,ab->n", basis[0], basis[1], coeffs)
    return np.einsum("na,nb,nc,abc->n", basis[0], basis[1], basis[2], coeffs)


def _grid_points(grid: Grid) -> np.ndarray:
    axes = [grid_node_coords_1d(grid, a) for a in range(grid.d)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")  # C order: last axis fastest = axis 0
    return np.stack([m.ravel() for m in mesh[::-1]], axis=1)


def fourier_rhs(seed: int, grid: Grid, box_lo=None, box_len=None, modes: int = 4) -> np.ndarray:
    """Smooth random f sampled at every grid node, C order (last index fastest).

    Grid arrays are indexed [i_{d-1}, ..., i_0] in C order with i_0 (the x
    index) fastest, i.e. a 2D field f[j, i] holds f at (x_i, y_j).
    """
    if box_lo is None:
        box_lo = [c - grid.R for c in grid.center]
    if box_len is None:
        box_len = [2 * grid.R] * grid.d
    c = fourier_coeffs(seed, grid.d, modes)
    pts = _grid_points(grid)
    return np.ascontiguousarray(eval_fourier(c, pts, box_lo, box_len).reshape((grid.W,) * grid.d))


def constant_rhs(grid: Grid, value: float = 1.0) -> np.ndarray:
    return np.full((grid.W,) * grid.d, value, dtype=np.float64)
