"""The GoFD operator and the linear system that is solved (Section 3).

* A_h = D_h^{-1} (I_h^FD)^T A_FD I_h^FD                         (eq. Ah-1)
* A~_h = (I D^{-1/2})^T A_FD (I D^{-1/2}), similar to A_h         (eqs. Ah-2, Ah-3)
* GoFD-2 on the interior block J:
      K u_J = b,  K = I_J^T A_FD I_J,  b = h^{2s} I_J^T f_FD       (eq. GoFD-2, remark after it)
  where f_FD holds f at the grid nodes (zero outside the domain, eq. GoFD-1)
* GoFD-3 (f at the mesh vertices): D^{-1} I^T A_FD I u = h^{2s} f_h on J
  (eq. GoFD-3), i.e. K u_J = h^{2s} D_J f_h,J.

A_FD products go through ``afd.apply_direct`` (the definition) on small grids
and ``afd.apply_fft`` (eq. AU-1) otherwise.
"""

from __future__ import annotations

import numpy as np

from . import afd


def afd_apply(T, v, mode="auto"):
    if mode == "direct" or (mode == "auto" and v.size <= 70 ** 2 and v.ndim <= 2):
        return afd.apply_direct(T, v)
    return afd.apply_fft(T, v)


def grid_shape(tr):
    return (tr.W,) * tr.d


def apply_Ah(tr, T, u, mode="auto") -> np.ndarray:
    """A_h u = D^{-1} I^T A_FD I u for a full vertex vector u (eq. Ah-1)."""
    v = (tr.I @ u).reshape(grid_shape(tr))
    y = afd_apply(T, v, mode).ravel()
    return (tr.I.T @ y) / tr.D


def apply_Ah_sym(tr, T, u, mode="auto") -> np.ndarray:
    """A~_h u = D^{-1/2} I^T A_FD I D^{-1/2} u (eq. Ah-3)."""
    r = 1.0 / np.sqrt(tr.D)
    v = (tr.I @ (r * u)).reshape(grid_shape(tr))
    y = afd_apply(T, v, mode).ravel()
    return r * (tr.I.T @ y)


def apply_K(tr, T, uJ, mode="auto") -> np.ndarray:
    """K u_J = I_J^T A_FD I_J u_J (left side of eq. GoFD-2 on the interior block)."""
    v = (tr.IJ @ uJ).reshape(grid_shape(tr))
    y = afd_apply(T, v, mode).ravel()
    return tr.IJ.T @ y


def dense_K(tr, T) -> np.ndarray:
    """K as a dense matrix (tiny cases): I_J^T A_FD I_J."""
    A = afd.dense(T, tr.d, tr.W)
    IJ = tr.IJ.toarray()
    return IJ.T @ A @ IJ


def dense_Ah(tr, T) -> np.ndarray:
    """A_h (all vertices) as a dense matrix (tiny cases)."""
    A = afd.dense(T, tr.d, tr.W)
    I = tr.I.toarray()
    return (I.T @ A @ I) / tr.D[:, None]


def rhs_grid(tr, s, f_grid) -> np.ndarray:
    """b = h^{2s} I_J^T f_FD (right side of eq. GoFD-2)."""
    return tr.h ** (2 * s) * (tr.IJ.T @ np.asarray(f_grid, dtype=np.float64).ravel())


def rhs_vertex(tr, s, f_vert) -> np.ndarray:
    """b = h^{2s} D_J f_h,J: eq. GoFD-3 multiplied through by D."""
    return tr.h ** (2 * s) * tr.D[tr.J] * np.asarray(f_vert, dtype=np.float64)[tr.J]
