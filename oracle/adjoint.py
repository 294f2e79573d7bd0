"""Gradients of a loss of the GoFD-2 solution, by the adjoint method (dense, tiny cases).

System (eq. GoFD-2, interior block J):  K u = b,  K = I_J^T A I_J,
b = h^{2s} I_J^T f_FD.  For a loss L(u) with g = dL/du:

    lambda = K^{-1} g                                  (K is symmetric)
    dL/df_FD = h^{2s} I_J lambda
    dL/dI_kj = lambda_j r_k - (A I_J lambda)_k u_j,   r = h^{2s} f_FD - A I_J u   (j in J)

The transfer entries are barycentric weights, I_kj = phi_j(x_k), with
[phi] = E^{-1} [x; 1] (proof of the simplex interpolation lemma).  Moving
vertex i of the element that holds x_k changes E by one entry, so
d phi_r / d X_{i,a} = -(E^{-1})_{r,a} phi_i.  Point location is held fixed
(the loss is piecewise smooth in X; the map node -> element is locally
constant almost everywhere), and so is the grid.

The paper has no gradients; this is the plain chain rule through its
operators.  Pins: central finite differences of the loss (tests).
"""

from __future__ import annotations

import numpy as np

from . import afd, operator, solve


def forward_dense(tr, T, s, f_grid):
    """u_J = K^{-1} b by dense LU."""
    K = operator.dense_K(tr, T)
    b = operator.rhs_grid(tr, s, f_grid)
    return solve.solve_dense(K, b), K


def gradients(tr, T, s, f_grid, uJ, g):
    """(dL/df_FD as a grid array, dL/dX of shape (nv, d)) for dL/du_J = g."""
    K = operator.dense_K(tr, T)
    lam = solve.solve_dense(K, g)
    shape = (tr.W,) * tr.d
    h2s = tr.h ** (2 * s)
    grad_f = (h2s * (tr.IJ @ lam)).reshape(shape)
    A = afd.dense(T, tr.d, tr.W)
    Iu = tr.IJ @ uJ
    Il = tr.IJ @ lam
    r = h2s * np.asarray(f_grid, dtype=np.float64).ravel() - A @ Iu
    AIl = A @ Il
    # full-length vertex vectors (zero on Dirichlet vertices)
    u_full = np.zeros(tr.nv)
    u_full[tr.J] = uJ
    l_full = np.zeros(tr.nv)
    l_full[tr.J] = lam
    d = tr.d
    grad_X = np.zeros((tr.nv, d))
    for row, k in enumerate(tr.inside):
        e = tr.elem[k]
        vs = tr.elems[e]
        P = tr.X[vs]                                     # (d+1, d)
        E = np.ones((d + 1, d + 1))
        E[:d, :] = P.T
        Einv = np.linalg.inv(E)
        phi = tr.lam[row]                                # (d+1,)
        # dL/dI_{k, v_r} for the element's vertices (zero for Dirichlet vertices)
        G = l_full[vs] * r[k] - AIl[k] * u_full[vs]
        G = np.where(tr.bnd[vs], 0.0, G)
        for i in range(d + 1):
            for a in range(d):
                dphi = -Einv[:, a] * phi[i]              # d phi_r / d X_{v_i, a}
                grad_X[vs[i], a] += float(G @ dphi)
    return grad_f, grad_X
