"""The uniform-grid FD matrix A_FD and its products (Sections 2.1-2.2).

A_FD is the (2N+1)^d section of the infinite multilevel Toeplitz matrix with
entries A_{(j),(m)} = T_{j-m} (eqs. A-1, AFD-1); T is even in every index
(eq. T-2), so A_{(j),(m)} = T[|j_0 - m_0|, ..., |j_{d-1} - m_{d-1}|] with the
octant table of ``fdweights``.

* ``apply_direct``  -- the definition, y_j = sum_m T_{j-m} v_m (O(W^{2d}));
* ``apply_rows``    -- the same sums for selected output nodes only;
* ``dense``         -- the explicit matrix for small grids;
* ``apply_fft``     -- the paper's circulant-embedding evaluation (eq. AU-1):
  the DFT of T on the 4N-periodic grid in the paper's centred index range
  -2N..2N-1, the DFT of the zero-extended u, the product with the phase
  (-1)^{p+2N} per axis and an inverse DFT (scipy's FFT on the host cores as the
  DFT primitive).
"""

from __future__ import annotations

import os

import numpy as np
import scipy.fft

# host threads for the DFTs: the process's CPU share (OMP_NUM_THREADS when the
# environment sets it, else the cores this process may run on)
WORKERS = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))


def _check(T: np.ndarray, v: np.ndarray):
    d = v.ndim
    W = v.shape[0]
    if T.ndim != d or any(n < W for n in T.shape) or any(n != W for n in v.shape):
        raise ValueError("T octant must cover offsets 0..W-1 in every axis")
    return d, W


def dense(T: np.ndarray, d: int, W: int) -> np.ndarray:
    """Explicit A_FD (W^d x W^d) in the natural node order (x index fastest)."""
    idx = np.indices((W,) * d).reshape(d, -1)        # idx[0] = slowest array axis
    diff = [np.abs(idx[a][:, None] - idx[a][None, :]) for a in range(d)]
    return T[tuple(diff)]


def apply_direct(T: np.ndarray, v: np.ndarray) -> np.ndarray:
    """y = A_FD v by the direct Toeplitz sums (definition, eq. A-1 and AFD-1)."""
    d, W = _check(T, v)
    if d == 1:
        return dense(T, 1, W) @ v
    idx = np.arange(W)
    absd = np.abs(idx[:, None] - idx[None, :])        # |j - m| along one axis
    if d == 2:
        y = np.zeros_like(v)
        for j in range(W):                             # output row j (slow axis)
            # y[j, i] = sum_n sum_m T[|j-n|, |i-m|] v[n, m]
            for n in range(W):
                y[j] += T[absd[j, n]][absd] @ v[n]
        return y
    if d == 3:
        y = np.zeros_like(v)
        for k in range(W):
            for j in range(W):
                acc = np.zeros(W)
                for c in range(W):
                    for n in range(W):
                        acc += T[absd[k, c], absd[j, n]][absd] @ v[c, n]
                y[k, j] = acc
        return y
    raise ValueError("d must be 1, 2 or 3")


def apply_rows(T: np.ndarray, v: np.ndarray, nodes) -> np.ndarray:
    """(A_FD v)_k for the listed output nodes only (multi-indices in array order)."""
    d, W = _check(T, v)
    idx = np.indices((W,) * d)
    out = np.empty(len(nodes))
    for r, k in enumerate(nodes):
        off = tuple(np.abs(idx[a] - k[a]) for a in range(d))
        out[r] = np.sum(T[off] * v)
    return out


def apply_fft(T: np.ndarray, v: np.ndarray) -> np.ndarray:
    """y = A_FD v through three DFTs of length 4N per axis (eq. AU-1).

    Index k = p + 2N in 0..4N-1 stands for the paper's p = -2N..2N-1.
      T_full[k]  = T_{k-2N}                       (p = -2N..2N-1)
      T_hat      = DFT(T_full)                    (exponent (m+2N)(p+2N))
      u_ext[m+N] = u_m for m = -N..N, else 0      (m = -N..3N-1)
      u_hat      = DFT(u_ext)                     (exponent (p+2N)(m+N))
      y_{j}      = IDFT(T_hat * u_hat * (-1)^{p+2N})[j+N],  j = -N..N
    """
    d, W = _check(T, v)
    N = (W - 1) // 2
    L = 4 * N
    p = np.arange(L) - 2 * N                         # paper's p
    Tfull = T[tuple(np.meshgrid(*([np.abs(p)] * d), indexing="ij"))]
    That = scipy.fft.fftn(Tfull, workers=WORKERS)
    uext = np.zeros((L,) * d)
    uext[(slice(0, W),) * d] = v                     # position m + N for m = -N..N
    uhat = scipy.fft.fftn(uext, workers=WORKERS)
    k = np.arange(L)
    phase1 = np.where(k % 2 == 0, 1.0, -1.0)          # (-1)^{p+2N} = (-1)^k
    phase = np.ones((L,) * d)
    for a in range(d):
        shape = [1] * d
        shape[a] = L
        phase = phase * phase1.reshape(shape)
    y = scipy.fft.ifftn(That * uhat * phase, workers=WORKERS)
    return y[(slice(0, W),) * d].real.copy()          # positions j + N for j = -N..N
