"""Pins for the oracle's A_FD products (Sections 2.1-2.2)."""

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

from oracle import afd, fdweights as fw


@pytest.mark.parametrize("d,W,M", [(1, 41, 512), (2, 17, 256), (3, 7, 64)])
def test_fft_embedding_equals_direct_sums(d, W, M):
    rng = np.random.default_rng(d)
    T = fw.filon_richardson(0.37, d, W - 1, M)
    v = rng.standard_normal((W,) * d)
    y1 = afd.apply_direct(T, v)
    y2 = afd.apply_fft(T, v)
    assert np.max(np.abs(y1 - y2)) <= 1e-13 * np.max(np.abs(y1))
    A = afd.dense(T, d, W)
    assert np.allclose(A @ v.ravel(), y1.ravel(), rtol=0, atol=1e-13)


def test_1d_matrix_is_scipy_toeplitz():
    T = fw.closed_form_1d(0.3, 20)
    assert np.array_equal(afd.dense(T, 1, 21), scipy.linalg.toeplitz(T))


def test_s_one_gives_five_point_laplacian():
    W = 9
    T = fw.trapezoid(1.0, 2, W - 1, 64)
    A = afd.dense(T, 2, W)
    lap1 = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(W, W))
    L5 = (sp.kron(sp.eye(W), lap1) + sp.kron(lap1, sp.eye(W))).toarray()
    assert np.max(np.abs(A - L5)) < 1e-14


@pytest.mark.parametrize("s", [0.2, 0.5, 0.9])
def test_afd_spd_and_spectrum_bounds(s):
    W, d = 15, 2
    T = fw.filon_richardson(s, d, W - 1, 256)
    A = afd.dense(T, d, W)
    assert np.array_equal(A, A.T)
    np.linalg.cholesky(A)
    ev = np.linalg.eigvalsh(A)
    # the symbol psi lies in [0, (4d)^s]; sections of a Toeplitz operator stay inside
    assert ev[0] > 0 and ev[-1] < (4 * d) ** s


def test_rows_match_full_product():
    rng = np.random.default_rng(3)
    W = 21
    T = fw.filon_richardson(0.7, 2, W - 1, 256)
    v = rng.standard_normal((W, W))
    y = afd.apply_direct(T, v)
    nodes = [(0, 0), (20, 20), (5, 13), (10, 0)]
    assert np.allclose(afd.apply_rows(T, v, nodes), [y[k] for k in nodes], rtol=0, atol=1e-13)
