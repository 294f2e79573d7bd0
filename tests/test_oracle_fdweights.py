"""Pins for the oracle's Toeplitz coefficients T (Section 2.3)."""

import math

import numpy as np
import pytest

from oracle import fdweights as fw


def test_closed_form_1d_hand_values():
    # s = 1/2: Gamma(3/2) = sqrt(pi)/2, Gamma(5/2) = 3 sqrt(pi)/4, Gamma(-1/2) = -2 sqrt(pi)
    T = fw.closed_form_1d(0.5, 3)
    assert T[0] == pytest.approx(4 / math.pi, rel=1e-15)
    assert T[1] == pytest.approx(-4 / (3 * math.pi), rel=1e-15)
    assert T[2] == pytest.approx(-4 / (15 * math.pi), rel=1e-14)


@pytest.mark.parametrize("s", [0.1, 0.3, 0.6, 0.9])
def test_closed_form_1d_gamma_recurrence(s):
    # Gamma(z+1) = z Gamma(z) turns eq. T-1D-0 into T_{p+1} = T_p (p - s) / (p + s + 1)
    T = fw.closed_form_1d(s, 40)
    p = np.arange(40)
    assert np.allclose(T[1:], T[:-1] * (p - s) / (p + s + 1), rtol=1e-13, atol=0)


@pytest.mark.parametrize("s", [0.1, 0.25, 0.5, 0.75, 0.9])
def test_bessel_route_matches_closed_form_1d(s):
    T = fw.closed_form_1d(s, 8)
    B = np.array([fw.bessel_route(s, [p]) for p in range(9)])
    assert np.max(np.abs(T - B)) < 1e-12


@pytest.mark.parametrize("s", [0.25, 0.5, 0.75])
def test_filon_richardson_1d_converges_to_closed_form(s):
    T = fw.closed_form_1d(s, 6)
    errs = []
    for M in (1024, 2048, 4096):
        errs.append(np.max(np.abs(fw.filon_richardson(s, 1, 6, M) - T)))
    # remaining error ~ M^{-(1+2s)} from the |cos|^{2s} cusp of psi~ at xi = 1/2
    assert errs[-1] < 10 * 4096.0 ** (-(1 + 2 * s))
    if s != 0.5:   # s = 1/2 makes psi~ a trigonometric polynomial: error is round-off only
        assert errs[0] / errs[-1] > 0.5 * 4.0 ** (1 + 2 * s)


@pytest.mark.parametrize("s", [0.25, 0.5, 0.75])
def test_filon_richardson_2d_matches_bessel(s):
    F = fw.filon_richardson(s, 2, 3, 2048)
    B = np.array([[fw.bessel_route(s, [i, j]) for i in range(4)] for j in range(4)])
    assert np.max(np.abs(F - B)) < 5e-9


def test_filon_richardson_3d_matches_bessel():
    F = fw.filon_richardson(0.5, 3, 2, 256)
    for p in [(0, 0, 0), (1, 0, 0), (1, 1, 0), (2, 1, 1)]:
        assert abs(F[p] - fw.bessel_route(0.5, p)) < 1e-6


def test_trapezoid_at_s_one_is_five_point_laplacian():
    # psi~ = 4cos^2(pi xi) + 4cos^2(pi eta) = 4 + 2cos(2 pi xi) + 2cos(2 pi eta)
    T = fw.trapezoid(1.0, 2, 3, 64)
    E = np.zeros((4, 4))
    E[0, 0] = 4.0
    E[0, 1] = E[1, 0] = -1.0
    assert np.max(np.abs(T - E)) < 1e-14


def test_filon_is_trapezoid_times_sinc_squared():
    # summation by parts turns eq. Tp-1D-2 into trapezoid * (sin(pi p/M)/(pi p/M))^2 per axis
    M, P = 256, 7
    for s in (0.3, 0.8):
        F = fw.filon(s, 2, P, M)
        Tz = fw.trapezoid(s, 2, P, M)
        p = np.arange(P + 1)
        x = np.pi * p / M
        sig = np.where(p == 0, 1.0, (np.sin(x) / np.where(p == 0, 1, x)) ** 2)
        assert np.allclose(F, Tz * sig[:, None] * sig[None, :], rtol=1e-11, atol=1e-15)


def test_symmetry_sign_and_dominance():
    T = fw.filon_richardson(0.6, 2, 10, 1024)
    assert np.allclose(T, T.T, atol=1e-15)
    off = T.copy()
    off[0, 0] = 0
    assert T[0, 0] > 0 and np.all(off[np.nonzero(off)] < 0)
    # T_0 = -sum_{p != 0} T_p over the whole lattice, so any finite window is dominated
    full = 4 * np.abs(off[1:, 1:]).sum() + 2 * np.abs(off[0, 1:]).sum() + 2 * np.abs(off[1:, 0]).sum()
    assert T[0, 0] > full


def test_small_s_tends_to_identity():
    T = fw.filon_richardson(1e-4, 2, 3, 512)
    E = np.zeros((4, 4))
    E[0, 0] = 1.0
    assert np.max(np.abs(T - E)) < 1e-3
