"""Toeplitz coefficients T of the uniform-grid fractional FD operator (Section 2).

T_p is the p-th Fourier coefficient of the symbol
psi(xi) = (sum_a 4 sin^2(xi_a / 2))^s  (eqs. FL-6, T-1), even in every index
(eq. T-2), so only the octant p in {0..P}^d is stored.  Tables are indexed
T[p_{d-1}, ..., p_0]; psi is symmetric under axis permutations, so the order
of the axes does not change any value.

Three routes:

* ``closed_form_1d``        -- the 1D analytic formula (eq. T-1D-0);
* ``trapezoid``             -- the composite trapezoid rule (eq. T-3);
* ``filon`` / ``filon_richardson`` -- Filon's method with piecewise-linear
  interpolation of psi~ (eq. Tp-1D-2, derived in the paper in 1D and applied
  here axis by axis), combined with two-level Richardson extrapolation
  (Section 2.3, M = 2^14 in 2D and 2^11 in 3D at the finest level).

``bessel_route`` is *not* from the paper: it evaluates T_p from the
subordination identity lambda^s = s/Gamma(1-s) int_0^inf (1-e^{-t lambda})
t^{-1-s} dt together with the modified-Bessel generating function
(1/2pi) int e^{2t cos x} e^{ipx} dx = I_p(2t).  It is an independent truth
used only to pin the paper's quadrature routes.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def psi_tilde(xis, s: float) -> np.ndarray:
    """psi~(xi) = (sum_a 4 cos^2(pi xi_a))^s  (eq. psi-2), on a tensor grid.

    ``xis`` is a list of 1D sample arrays, one per axis (axis 0 first); the
    result has shape (len(xis[d-1]), ..., len(xis[0])).
    """
    d = len(xis)
    acc = 0.0
    for a in range(d):
        c = 4.0 * np.cos(np.pi * np.asarray(xis[a], dtype=np.float64)) ** 2
        shape = [1] * d
        shape[d - 1 - a] = c.size
        acc = acc + c.reshape(shape)
    return np.asarray(acc, dtype=np.float64) ** s


def closed_form_1d(s: float, P: int) -> np.ndarray:
    """T_p = (-1)^p Gamma(2s+1) / (Gamma(p+s+1) Gamma(s-p+1)), p = 0..P (eq. T-1D-0).

    Evaluated in logarithms (ln|Gamma| and the sign of Gamma) so that the large
    factors of the two gammas never overflow separately.
    """
    p = np.arange(P + 1, dtype=np.float64)
    sign = np.where(p % 2 == 0, 1.0, -1.0) * special.gammasgn(s - p + 1)
    logmag = special.gammaln(2 * s + 1) - special.gammaln(p + s + 1) - special.gammaln(s - p + 1)
    return sign * np.exp(logmag)


def _signs(P: int, d: int) -> np.ndarray:
    """(-1)^{p_0 + ... + p_{d-1}} on the octant."""
    p = np.arange(P + 1)
    sgn = np.where(p % 2 == 0, 1.0, -1.0)
    out = np.ones((P + 1,) * d)
    for a in range(d):
        shape = [1] * d
        shape[a] = P + 1
        out = out * sgn.reshape(shape)
    return out


def trapezoid(s: float, d: int, P: int, M: int) -> np.ndarray:
    """Composite trapezoid rule for eq. T-0 (eq. T-3), outputs p in {0..P}^d.

    T_p ~ (-1)^{|p|} M^{-d} sum_j psi~(j/M) exp(i 2 pi p.j / M); the sum is an
    inverse DFT of the samples (numpy's ifftn carries the 1/M^d factor).
    Requires M >= 2P + 1.
    """
    if M < 2 * P + 1:
        raise ValueError("trapezoid rule needs M >= 2P+1")
    xi = np.arange(M, dtype=np.float64) / M
    samples = psi_tilde([xi] * d, s)
    S = np.fft.ifftn(samples)                 # = M^{-d} sum_j psi~ e^{+i 2pi p.j/M}
    sl = (slice(0, P + 1),) * d
    return _signs(P, d) * S[sl].real


def _second_difference(F: np.ndarray, axis: int) -> np.ndarray:
    """Periodic second difference psi~_{j+1} - 2 psi~_j + psi~_{j-1} along one axis."""
    return np.roll(F, -1, axis=axis) - 2.0 * F + np.roll(F, 1, axis=axis)


def filon(s: float, d: int, P: int, M: int) -> np.ndarray:
    """Filon's method with piecewise-linear psi~ (eq. Tp-1D-2), outputs p in {0..P}^d.

    In 1D the paper integrates by parts, replaces psi~' by the slope of the
    linear interpolant on each cell and sums exactly:

        T_p ~ (-1)^{p+1} M / (2 pi p)^2  sum_j (psi~_{j+1} - 2 psi~_j + psi~_{j-1}) e^{i 2 pi p j / M},

    for p >= 1.  At p = 0 the integral of the linear interpolant is the
    trapezoid rule, (1/M) sum_j psi~_j.  In d dimensions the same 1D rule is
    applied along every axis (tensor-product Filon): along an axis with
    p_a != 0 the samples are second-differenced and weighted by
    (-1)^{p_a+1} M / (2 pi p_a)^2, along an axis with p_a = 0 they are weighted
    by 1/M.  One inverse DFT is taken per subset of differenced axes.
    """
    if M < 2 * P + 1:
        raise ValueError("Filon's rule needs M >= 2P+1")
    xi = np.arange(M, dtype=np.float64) / M
    samples = psi_tilde([xi] * d, s)
    p = np.arange(P + 1, dtype=np.float64)
    with np.errstate(divide="ignore"):
        filon_w = np.where(p % 2 == 0, -1.0, 1.0) * M / (2 * np.pi * p) ** 2   # (-1)^{p+1} M/(2 pi p)^2
    out = np.zeros((P + 1,) * d)
    for mask in range(1 << d):
        # axes (coordinate index a) that carry p_a != 0 for this block
        F = samples
        for a in range(d):
            if mask >> a & 1:
                F = _second_difference(F, axis=d - 1 - a)
        G = np.fft.ifftn(F).real * float(M) ** d  # = sum_j F_j e^{+i 2 pi p.j/M}
        G = G[(slice(0, P + 1),) * d]
        block = G.copy()
        sel = []
        for a in range(d):
            axis = d - 1 - a
            shape = [1] * d
            shape[axis] = P + 1
            if mask >> a & 1:
                w = np.where(p > 0, filon_w, 0.0)
                keep = p > 0
            else:
                w = np.where(p == 0, 1.0 / M, 0.0)
                keep = p == 0
            block = block * w.reshape(shape)
            sel.append(keep.reshape(shape))
        m = np.ones((P + 1,) * d, dtype=bool)
        for k in sel:
            m = m & k
        out = np.where(m, block, out)
    return out


def filon_richardson(s: float, d: int, P: int, M: int) -> np.ndarray:
    """Filon at levels M and M/2 combined by Richardson extrapolation (Section 2.3).

    The Filon error is O(1/M^2), so T = (4 T^{(M)} - T^{(M/2)}) / 3.  The
    coarse level also needs M/2 >= 2P + 1.
    """
    fine = filon(s, d, P, M)
    coarse = filon(s, d, P, M // 2)
    return (4.0 * fine - coarse) / 3.0


def _ive(q: int, x: float) -> float:
    """e^{-x} I_q(x); scipy for moderate x, the Hankel large-argument series beyond."""
    if x < 5e8:
        return float(special.ive(q, x))
    mu = 4.0 * q * q
    z8 = 8.0 * x
    term, acc = 1.0, 1.0
    for k in range(1, 6):
        term *= -(mu - (2 * k - 1) ** 2) / (k * z8)
        acc += term
    return acc / math.sqrt(2.0 * math.pi * x)


def bessel_route(s: float, p, epsabs: float = 1e-15, epsrel: float = 1e-13) -> float:
    """T_p from the subordination identity (independent of the paper; used as a pin).

    T_p = s/Gamma(1-s) int_0^inf (delta_{p0} - prod_a e^{-2t} I_{p_a}(2t)) t^{-1-s} dt.
    """
    p = [abs(int(q)) for q in p]
    is0 = all(q == 0 for q in p)

    def prod_ive(t):
        v = 1.0
        for q in p:
            v *= _ive(q, 2.0 * t)
        return v

    # [0, 1]: write the integrand as g(t) * t^{-s} with g(t) = (delta - prod)/t smooth
    def g(t):
        if t == 0.0:
            if is0:
                return 2.0 * len(p)           # d/dt (1 - prod ive) at 0
            return -1.0 if sum(p) == 1 else 0.0
        return ((1.0 if is0 else 0.0) - prod_ive(t)) / t

    a, _ = integrate.quad(g, 0.0, 1.0, weight="alg", wvar=(-s, 0.0), epsabs=epsabs, epsrel=epsrel,
                          limit=400)
    # [1, inf): delta part integrates to 1/s exactly.  In tau = ln t the rest is
    # int_0^inf prod ive(p_a, 2 e^tau) e^{-s tau} dtau, smooth with a bump near
    # t ~ |p|^2, so the range is split around it.
    def h(tau):
        return prod_ive(math.exp(tau)) * math.exp(-s * tau)

    tp = 2.0 * math.log(max(p) + 1.0)
    cuts = sorted({0.0, max(0.0, tp - 6), max(0.0, tp - 3), max(0.0, tp - 1), tp, tp + 1, tp + 3, tp + 6,
                   tp + 12, tp + 24})
    b = 0.0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        if hi > lo:
            b += integrate.quad(h, lo, hi, epsabs=epsabs, epsrel=epsrel, limit=400)[0]
    # up to t = e^{tp + 60}, then the large-t form e^{-2t} I_q(2t) ~ (4 pi t)^{-1/2}
    top = tp + 60.0
    b += integrate.quad(h, cuts[-1], top, epsabs=epsabs, epsrel=epsrel, limit=400)[0]
    e = 0.5 * len(p) + s
    b += (4.0 * math.pi) ** (-0.5 * len(p)) * math.exp(-e * top) / e
    tail = (1.0 / s if is0 else 0.0) - b
    return s / math.gamma(1.0 - s) * (a + tail)
