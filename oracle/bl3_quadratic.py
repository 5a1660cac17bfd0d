"""Plain FP64 construction of the quadratic-spline Battle-Lemarie function.

TEST INFRASTRUCTURE ONLY.  This module belongs to the CPU oracle: only the
test suite, the smoke check and the benchmark's CPU-baseline leg may use it.

The paper assigns objects with the "third-order" orthogonalised
Battle-Lemarie scaling function (Sec. 2.4.1, "Algorithm setup") without
printing it.  oracle.bl3 reads the order as the spline degree (cubic); this
module is the other reading, where order counts the polynomial's
coefficients (de Boor's convention), i.e. the degree-2 member of the family:

    phi_hat(w) = (sin(w/2)/(w/2))^3 / sqrt(A2(w)),
    A2(w) = sum_k |beta2_hat(w + 2 pi k)|^2 = sum_m beta5(m) cos(m w),

A2 being the integer samples of the degree-5 B-spline (the autocorrelation of
the quadratic B-spline), here taken from oracle.bspline's own evaluation of
beta5.  In real space phi(x) = sum_n c_n beta2(x - n), with c_n the Fourier
coefficients of A2^(-1/2) obtained by adaptive quadrature and beta2 the
centred quadratic B-spline (support [-3/2, 3/2], knots at half-integers).
phi is a quadratic on every interval between consecutive half-integers.

The assignment keeps the same support as the cubic reading, d in (-3, 3]
(six taps j = -2..3 relative to floor(u), weights phi(j - f)); the window of
the truncated function and its alias sum are computed from their
definitions by Gauss-Legendre quadrature on the half-unit pieces.
"""
from __future__ import annotations

import functools
import math
import warnings

import numpy as np
from scipy import integrate

from . import bspline

# c_n of A2^(-1/2) decays like 0.4306^|n|; |c_38| < 1e-14 relative to c_0.
N_FILTER = 38
TRUNC = 3
TAPS = np.arange(-2, 4)


@functools.lru_cache(maxsize=None)
def _beta5_at_integers() -> tuple:
    """beta5(m) for m = 0..2 (zero beyond |m| >= 3)."""
    return tuple(float(bspline.beta(5, np.array(float(m)))) for m in range(3))


def autocorr(w):
    """A2(w) = beta5(0) + 2 sum_{m >= 1} beta5(m) cos(m w)."""
    w = np.asarray(w, dtype=np.float64)
    b = _beta5_at_integers()
    return b[0] + 2.0 * b[1] * np.cos(w) + 2.0 * b[2] * np.cos(2 * w)


def phi_hat(w):
    """Closed-form Fourier transform of the untruncated function."""
    w = np.asarray(w, dtype=np.float64)
    half = 0.5 * w
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(half == 0.0, 1.0, np.sin(half) / np.where(half == 0, 1, half))
    return s ** 3 / np.sqrt(autocorr(w))


@functools.lru_cache(maxsize=None)
def filter_coefficients(n_max: int = N_FILTER) -> tuple:
    """c_n = (1/pi) int_0^pi A2(w)^(-1/2) cos(n w) dw for n = 0..n_max."""
    out = []
    for n in range(n_max + 1):
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", integrate.IntegrationWarning)
            val, _ = integrate.quad(
                lambda w: float(autocorr(w)) ** -0.5 * math.cos(n * w),
                0.0, math.pi, epsabs=1e-16, epsrel=1e-15, limit=400)
        out.append(val / math.pi)
    return tuple(out)


def bspline2(y):
    """Centred quadratic B-spline beta2(y)."""
    a = np.abs(np.asarray(y, dtype=np.float64))
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def phi(x):
    """phi(x) = sum_n c_n beta2(x - n): beta2(x - n) vanishes unless
    |x - n| < 3/2, so the shifts n = round(x) - 1 .. round(x) + 1 are summed
    (plus one more on either side, harmless where beta2 is zero)."""
    x = np.asarray(x, dtype=np.float64)
    c = np.asarray(filter_coefficients())
    m = np.floor(x).astype(np.int64)
    acc = np.zeros_like(x)
    for shift in (-1, 0, 1, 2):
        n = m + shift
        an = np.abs(n)
        cn = np.where(an <= N_FILTER, c[np.minimum(an, N_FILTER)], 0.0)
        acc = acc + cn * bspline2(x - n)
    return acc


def phi_trunc(x):
    """phi restricted to the assignment support (-3, 3]."""
    x = np.asarray(x, dtype=np.float64)
    return np.where((x > -TRUNC) & (x <= TRUNC), phi(x), 0.0)


def tap_weights(f):
    """Weights phi(j - f) of the six taps j = -2..3; shape (6,) + f.shape."""
    f = np.asarray(f, dtype=np.float64)
    return np.stack([phi(j - f) for j in TAPS])


_GL_X, _GL_W = np.polynomial.legendre.leggauss(24)


def _integrate_half_pieces(func, lo: float, hi: float):
    """Integrate over [lo, hi] (half-integers) as Gauss-Legendre pieces of
    width 1/2, on each of which phi is one quadratic."""
    total = 0.0
    for i in range(int(round(2 * (hi - lo)))):
        a = lo + 0.5 * i
        t = a + 0.25 * (_GL_X + 1.0)
        total = total + 0.25 * np.sum(_GL_W * func(t), axis=-1)
    return total


def window_trunc(w):
    """W_t(w) = int_{-3}^{3} phi(x) cos(w x) dx (phi even: real)."""
    w = np.atleast_1d(np.asarray(w, dtype=np.float64))
    return _integrate_half_pieces(
        lambda x: phi(x)[None, :] * np.cos(w[:, None] * x[None, :]), -TRUNC, TRUNC)


@functools.lru_cache(maxsize=None)
def trunc_autocorrelation() -> tuple:
    """a_m = int phi_t(x) phi_t(x + m) dx for m = 0..2*TRUNC."""
    out = []
    for m in range(2 * TRUNC + 1):
        lo, hi = -TRUNC, TRUNC - m
        if hi <= lo:
            out.append(0.0)
            continue
        out.append(float(_integrate_half_pieces(lambda x: phi(x) * phi(x + m), lo, hi)))
    return tuple(out)


def alias_sum_trunc(w):
    """C_t(w) = sum_J W_t(w + 2 pi J)^2 = sum_m a_m cos(m w) (Poisson)."""
    w = np.asarray(w, dtype=np.float64)
    a = trunc_autocorrelation()
    out = np.full(w.shape, a[0])
    for m in range(1, len(a)):
        out = out + 2.0 * a[m] * np.cos(m * w)
    return out
