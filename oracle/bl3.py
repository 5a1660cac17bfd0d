"""Plain FP64 construction of the cubic Battle-Lemarie (BL3) scaling function.

TEST INFRASTRUCTURE ONLY.  This module belongs to the CPU oracle: only the
test suite, the smoke check and the benchmark's CPU-baseline leg may use it.
The GPU library builds its own tables independently.

The paper assigns objects to the FFT grid with the third-order orthogonalised
Battle-Lemarie scaling function (Sec. 2.4.1, "Algorithm setup").  The paper
does not print its formula; we read "third order" as the cubic-spline member
of the family (integer knots, symmetric about 0), defined in Fourier space by

    phi_hat(w) = (sin(w/2)/(w/2))^4 / sqrt(A(w)),
    A(w) = sum_k |beta3_hat(w + 2 pi k)|^2
         = (2416 + 2382 cos w + 240 cos 2w + 2 cos 3w) / 5040,

where A is the integer-sampled degree-7 B-spline (the autocorrelation of the
cubic B-spline).  In real space phi(x) = sum_n c_n beta3(x - n) with c_n the
Fourier coefficients of A(w)^(-1/2).

Here c_n is obtained by adaptive quadrature of its defining integral and phi
is evaluated directly from the B-spline sum.  The assignment uses phi
truncated to the six taps d in (-3, 3]; the window of that truncated kernel
and its alias sum (Eq. rawPp's sum_J W^2(k + 2 k_N J)) are computed here from
their definitions by Gauss-Legendre quadrature.
"""
from __future__ import annotations

import functools
import math
import warnings

import numpy as np
from scipy import integrate

# c_n decays like 0.5085^|n|; |c_45| < 1e-13 relative to c_0.
N_FILTER = 45
TRUNC = 3            # support kept by the assignment: d in (-3, 3]
TAPS = np.arange(-2, 4)   # taps j = -2..3 relative to floor(u)


def autocorr_bspline7(w):
    """A(w): sum over aliases of |beta3_hat|^2, a trigonometric polynomial."""
    w = np.asarray(w, dtype=np.float64)
    return (2416.0 + 2382.0 * np.cos(w) + 240.0 * np.cos(2 * w)
            + 2.0 * np.cos(3 * w)) / 5040.0


def phi_hat(w):
    """Closed-form Fourier transform of the untruncated BL3 function."""
    w = np.asarray(w, dtype=np.float64)
    half = 0.5 * w
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(half == 0.0, 1.0, np.sin(half) / np.where(half == 0, 1, half))
    return s ** 4 / np.sqrt(autocorr_bspline7(w))


@functools.lru_cache(maxsize=None)
def filter_coefficients(n_max: int = N_FILTER) -> tuple:
    """c_n = (1/pi) int_0^pi A(w)^(-1/2) cos(n w) dw for n = 0..n_max."""
    out = []
    for n in range(n_max + 1):
        # tiny high-order coefficients trip quad's roundoff detector; the
        # absolute error requested (1e-16) is still met.
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", integrate.IntegrationWarning)
            val, _ = integrate.quad(
                lambda w: autocorr_bspline7(w) ** -0.5 * math.cos(n * w),
                0.0, math.pi, epsabs=1e-16, epsrel=1e-15, limit=400)
        out.append(val / math.pi)
    return tuple(out)


def bspline3(y):
    """Centred cubic B-spline beta3(y), support [-2, 2]."""
    a = np.abs(np.asarray(y, dtype=np.float64))
    inner = 2.0 / 3.0 - a * a + 0.5 * a ** 3
    outer = (2.0 - a) ** 3 / 6.0
    return np.where(a < 1.0, inner, np.where(a < 2.0, outer, 0.0))


def phi(x):
    """Untruncated BL3 scaling function phi(x) = sum_n c_n beta3(x - n).

    beta3(x - n) vanishes unless n is within 2 of x, so only the four shifts
    n = floor(x) - 1 .. floor(x) + 2 are summed; c_n is zero beyond N_FILTER.
    """
    x = np.asarray(x, dtype=np.float64)
    c = np.asarray(filter_coefficients())
    m = np.floor(x).astype(np.int64)
    acc = np.zeros_like(x)
    for shift in (-1, 0, 1, 2):
        n = m + shift
        an = np.abs(n)
        cn = np.where(an <= N_FILTER, c[np.minimum(an, N_FILTER)], 0.0)
        acc = acc + cn * bspline3(x - n)
    return acc


def phi_trunc(x):
    """phi restricted to the assignment support (-3, 3]."""
    x = np.asarray(x, dtype=np.float64)
    return np.where((x > -TRUNC) & (x <= TRUNC), phi(x), 0.0)


def tap_weights(f):
    """Weights phi(j - f) for the six taps j = -2..3 of a particle at fraction f.

    f has any shape with values in [0, 1); the result has shape (6,) + f.shape.
    """
    f = np.asarray(f, dtype=np.float64)
    return np.stack([phi(j - f) for j in TAPS])


_GL_X, _GL_W = np.polynomial.legendre.leggauss(24)


def _integrate_unit_pieces(func, lo: int, hi: int):
    """Integrate func over [lo, hi] as a sum of Gauss-Legendre unit pieces.

    phi is a cubic on every unit interval, so each piece is smooth.
    """
    total = 0.0
    for m in range(lo, hi):
        t = m + 0.5 * (_GL_X + 1.0)
        total = total + 0.5 * np.sum(_GL_W * func(t), axis=-1)
    return total


def window_trunc(w):
    """W_t(w) = int_{-3}^{3} phi(x) cos(w x) dx: window of the truncated kernel.

    w is in radians per grid cell (w = 2 pi n / N_g).  phi is even so the
    transform is real.
    """
    w = np.atleast_1d(np.asarray(w, dtype=np.float64))
    return _integrate_unit_pieces(
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
        out.append(float(_integrate_unit_pieces(
            lambda x: phi(x) * phi(x + m), lo, hi)))
    return tuple(out)


def alias_sum_trunc(w):
    """C_t(w) = sum_J W_t(w + 2 pi J)^2 = sum_m a_m cos(m w) (Poisson summation).

    This is the per-axis factor multiplying the shot noise in Eq. rawPp when
    the truncated kernel is used.
    """
    w = np.asarray(w, dtype=np.float64)
    a = trunc_autocorrelation()
    out = np.full(w.shape, a[0])
    for m in range(1, len(a)):
        out = out + 2.0 * a[m] * np.cos(m * w)
    return out
