"""Assignment with centred B-splines of order p = 1..6 (degree p - 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.4.1 compares the BL3 assignment with a fifth-order B-spline, and the
aliasing study of Sec. 2.4.3 with nearest-grid-point assignment (order 1).
The order-p B-spline beta_{p-1} is the p-fold convolution of the unit box;
its Fourier transform is sinc^p(w/2) and, by Poisson summation, its alias sum
sum_J sinc^{2p}((w + 2 pi J) / 2) is sum_m beta_{2p-1}(m) e^{i w m}, the
degree-(2p - 1) B-spline sampled at the integers.

beta_n is evaluated from its explicit form
    beta_n(x) = (1/n!) sum_{k=0}^{n+1} (-1)^k C(n+1, k) (x + (n+1)/2 - k)_+^n
with (t)_+^0 = 1 for t > 0 and 0 otherwise, so the box beta_0 is 1 on
(-1/2, 1/2]; for n >= 1 it is evaluated at -|x| (beta_n is even), where
fewer and smaller terms cancel, and set to 0 outside |x| < (n + 1) / 2.
Node g collects beta_{p-1}(g - u) with u = x N / L in FP64.  Nodes are
enumerated from floor(u) for even p and floor(u + 1/2) (the
nearest node, the sum u + 1/2 rounded in FP64) for odd p, where the box's
half-open ends decide which node a particle at a half-integer u joins.
"""
from __future__ import annotations

import math

import numpy as np

from . import estimator as E

ORDERS = range(1, 7)


def beta(n: int, x):
    """Centred B-spline of degree n at x (float64 array)."""
    x = np.asarray(x, dtype=np.float64)
    inside = None
    if n >= 1:
        inside = np.abs(x) < 0.5 * (n + 1)
        x = -np.abs(x)
    out = np.zeros_like(x)
    for k in range(n + 2):
        t = x + 0.5 * (n + 1) - k
        if n == 0:
            tp = (t > 0).astype(np.float64)
        else:
            tp = np.where(t > 0, t, 0.0) ** n
        out += (-1) ** k * math.comb(n + 1, k) * tp
    out = out / math.factorial(n)
    return out if inside is None else np.where(inside, out, 0.0)


def taps(order: int):
    """Tap offsets j (nodes c + j) and the origin shift s (c = floor(u + s))."""
    lo = -((order - 1) // 2)
    return np.arange(lo, lo + order), (0.5 if order % 2 else 0.0)


def assign(pos, charges, box: float, n_grid: int, order: int):
    """Periodic grids (n_charge, N, N, N) of q * prod_a beta_{p-1}(g_a - u_a)."""
    if order not in ORDERS:
        raise ValueError("B-spline order must be 1..6")
    charges = np.atleast_2d(np.asarray(charges, dtype=np.float64))
    n = n_grid
    u = np.asarray(pos, dtype=np.float64) * (n / box)
    offs, shift = taps(order)
    c = np.floor(u + shift)
    grids = np.zeros((charges.shape[0], n * n * n))
    node = [[None] * len(offs) for _ in range(3)]
    wts = [[None] * len(offs) for _ in range(3)]
    for a in range(3):
        for i, j in enumerate(offs):
            g = c[:, a] + j
            wts[a][i] = beta(order - 1, g - u[:, a])
            node[a][i] = (g - n * np.floor(g / n)).astype(np.int64)
    for ix in range(len(offs)):
        for iy in range(len(offs)):
            wxy = wts[0][ix] * wts[1][iy]
            for iz in range(len(offs)):
                flat = (node[0][ix] * n + node[1][iy]) * n + node[2][iz]
                wxyz = wxy * wts[2][iz]
                for q in range(charges.shape[0]):
                    grids[q] += np.bincount(flat, weights=charges[q] * wxyz, minlength=n ** 3)
    return grids.reshape(charges.shape[0], n, n, n)


def window(order: int, omega):
    """sinc^p(w / 2): the Fourier transform of beta_{p-1}."""
    h = 0.5 * np.asarray(omega, dtype=np.float64)
    s = np.where(h == 0, 1.0, np.sin(h) / np.where(h == 0, 1.0, h))
    return s ** order


def alias_sum(order: int, omega):
    """sum_J window(w + 2 pi J)^2 = sum_m beta_{2p-1}(m) cos(m w)."""
    omega = np.asarray(omega, dtype=np.float64)
    out = np.zeros_like(omega)
    for m in range(-order, order + 1):
        out += float(beta(2 * order - 1, np.array(float(m)))) * np.cos(m * omega)
    return out


def axis_tables(n_grid: int, order: int):
    nf = np.rint(np.fft.fftfreq(n_grid) * n_grid)
    omega = 2.0 * math.pi * nf / n_grid
    return window(order, omega) ** 2, alias_sum(order, omega)


# kernel names used by the estimator
NAMES = {"ngp": 1, "cic": 2, "tsc": 3, "pcs": 4, "pqs": 5, "bspline6": 6}
for _p in ORDERS:
    NAMES.setdefault(f"bspline{_p}", _p)


def order_of(kernel: str):
    return NAMES.get(kernel)


def estimate(pos, vel, weight=None, *, order, **kw):
    """The estimator with B-spline assignment (same keywords as
    oracle.estimate)."""
    name = [k for k, v in NAMES.items() if v == order][0]
    return E.estimate(pos, vel, weight, kernel=name, **kw)
