"""One-loop standard perturbation theory (SPT) predictions of the momentum
spectra (the one-loop section and its appendices: Eqs. Ppd, PpdD4, pdivpD4,
the P13 / P22 formulas, Eq. intBktree with I1-I3, Eq. Pcov).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every quantity is an integral over the linear spectrum P0 at z = 0:

* P_xy,13(k) = c P0(k) k^3/(4 pi^2) int dr P0(kr) K_xy(r), with
  c = 1/504, 1/504, 1/168 for dd, d-theta, theta-theta;
* P_xy,22(k) = 1/98 k^3/(4 pi^2) int dr P0(kr) int_{-1}^{1} dx
  P0(k sqrt(1 + r^2 - 2rx)) N_x N_y / (1 + r^2 - 2rx)^2 with
  N_d = 3r + 7x - 10 r x^2, N_t = 7x - r - 6 r x^2;
* I1, I2, I3 (their sum is the bispectrum integral B_dtt,0) and the
  convolution terms P_cov^I, P_cov^II, as printed.

Combinations (D = D_z, Haf as in the estimator):
  P^(1)          = D^2 P0 + D^4 (2 P13 + P22)
  P_theta_p^(1)  = D^2 P0 + D^4 (6 P13 + 4 P22)              (Eq. pdivpD4)
  P_dtheta_p^(1) = D^2 P0 + D^4 (4 P13 + 2 P22)
  (k/Haf)^2 P_p^(1) = D^2 P0 + D^4 (P_tt,1 + P_cov^I + P_cov^II + 2 k^2 B_dtt,0),
  P_tt,1 = 2 P_tt,13 + P_tt,22                               (Eq. PpdD4)

Readings:
* the logarithm of each P13 kernel is multiplied by 3/r^3; the printed
  3/r^2 makes every kernel diverge like 1/r as r -> 0, whereas with 3/r^3 the
  kernels tend to -168, -168 and -56, which gives the known damping
  P_xy,13 -> -k^2 sigma_v^2 P0(k) / 2 of modes far above the spectrum's
  support;
* P0 is a table (k_i, P_i), k_i > 0 ascending and P_i > 0, interpolated
  linearly in (ln k, ln P) and zero outside [k_0, k_last].

The integrals are taken in the printed variables r and x: adaptive
quadrature (scipy.integrate.quad, quad_vec) over r with breakpoints where the
integrand is not smooth (r = 1, the table nodes, the ends of the inner
range), and over x 20-point Gauss-Legendre on every panel between the points
where k sqrt(1 + r^2 - 2rx) meets a table node.  The P13 kernels are
evaluated with mpmath at 40 significant digits.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np
from scipy import integrate


class Table:
    """Log-log linear P0(q), zero outside the table."""

    def __init__(self, k, p):
        self.k = np.asarray(k, dtype=np.float64)
        self.p = np.asarray(p, dtype=np.float64)
        if np.any(np.diff(self.k) <= 0) or np.any(self.k <= 0) or np.any(self.p <= 0):
            raise ValueError("table needs ascending positive k and positive P")
        self.lk = np.log(self.k)
        self.lp = np.log(self.p)

    def __call__(self, q):
        q = np.asarray(q, dtype=np.float64)
        out = np.zeros_like(q)
        inside = (q >= self.k[0]) & (q <= self.k[-1])
        if np.any(inside):
            out[inside] = np.exp(np.interp(np.log(q[inside]), self.lk, self.lp))
        return out

    def scalar(self, q):
        return float(self(np.array(q)))


_KERNEL13 = {  # (c, a0 / r^2, a1, a2 r^2, a3 r^4, (A r^2 + B) in the log term)
    "dd": (1.0 / 504.0, 12, -158, 100, -42, (7, 2)),
    "dt": (1.0 / 504.0, 24, -202, 56, -30, (5, 4)),
    "tt": (1.0 / 168.0, 12, -82, 4, -6, (1, 2)),
}

mpmath.mp.dps = 40


def kernel13(kind, r):
    """K_xy(r) of P_xy,13 (40-digit evaluation, returned as float)."""
    _, a0, a1, a2, a3, (A, B) = _KERNEL13[kind]
    r = mpmath.mpf(r)
    if r == 1:
        log_term = mpmath.mpf(0)
    else:
        log_term = 3 / r ** 3 * (r * r - 1) ** 3 * (A * r * r + B) * mpmath.log(abs((1 + r) / (1 - r)))
    return float(a0 / r ** 2 + a1 + a2 * r ** 2 + a3 * r ** 4 + log_term)


def _quad(f, a, b, points=()):
    pts = sorted(p for p in set(points) if a < p < b)
    edges = [a] + pts + [b]
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(f, lo, hi, epsabs=0.0, epsrel=1e-11, limit=200)
        tot += v
    return tot


def _r_range(k, tab):
    return tab.k[0] / k, tab.k[-1] / k


def p13(k, tab, kind="dd"):
    c = _KERNEL13[kind][0]
    lo, hi = _r_range(k, tab)
    nodes = list(tab.k / k) + [1.0]
    val = _quad(lambda r: tab.scalar(k * r) * kernel13(kind, r), lo, hi, nodes)
    return c * tab.scalar(k) * k ** 3 / (4 * math.pi ** 2) * val


# The two-dimensional integrands g(r, x, y), y = 1 + r^2 - 2 r x, each
# multiplied by P0(k sqrt(y)) and, except I2, by P0(k r).
_G2D = {
    "p22": lambda r, x, y: (3 * r + 7 * x - 10 * r * x * x) ** 2 / (y * y),
    "p22_dt": lambda r, x, y: (3 * r + 7 * x - 10 * r * x * x) * (7 * x - r - 6 * r * x * x) / (y * y),
    "p22_tt": lambda r, x, y: (7 * x - r - 6 * r * x * x) ** 2 / (y * y),
    "i1": lambda r, x, y: x * (r - 7 * x + 6 * r * x * x) / y,
    "pcov1": lambda r, x, y: 1.0,
    "pcov2": lambda r, x, y: r * (x - r) / y,
    "i2": lambda r, x, y: r ** 3 * x * (7 * r * x - 1 - 6 * x * x) / y,
}
_NAMES2D = tuple(_G2D)


_GL_X, _GL_W = np.polynomial.legendre.leggauss(20)


def _inner_x(k, r, tab):
    """int_{-1}^{1} dx P0(k sqrt(y)) g(r, x, y) for the seven g: 20-point
    Gauss-Legendre on every panel between the x where k sqrt(y) meets a
    table node (the integrand is smooth inside each panel)."""
    xs = (1.0 + r * r - (tab.k / k) ** 2) / (2.0 * r)
    edges = np.unique(np.concatenate([[-1.0, 1.0], xs[(xs > -1.0) & (xs < 1.0)]]))
    lo, hi = edges[:-1, None], edges[1:, None]
    x = 0.5 * (hi - lo) * _GL_X[None, :] + 0.5 * (hi + lo)
    w = 0.5 * (hi - lo) * _GL_W[None, :]
    y = 1.0 + r * r - 2.0 * r * x
    pk = tab(k * np.sqrt(np.maximum(y, 0.0))) * w
    ys = np.where(y > 0, y, 1.0)
    return np.array([np.sum(pk * _G2D[n](r, x, ys)) for n in _NAMES2D])


def _two_d(k, tab):
    """The seven double integrals int dr [P0(kr)] int_{-1}^{1} dx
    P0(k sqrt(y)) g(r, x, y): adaptive quadrature over r with breakpoints,
    Gauss-Legendre panels over x."""
    k1 = tab.k[-1] / k
    i2 = _NAMES2D.index("i2")

    def outer(r):
        if r <= 0.0:
            return np.zeros(len(_NAMES2D))
        v = _inner_x(k, r, tab)
        w = np.full(len(_NAMES2D), tab.scalar(k * r))
        w[i2] = 1.0
        return w * v

    hi = 1.0 + k1
    # kinks of P0(kr) at the nodes, and where a kink of P0(k sqrt(y)) enters
    # or leaves the x range: sqrt(y) = node / k at x = +-1, r = |1 -+ node / k|
    kn = tab.k / k
    nodes = [x for x in np.concatenate([kn, np.abs(1.0 - kn), 1.0 + kn, [1.0]]) if 0.0 < x < hi]
    v, _ = integrate.quad_vec(outer, 0.0, hi, epsabs=0.0, epsrel=1e-12, points=sorted(set(nodes)), limit=2000)
    return dict(zip(_NAMES2D, v))


def p22(k, tab, kind="dd"):
    name = {"dd": "p22", "dt": "p22_dt", "tt": "p22_tt"}[kind]
    return k ** 3 / (98.0 * 4 * math.pi ** 2) * _two_d(k, tab)[name]


def i3(k, tab):
    lo, hi = _r_range(k, tab)
    val = _quad(lambda r: (r * r + 1.0) * tab.scalar(k * r), lo, hi, list(tab.k / k) + [1.0])
    return -2.0 / 3.0 * k / (4 * math.pi ** 2) * tab.scalar(k) * val


def at(k, tab):
    """All eleven integrals at one k."""
    d = _two_d(k, tab)
    c3 = k ** 3 / (4 * math.pi ** 2)
    return {
        "p13": p13(k, tab, "dd"), "p22": c3 / 98.0 * d["p22"],
        "p13_dt": p13(k, tab, "dt"), "p22_dt": c3 / 98.0 * d["p22_dt"],
        "p13_tt": p13(k, tab, "tt"), "p22_tt": c3 / 98.0 * d["p22_tt"],
        "i1": -k / (7.0 * 4 * math.pi ** 2) * d["i1"],
        "i2": k / (7.0 * 4 * math.pi ** 2) * tab.scalar(k) * d["i2"],
        "i3": i3(k, tab),
        "pcov1": c3 * d["pcov1"], "pcov2": c3 * d["pcov2"],
    }


QUANTITIES = ("p13", "p22", "p13_dt", "p22_dt", "p13_tt", "p22_tt", "i1", "i2", "i3", "pcov1", "pcov2")


def one_loop(k_values, tab, d_z=1.0, haf=50.0):
    """All integrals and the combined one-loop spectra at each k."""
    rows = [at(k, tab) for k in k_values]
    out = {q: np.array([r[q] for r in rows]) for q in QUANTITIES}
    k = np.asarray(k_values, dtype=np.float64)
    p0 = tab(k)
    d2, d4 = d_z ** 2, d_z ** 4
    out["p_lin"] = d2 * p0
    out["p_dd"] = d2 * p0 + d4 * (2 * out["p13"] + out["p22"])
    out["p_theta_p"] = d2 * p0 + d4 * (6 * out["p13"] + 4 * out["p22"])
    out["p_dtheta_p"] = d2 * p0 + d4 * (4 * out["p13"] + 2 * out["p22"])
    b0 = out["i1"] + out["i2"] + out["i3"]
    ptt1 = 2 * out["p13_tt"] + out["p22_tt"]
    out["p_mom"] = (haf / k) ** 2 * (d2 * p0 + d4 * (ptt1 + out["pcov1"] + out["pcov2"] + 2 * k * k * b0))
    return out
