"""Pins of the one-loop SPT oracle (the one-loop section and its appendices):
limits of the P13 kernels, the damping of modes far above the spectrum,
the low-k limits, and every two-dimensional formula against the
three-dimensional definition with the textbook F2 and G2 kernels."""
import math

import numpy as np
import pytest

from oracle import spt

KT = np.geomspace(1e-3, 4.0, 24)
TAB = spt.Table(KT, 2e3 * KT ** -1.5 * np.exp(-KT / 0.5))


def test_p13_kernel_limits():
    # r -> 0: 12/r^2 cancels the logarithm's -12/r^2 (24/r^2 for d-theta)
    for kind, want in (("dd", -168.0), ("dt", -168.0), ("tt", -56.0)):
        assert abs(spt.kernel13(kind, 1e-4) - want) < 1e-5, kind
    # r -> infinity: the r^4 and r^2 terms cancel, leaving -488/5 and -504/5
    assert abs(spt.kernel13("dd", 1e4) - (-488.0 / 5.0)) < 1e-5
    assert abs(spt.kernel13("tt", 1e4) - (-504.0 / 5.0)) < 1e-5
    # continuous through r = 1, where the logarithm diverges
    for kind in ("dd", "dt", "tt"):
        a, b, c = (spt.kernel13(kind, r) for r in (1 - 1e-7, 1.0, 1 + 1e-7))
        assert abs(a - b) < 1e-4 and abs(c - b) < 1e-4, kind


def _bump_table(lo, hi, n, q_peak, floor=1e-250):
    """A spectrum concentrated near q_peak, with a negligible floor so that
    the log-log table stays positive over [lo, hi]."""
    q = np.geomspace(lo, hi, n)
    p = 1e4 * np.exp(-0.5 * (np.log(q / q_peak) / 0.3) ** 2)
    return spt.Table(q, np.maximum(p, floor))


def _sigma_v2(tab):
    """sigma_v^2 = (1 / 6 pi^2) int P0(q) dq (trapezoid in ln q on a fine
    grid; the integrand is log-log linear between nodes)."""
    q = np.geomspace(tab.k[0], tab.k[-1], 200001)
    f = tab(q) * q
    return float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(np.log(q)))) / (6 * math.pi ** 2)


@pytest.mark.parametrize("kind", ["dd", "dt", "tt"])
def test_p13_damps_modes_far_above_the_spectrum(kind):
    """For k far above the support of P0: P_xy,13 -> -k^2 sigma_v^2 P0(k)/2
    (the one-loop term of the propagator exp(-k^2 sigma_v^2 / 2))."""
    tab = _bump_table(1e-4, 4.0, 60, 3e-3)
    k = 2.0
    ratio = spt.p13(k, tab, kind) / tab.scalar(k)
    want = -0.5 * k * k * _sigma_v2(tab)
    assert abs(ratio / want - 1) < 1e-4, (ratio, want)


def test_p13_low_k_limit():
    """For k far below the support: 2 P13 -> -(61/105) k^2 sigma_v^2 P0(k)."""
    tab = _bump_table(1e-6, 50.0, 80, 1.0)
    k = 1e-4
    ratio = 2 * spt.p13(k, tab, "dd") / tab.scalar(k)
    want = -61.0 / 105.0 * k * k * _sigma_v2(tab)
    assert abs(ratio / want - 1) < 1e-4, (ratio, want)


def test_p22_is_k4_at_low_k():
    """Mass and momentum conservation: P22 ~ k^4 as k -> 0."""
    tab = _bump_table(1e-6, 50.0, 80, 1.0)
    a, b = (spt.at(k, tab) for k in (1e-4, 2e-4))
    for key in ("p22", "p22_dt", "p22_tt"):
        assert abs(b[key] / a[key] / 16.0 - 1) < 1e-3, key


# ---------------------------------------------------------------- the 3D definitions
def _f2(a, b, s):
    """Symmetrised second-order kernels from explicit vectors:
    F2 (s = 'F') = 5/7 + mu/2 (a/b + b/a) + 2/7 mu^2,
    G2 (s = 'G') = 3/7 + mu/2 (a/b + b/a) + 4/7 mu^2."""
    ab = np.sum(a * b, axis=0)
    a2, b2 = np.sum(a * a, axis=0), np.sum(b * b, axis=0)
    c0, c2 = (5.0 / 7.0, 2.0 / 7.0) if s == "F" else (3.0 / 7.0, 4.0 / 7.0)
    return c0 + 0.5 * ab * (1.0 / a2 + 1.0 / b2) + c2 * ab * ab / (a2 * b2)


_X16, _W16 = np.polynomial.legendre.leggauss(16)


def _panels(edges):
    edges = np.unique(edges)
    lo, hi = edges[:-1, None], edges[1:, None]
    return (0.5 * (hi - lo) * _X16 + 0.5 * (hi + lo)).ravel(), (0.5 * (hi - lo) * _W16).ravel()


def _definitions(k, tab):
    """(1/(2 pi)^3) int d^3q of each integrand, over q in spherical
    coordinates about k = k z_hat (the azimuth gives 2 pi)."""
    k0, k1 = tab.k[0], tab.k[-1]
    # breakpoints where P0(q) has a kink and where a kink of P0(|k - q|)
    # enters or leaves the mu range (|k - q| = k_n at mu = +-1)
    qn, qw = _panels(np.concatenate([[1e-12, k + k1], tab.k, np.abs(k - tab.k), k + tab.k, [k]]))
    out = {n: 0.0 for n in ("p22", "p22_dt", "p22_tt", "pcov1", "pcov2", "t1", "t2", "t3")}
    kv = np.array([0.0, 0.0, k])[:, None]
    pk = tab.scalar(k)
    for q, wq in zip(qn, qw):
        mus = (k * k + q * q - tab.k ** 2) / (2 * k * q)
        mu, wm = _panels(np.concatenate([[-1.0, 1.0], mus[(mus > -1) & (mus < 1)]]))
        s = np.sqrt(1 - mu * mu)
        qv = np.stack([q * s, 0 * mu, q * mu])
        pv = kv - qv                                  # k - q
        p = np.sqrt(np.sum(pv * pv, axis=0))
        Pq, Pp = tab.scalar(q), tab(p)
        meas = wq * 2 * math.pi * q * q / (2 * math.pi) ** 3 * wm
        F, G = _f2(qv, pv, "F"), _f2(qv, pv, "G")
        base = meas * Pq * Pp
        out["p22"] += np.sum(2 * base * F * F)
        out["p22_dt"] += np.sum(2 * base * F * G)
        out["p22_tt"] += np.sum(2 * base * G * G)
        out["pcov1"] += np.sum(base * k * k / (p * p))            # k^2 P0 (x) (P0 / k^2)
        qp = np.sum(qv * pv, axis=0)
        out["pcov2"] += np.sum(base * k * k * qp / (q * q * p * p))  # k^2 (q P0/q^2).(p P0/p^2)
        wkq = meas * (k * q * mu) / (k * k * q * q)              # (k.q) / (k^2 q^2)
        mk = np.broadcast_to(-kv, qv.shape)
        out["t1"] += np.sum(wkq * 2 * Pp * Pq * _f2(pv, qv, "G"))
        out["t2"] += np.sum(wkq * 2 * Pp * pk * _f2(pv, mk, "G"))
        out["t3"] += np.sum(wkq * 2 * Pq * pk * _f2(qv, mk, "F"))
    return out


@pytest.mark.parametrize("k", [0.03, 0.1])
def test_two_dimensional_formulas_against_the_definitions(k):
    got = spt.at(k, TAB)
    ref = _definitions(k, TAB)
    pairs = {"p22": "p22", "p22_dt": "p22_dt", "p22_tt": "p22_tt", "pcov1": "pcov1",
             "pcov2": "pcov2", "i1": "t1", "i2": "t2", "i3": "t3"}
    for mine, theirs in pairs.items():
        assert abs(got[mine] / ref[theirs] - 1) < 1e-8, (k, mine, got[mine], ref[theirs])
