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


# ------------------------------------------------------- the combined spectra
def _components(k, tab):
    """<delta_(j) delta_(m)^*> of the SPT expansion that enter at D_z^4:
    (1, 1) = P0, (1, 3) = (3, 1) = P13, (2, 2) = P22 (appendix notation)."""
    a = spt.at(k, tab)
    return {(1, 1): tab.scalar(k), (1, 3): a["p13"], (3, 1): a["p13"], (2, 2): a["p22"]}


def _bilinear(c, d1, d2):
    """Q(D1, D2) = sum_{j, m} D1^j D2^m <delta_(j) delta_(m)^*>: the density
    spectrum with the two fields taken at growth factors D1 and D2."""
    return sum(v * d1 ** j * d2 ** m for (j, m), v in c.items())


@pytest.mark.parametrize("k", [0.03, 0.2])
def test_divergence_spectra_are_growth_derivatives(k):
    """Eq. Ppc: theta_p = (1/f) d delta / d ln a = d delta / d ln D, so
    P_theta_p = d^2 Q / d ln D1 d ln D2 and P_delta_theta_p = d Q / d ln D2
    at D1 = D2 = D_z, and P = Q(D_z, D_z).  Central differences in ln D of
    the bilinear form, against the oracle's combined spectra."""
    c = _components(k, TAB)
    d_z, h = 0.7, 1e-3
    out = spt.one_loop([k], TAB, d_z=d_z, haf=50.0)
    e = math.exp
    q = lambda a, b: _bilinear(c, d_z * e(a), d_z * e(b))
    dq2 = (q(0, h) - q(0, -h)) / (2 * h)
    d2q = (q(h, h) - q(h, -h) - q(-h, h) + q(-h, -h)) / (4 * h * h)
    assert abs(out["p_dd"][0] / q(0, 0) - 1) < 1e-12
    assert abs(out["p_dtheta_p"][0] / dq2 - 1) < 1e-5, (out["p_dtheta_p"][0], dq2)
    assert abs(out["p_theta_p"][0] / d2q - 1) < 1e-5, (out["p_theta_p"][0], d2q)


def _ppcexp(c, d_z, n_max=2):
    """Eq. Ppcexp's sums over orders, truncated at D_z^(2 n_max): returns
    (P_theta_p, P_delta_theta_p); missing components count as zero."""
    g = lambda j, m: c.get((j, m), 0.0)
    pt, pdt = 0.0, 0.0
    for n in range(1, n_max + 1):
        st = sum(2 * j * (2 * n - j) * g(j, 2 * n - j) for j in range(1, n))
        sdt = sum(2 * n * g(j, 2 * n - j) for j in range(1, n))
        pt += d_z ** (2 * n) * (st + n * n * g(n, n))
        pdt += d_z ** (2 * n) * (sdt + n * g(n, n))
    return pt, pdt


def test_divergence_spectra_follow_the_general_sums():
    """Eq. pdivpD4 is Eq. Ppcexp at n <= 2: the general sums, evaluated order
    by order from the components, give the oracle's combinations."""
    k, d_z = 0.1, 0.8
    c = _components(k, TAB)
    pt, pdt = _ppcexp(c, d_z)
    out = spt.one_loop([k], TAB, d_z=d_z, haf=50.0)
    assert abs(out["p_theta_p"][0] / pt - 1) < 1e-13
    assert abs(out["p_dtheta_p"][0] / pdt - 1) < 1e-13


def _curl_power(k, tab):
    """(k / Haf)^2 times the D_z^4 power of the transverse (curl) part of the
    momentum, from its definition.  At second order p = v_(1) + delta_(1) v_(1)
    + v_(2) with curl-free v; only delta_(1) v_(1) has a transverse part.
    With v_(1)(q) = i Haf q / q^2 delta_(1)(q) and T = 1 - k k^T / k^2, the two
    Wick pairings give, after symmetrising q <-> p = k - q,
    P_perp = Haf^2 / (2 pi)^3 int d^3q P0(q) P0(p) |T q|^2 (1/q^2 - 1/p^2)^2 / 2,
    evaluated in 3D over q in spherical coordinates about k."""
    qn, qw = _panels(np.concatenate([[1e-12, k + tab.k[-1]], tab.k, np.abs(k - tab.k), k + tab.k, [k]]))
    tot = 0.0
    for q, wq in zip(qn, qw):
        mus = (k * k + q * q - tab.k ** 2) / (2 * k * q)
        mu, wm = _panels(np.concatenate([[-1.0, 1.0], mus[(mus > -1) & (mus < 1)]]))
        p2 = k * k + q * q - 2 * k * q * mu
        meas = wq * 2 * math.pi * q * q / (2 * math.pi) ** 3 * wm
        tq2 = q * q * (1 - mu * mu)
        tot += np.sum(meas * tab.scalar(q) * tab(np.sqrt(p2)) * 0.5 * tq2 * (1 / (q * q) - 1 / p2) ** 2)
    return k * k * tot


@pytest.mark.parametrize("k", [0.03, 0.1, 0.3])
def test_momentum_spectrum_is_divergence_plus_curl(k):
    """P_p splits into a longitudinal part, |k.p|^2 / k^2 = (Haf / k)^2
    P_theta_p exactly (theta_p = -div p / Haf), and a transverse part.
    So (k/Haf)^2 P_p^(1) (Eq. PpdD4) minus P_theta_p^(1) (Eq. pdivpD4) is the
    D_z^4 curl power, evaluated here from its own definition.  The D_z^2
    terms cancel; every coefficient of Eq. PpdD4 (P_tt,1, both P_cov, P_B =
    2 k^2 B) and of Eq. pdivpD4 enters the difference."""
    d_z, haf = 0.6, 37.0
    out = spt.one_loop([k], TAB, d_z=d_z, haf=haf)
    lhs = ((k / haf) ** 2 * out["p_mom"][0] - out["p_theta_p"][0]) / d_z ** 4
    rhs = _curl_power(k, TAB)
    assert rhs > 0
    assert abs(lhs / rhs - 1) < 1e-8, (lhs, rhs)


def test_momentum_one_loop_term_is_k4_at_low_k():
    """Momentum conservation: for k far below the spectrum, P_cov^I and
    P_cov^II are each ~ k^2 but cancel, so the D_z^4 term of (k/Haf)^2 P_p
    grows like k^4 (a sign or factor error on either P_cov would leave k^2)."""
    tab = _bump_table(1e-6, 50.0, 80, 1.0)
    a, b = (spt.one_loop([k], tab, d_z=1.0, haf=50.0) for k in (1e-4, 2e-4))
    d4 = lambda o, k: (k / 50.0) ** 2 * o["p_mom"][0] - o["p_lin"][0]
    assert abs(d4(b, 2e-4) / d4(a, 1e-4) / 16.0 - 1) < 2e-3
    assert abs(a["pcov1"][0] / a["pcov2"][0] + 1) < 1e-6
