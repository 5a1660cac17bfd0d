"""Pins of the oracle's quadratic-spline reading of the BL3 function
(Sec. 2.4.1 names the third-order orthogonalised Battle-Lemarie function;
counting order as the number of polynomial coefficients gives the degree-2
member).  The defining properties are tested: the closed-form Fourier
transform with the alias sum taken over images, orthonormality, partition of
unity, symmetry, C^1 smoothness at the half-integer knots and the jump of
the second derivative there; the truncated kernel's window and alias sum as
the gridded amplitude and power of a uniformly placed particle; brute-force
assignment; and zero-mean shot-noise subtraction through the estimator.
"""
import math

import numpy as np

import oracle
from oracle import bl3, bl3_quadratic as q

GL_X, GL_W = np.polynomial.legendre.leggauss(32)


def _integrate(func, lo, hi):
    """Gauss-Legendre on half-unit pieces (phi is one quadratic on each)."""
    tot = 0.0
    for i in range(int(round(2 * (hi - lo)))):
        a = lo + 0.5 * i
        t = a + 0.25 * (GL_X + 1)
        tot += 0.25 * np.sum(GL_W * func(t))
    return tot


def _closed_form_phi_hat(w):
    # sinc^3(w/2) / sqrt(sum_k sinc^6((w + 2 pi k)/2)), the alias sum over
    # images instead of its trigonometric closed form
    ks = np.arange(-400, 401)
    sinc = lambda x: 1.0 if x == 0 else math.sin(x) / x
    den = sum(sinc((w + 2 * math.pi * k) / 2) ** 6 for k in ks)
    return sinc(w / 2) ** 3 / math.sqrt(den)


def test_phi_fourier_transform_is_closed_form():
    for w in [0.0, 0.3, 1.0, 2.0, math.pi, 4.0, 2 * math.pi + 0.3, 9.0]:
        ft = _integrate(lambda x: q.phi(x) * np.cos(w * x), -40, 40)
        assert abs(ft - _closed_form_phi_hat(w)) < 1e-9, w


def test_orthonormal_integer_shifts():
    for n in range(0, 5):
        val = _integrate(lambda x: q.phi(x) * q.phi(x - n), -40, 40)
        assert abs(val - (1.0 if n == 0 else 0.0)) < 1e-11, n


def test_partition_of_unity_and_symmetry():
    x = np.linspace(0.0, 1.0, 37)
    total = sum(q.phi(x - n) for n in range(-40, 41))
    assert np.max(np.abs(total - 1.0)) < 1e-10
    xs = np.linspace(-6, 6, 121)
    assert np.allclose(q.phi(xs), q.phi(-xs), rtol=0, atol=1e-15)


def test_quadratic_spline_knots_are_half_integers():
    """C^1 everywhere; the second derivative jumps at half-integers and is
    constant between them (a quadratic piece)."""
    h = 1e-4
    for m in (-2.5, -1.5, -0.5, 0.5, 1.5, 2.5):
        left = [q.phi(m - h * i) for i in range(3)]
        right = [q.phi(m + h * i) for i in range(3)]
        assert abs((left[0] - left[1]) / h - (right[1] - right[0]) / h) < 1e-3
        d2l = (left[0] - 2 * left[1] + left[2]) / h ** 2
        d2r = (right[0] - 2 * right[1] + right[2]) / h ** 2
        assert abs(d2l - d2r) > 1e-2, m
    for m in (-2.0, -1.0, 0.0, 1.0, 2.0):   # inside a piece: smooth
        d2l = (q.phi(m) - 2 * q.phi(m - h) + q.phi(m - 2 * h)) / h ** 2
        d2r = (q.phi(m + 2 * h) - 2 * q.phi(m + h) + q.phi(m)) / h ** 2
        assert abs(d2l - d2r) < 1e-3, m


def test_differs_from_the_cubic_reading():
    # the two readings of "third order" are different functions: phi(3) is
    # -0.0155 (quadratic) against -0.0250 (cubic)
    assert abs(q.phi(3.0) - bl3.phi(3.0)) > 5e-3
    assert -0.016 < q.phi(3.0) < -0.015


def _uniform_average(func):
    # average over u in [0, 1): each tap weight is a quadratic on [0, 1/2)
    # and on [1/2, 1), so Gauss-Legendre on the two halves is exact
    out = 0.0
    for a in (0.0, 0.5):
        u = a + 0.25 * (GL_X + 1)
        out = out + 0.25 * np.sum(GL_W * func(u))
    return out


def test_window_is_mean_gridded_amplitude():
    taps = np.arange(-2, 4)
    for w in [0.0, 0.4, 1.3, 2.5, math.pi]:
        def amp(u):
            wt = q.tap_weights(u)
            return np.sum(wt * np.exp(-1j * w * (taps[:, None] - u[None, :])), axis=0)
        val = _uniform_average(amp)
        assert abs(val.imag) < 1e-13
        assert abs(val.real - q.window_trunc(w)[0]) < 1e-12, w


def test_alias_sum_is_mean_gridded_power():
    taps = np.arange(-2, 4)
    for w in [0.0, 0.4, 1.3, 2.5, math.pi]:
        def pw(u):
            wt = q.tap_weights(u)
            return np.abs(np.sum(wt * np.exp(-1j * w * taps)[:, None], axis=0)) ** 2
        assert abs(_uniform_average(pw) - float(q.alias_sum_trunc(w))) < 1e-12, w


def test_untruncated_alias_sum_is_one():
    for w in [0.1, 1.0, 2.0, 3.0]:
        J = np.arange(-2000, 2001)
        assert abs(np.sum(q.phi_hat(w + 2 * math.pi * J) ** 2) - 1) < 1e-8


def test_assignment_matches_brute_force(rng):
    n, box = 12, 100.0
    pos = (rng.random((20, 3)) * box).astype(np.float32)
    pos[0] = [0.0, 50.0, 100.0 * 5.5 / 12]     # on a node and on a knot
    pos[1] = [box, -8.0, 37.5]
    qv = rng.normal(size=20)
    got = oracle.assign(pos, qv[None, :], box, n, kernel="bl3q")[0]
    u = pos.astype(np.float64) * (n / box)
    g = np.arange(n)
    want = np.zeros((n, n, n))
    for j in range(len(pos)):
        w = []
        for a in range(3):
            d = g - u[j, a]
            d = d - n * np.ceil((d - n / 2) / n)
            w.append(q.phi_trunc(d))
        want += qv[j] * w[0][:, None, None] * w[1][None, :, None] * w[2][None, None, :]
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def test_shot_noise_is_removed_for_uniform_catalogs():
    """E|F|^2 / W^2 = S C_t(k) for uniform positions: the subtracted spectra
    average to zero over seeds with this kernel's own window and alias sum
    (dropping C_t would leave up to 6 % of the shot term at k_N)."""
    n, box = 16, 500.0
    acc = []
    for seed in range(24):
        rng = np.random.default_rng(2000 + seed)
        pos = (rng.random((4000, 3)) * box).astype(np.float32)
        vel = rng.normal(0, 300, (4000, 3)).astype(np.float32)
        r = oracle.estimate(pos, vel, box=box, n_grid=n, haf=50.0, kernel="bl3q")
        acc.append([r.p_pp / r.sn_pp, r.p_dd / r.sn_dd, r.p_tt / r.sn_tt])
    acc = np.array(acc)
    ok = np.isfinite(acc).all(axis=0)
    m = acc.mean(axis=0)
    se = acc.std(axis=0) / math.sqrt(acc.shape[0])
    assert np.all(np.abs(m[ok]) < 4.5 * se[ok] + 1e-12), np.max(np.abs(m[ok]) / se[ok])
    assert np.max(np.abs(q.alias_sum_trunc(np.linspace(0, np.pi, 9)) - 1)) > 0.05
