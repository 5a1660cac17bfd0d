"""Pins of the oracle's BL3 construction against facts fixed by mathematics.

The paper names the third-order orthogonalised Battle-Lemarie scaling
function (Sec. 2.4.1) without printing it.  Its defining properties are
tested here: the closed-form Fourier transform, orthonormality, partition of
unity, symmetry and C^2 smoothness of the cubic spline.  The truncated
kernel's window and alias sum are checked against their definitions as the
expected gridded amplitude and power of a randomly placed particle.
"""
import math

import numpy as np

from oracle import bl3

GL_X, GL_W = np.polynomial.legendre.leggauss(32)


def _integrate(func, lo, hi):
    tot = 0.0
    for m in range(lo, hi):
        t = m + 0.5 * (GL_X + 1)
        tot += 0.5 * np.sum(GL_W * func(t))
    return tot


def _closed_form_phi_hat(w):
    # BL3 in Fourier space: sinc^4(w/2) / sqrt(sum_k sinc^8((w + 2 pi k)/2))
    ks = np.arange(-200, 201)
    def sinc(x):
        return 1.0 if x == 0 else math.sin(x) / x
    num = sinc(w / 2) ** 4
    den = sum(sinc((w + 2 * math.pi * k) / 2) ** 8 for k in ks)
    return num / math.sqrt(den)


def test_phi_fourier_transform_is_closed_form():
    for w in [0.0, 0.3, 1.0, 2.0, math.pi, 4.0, 2 * math.pi + 0.3, 9.0]:
        ft = _integrate(lambda x: bl3.phi(x) * np.cos(w * x), -45, 45)
        assert abs(ft - _closed_form_phi_hat(w)) < 1e-9, w


def test_orthonormal_integer_shifts():
    for n in range(0, 5):
        val = _integrate(lambda x: bl3.phi(x) * bl3.phi(x - n), -45, 45)
        assert abs(val - (1.0 if n == 0 else 0.0)) < 1e-11, n


def test_partition_of_unity_and_symmetry():
    x = np.linspace(0.0, 1.0, 37)
    total = sum(bl3.phi(x - n) for n in range(-44, 45))
    assert np.max(np.abs(total - 1.0)) < 1e-10
    xs = np.linspace(-6, 6, 121)
    assert np.allclose(bl3.phi(xs), bl3.phi(-xs), rtol=0, atol=1e-15)


def test_cubic_spline_is_c2_at_knots():
    h = 1e-4
    for m in range(-3, 4):
        left = [bl3.phi(m - h * i) for i in range(3)]
        right = [bl3.phi(m + h * i) for i in range(3)]
        d1l = (left[0] - left[1]) / h
        d1r = (right[1] - right[0]) / h
        d2l = (left[0] - 2 * left[1] + left[2]) / h ** 2
        d2r = (right[0] - 2 * right[1] + right[2]) / h ** 2
        assert abs(d1l - d1r) < 1e-3
        assert abs(d2l - d2r) < 1e-2


def test_tap_weights_cover_the_half_open_support():
    f = np.array([0.0, 0.25, 0.999999])
    w = bl3.tap_weights(f)
    # tap j = 3 at f = 0 sits exactly at d = 3 (kept); j = -2 at f -> 1 tends to -3
    assert np.allclose(w[5, 0], bl3.phi(3.0))
    assert np.allclose(w[:, 1], [bl3.phi(j - 0.25) for j in range(-2, 4)])


def _uniform_average(func):
    # average over the particle fraction u in [0, 1): the truncated kernel's
    # tap weights are cubic polynomials of u, so Gauss-Legendre is exact
    u = 0.5 * (GL_X + 1)
    return 0.5 * np.sum(GL_W * func(u))


def test_window_is_mean_gridded_amplitude():
    # W_t(w) = E_u sum_j phi(j - u) e^{-i w (j - u)}: the expected
    # phase-corrected amplitude of a randomly placed particle
    for w in [0.0, 0.4, 1.3, 2.5, math.pi]:
        taps = np.arange(-2, 4)
        def amp(u):
            wt = bl3.tap_weights(u)            # (6, m)
            ph = np.exp(-1j * w * (taps[:, None] - u[None, :]))
            return np.sum(wt * ph, axis=0)
        val = _uniform_average(amp)
        assert abs(val.imag) < 1e-13
        assert abs(val.real - bl3.window_trunc(w)[0]) < 1e-12, w


def test_alias_sum_is_mean_gridded_power():
    # C_t(w) = E_u |sum_j phi(j - u) e^{-i w j}|^2: a uniformly placed
    # particle's expected power on the grid (the shot-noise factor)
    for w in [0.0, 0.4, 1.3, 2.5, math.pi]:
        taps = np.arange(-2, 4)
        def pw(u):
            wt = bl3.tap_weights(u)
            ph = np.exp(-1j * w * taps)[:, None]
            return np.abs(np.sum(wt * ph, axis=0)) ** 2
        val = _uniform_average(pw)
        assert abs(val - float(bl3.alias_sum_trunc(w))) < 1e-12, w


def test_untruncated_alias_sum_is_one():
    # orthonormality in Fourier space: sum_J |phi_hat(w + 2 pi J)|^2 = 1
    for w in [0.1, 1.0, 2.0, 3.0]:
        J = np.arange(-300, 301)
        assert abs(np.sum(bl3.phi_hat(w + 2 * math.pi * J) ** 2) - 1) < 1e-9
