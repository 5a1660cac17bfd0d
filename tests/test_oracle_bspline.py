"""Pins of the B-spline assignment kernels (orders 1..6: NGP .. quintic),
the comparison kernels of Secs. 2.4.1 and 2.4.3."""
import math

import numpy as np
import pytest

import oracle
from oracle import bspline as B


def test_textbook_values():
    # centred B-splines at integers and half-integers (de Boor's tables)
    cases = {0: {0.0: 1.0, 0.5: 1.0, -0.5: 0.0, 0.7: 0.0},
             1: {0.0: 1.0, 0.5: 0.5, 1.0: 0.0},
             2: {0.0: 0.75, 0.5: 0.5, 1.0: 0.125, 1.5: 0.0},
             3: {0.0: 2 / 3, 1.0: 1 / 6, 2.0: 0.0},
             4: {0.0: 115 / 192, 1.0: 19 / 96, 2.0: 1 / 384},
             5: {0.0: 11 / 20, 1.0: 13 / 60, 2.0: 1 / 120, 3.0: 0.0}}
    for n, vals in cases.items():
        for x, want in vals.items():
            assert abs(float(B.beta(n, np.array(x))) - want) < 1e-14, (n, x)
            if not (n == 0 and abs(x) == 0.5):   # the box is half-open: 1 on (-1/2, 1/2]
                assert abs(float(B.beta(n, np.array(-x))) - want) < 1e-14, (n, -x)


@pytest.mark.parametrize("n", range(6))
def test_partition_of_unity(n):
    x = np.random.default_rng(n).random(200) * 10 - 5
    tot = sum(B.beta(n, x - k) for k in range(-10, 11))
    assert np.max(np.abs(tot - 1.0)) < 1e-12


@pytest.mark.parametrize("n", range(1, 6))
def test_recursive_convolution(n):
    """beta_n = beta_{n-1} * box, by quadrature on the unit pieces."""
    gx, gw = np.polynomial.legendre.leggauss(12)
    x = np.linspace(-3.2, 3.2, 37)
    # (beta_{n-1} * box)(x) = int_{x-1/2}^{x+1/2} beta_{n-1}(t) dt, split at knots
    knots = np.arange(-4.0, 4.01, 0.5)
    for xi in x:
        a, b = xi - 0.5, xi + 0.5
        pts = np.concatenate([[a], knots[(knots > a) & (knots < b)], [b]])
        val = 0.0
        for lo, hi in zip(pts[:-1], pts[1:]):
            t = 0.5 * (hi - lo) * gx + 0.5 * (hi + lo)
            val += 0.5 * (hi - lo) * np.sum(gw * B.beta(n - 1, t))
        assert abs(val - float(B.beta(n, np.array(xi)))) < 1e-13, (n, xi)


@pytest.mark.parametrize("order", B.ORDERS)
def test_window_is_the_fourier_transform(order):
    gx, gw = np.polynomial.legendre.leggauss(12)
    half = order / 2
    edges = np.arange(-half, half + 0.01, 0.5)
    for w in (0.0, 0.3, 1.0, 2.0, math.pi):
        val = 0.0
        for lo, hi in zip(edges[:-1], edges[1:]):
            t = 0.5 * (hi - lo) * gx + 0.5 * (hi + lo)
            val += 0.5 * (hi - lo) * np.sum(gw * B.beta(order - 1, t) * np.cos(w * t))
        assert abs(val - float(B.window(order, np.array(w)))) < 1e-13, (order, w)


@pytest.mark.parametrize("order", B.ORDERS)
def test_alias_sum_matches_the_sum_over_images(order):
    w = np.linspace(0.0, math.pi, 9)
    closed = B.alias_sum(order, w)
    if order == 1:
        np.testing.assert_allclose(closed, 1.0, rtol=0, atol=1e-15)  # sum_J sinc^2 = 1
        return
    J = np.arange(-20000, 20001)
    direct = np.array([np.sum(B.window(order, wi + 2 * math.pi * J) ** 2) for wi in w])
    # the omitted images |J| > 20000 add less than 2 (1 / (pi J))^(2p) J
    np.testing.assert_allclose(direct, closed, rtol=1e-12, atol=0)


@pytest.mark.parametrize("order", B.ORDERS)
def test_assignment_brute_force(order):
    rng = np.random.default_rng(40 + order)
    n, box = 8, 100.0
    pos = (rng.random((30, 3)) * 1.4 * box - 0.2 * box).astype(np.float32)
    q = rng.normal(size=(2, 30))
    got = B.assign(pos, q, box, n, order)
    u = pos.astype(np.float64) * (n / box)
    want = np.zeros((2, n, n, n))
    g = np.arange(n)
    for p in range(30):
        per_axis = []
        for a in range(3):
            # every node, every periodic image within reach
            d = g[:, None] - u[p, a] + n * np.arange(-3, 4)[None, :]
            per_axis.append(B.beta(order - 1, d).sum(axis=1))
        w3 = per_axis[0][:, None, None] * per_axis[1][None, :, None] * per_axis[2][None, None, :]
        want += q[:, p, None, None, None] * w3[None]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(got.sum(axis=(1, 2, 3)), q.sum(axis=1), rtol=1e-12)


def test_order_four_is_the_untruncated_bl3_estimate():
    """phi = sum_n c_n beta3(x - n) with |c_hat|^2 = 1 / A: the deconvolved
    cubic B-spline estimate with alias sum A equals the exact BL3 one."""
    pos, vel, w = (np.random.default_rng(3).random((2000, 3)) * 500.0).astype(np.float32), \
        np.random.default_rng(4).normal(0, 300, (2000, 3)).astype(np.float32), None
    a = oracle.estimate(pos, vel, w, box=500.0, n_grid=16, haf=50.0, kernel="pcs")
    b = oracle.estimate(pos, vel, w, box=500.0, n_grid=16, haf=50.0, kernel="bl3_exact")
    for key in ("p_pp", "p_tt", "p_dt", "p_dd", "sn_pp", "sn_tt", "sn_dd"):
        ok = np.isfinite(getattr(b, key))
        np.testing.assert_allclose(getattr(a, key)[ok], getattr(b, key)[ok], rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_shot_noise_is_removed_for_uniform_catalogs(order):
    """For uniform positions E|F|^2 / W^2 = S C(k) with the kernel's own
    alias sum: the subtracted spectra average to zero over seeds."""
    n, box = 16, 500.0
    acc = []
    for seed in range(24):
        rng = np.random.default_rng(1000 + seed)
        pos = (rng.random((4000, 3)) * box).astype(np.float32)
        vel = rng.normal(0, 300, (4000, 3)).astype(np.float32)
        r = oracle.estimate(pos, vel, box=box, n_grid=n, haf=50.0, kernel=f"bspline{order}")
        acc.append([r.p_pp / r.sn_pp, r.p_dd / r.sn_dd])
    acc = np.array(acc)           # (seeds, 2, bins), in units of the shot term
    ok = np.isfinite(acc).all(axis=0)  # the bins with modes (the same in every seed)
    m = acc.mean(axis=0)
    se = acc.std(axis=0) / math.sqrt(acc.shape[0])
    # no bin's mean is more than 4.5 standard errors from zero
    assert np.all(np.abs(m[ok]) < 4.5 * se[ok] + 1e-12), np.max(np.abs(m[ok]) / se[ok])
