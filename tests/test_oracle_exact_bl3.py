"""Pins of the oracle's untruncated BL3 assignment (oracle.exact_bl3).

* The cubic B-spline taps sum to one for every fraction, so the cubic
  B-spline grid holds the total charge exactly.
* The exact grid (cubic B-spline grid filtered by c_n) equals the direct sum
  of the untruncated phi over every periodic image of every particle within
  |d| <= 30 (phi decays like 0.51^|d|), on small grids.
* phi is orthonormal: the alias sum of phi_hat^2 is 1 at every frequency.
* A Zel'dovich plane wave assigned with the exact kernel reproduces its
  closed form (Sec. 2.2; the same construction as the truncated-kernel pin,
  with the alias sum equal to 1).
"""
import math

import numpy as np
import pytest
from scipy.special import jv, jvp

import oracle
from oracle import bl3, exact_bl3
from synth import catalogs


def test_bspline_taps_partition_unity(rng):
    f = rng.random(1000)
    s = sum(bl3.bspline3(j - f) for j in exact_bl3.PCS_TAPS)
    assert np.max(np.abs(s - 1.0)) < 1e-14
    pos = (rng.random((300, 3)) * 100.0).astype(np.float32)
    q = rng.normal(size=(1, 300))
    g = exact_bl3.assign_pcs(pos, q, 100.0, 16)
    assert abs(g.sum() - q.sum()) < 1e-11 * np.abs(q).sum()


def _direct_exact(pos, q, box, n, reach=30):
    u = np.asarray(pos, dtype=np.float64) * (n / box)
    g = np.arange(n)
    out = np.zeros((n, n, n))
    for p in range(len(pos)):
        w = []
        for a in range(3):
            acc = np.zeros(n)
            base = g - u[p, a]
            for img in range(-(reach // n) - 2, reach // n + 3):
                d = base + img * n
                acc += np.where(np.abs(d) <= reach, bl3.phi(d), 0.0)
            w.append(acc)
        out += q[p] * w[0][:, None, None] * w[1][None, :, None] * w[2][None, None, :]
    return out


@pytest.mark.parametrize("n", [8, 16])
def test_exact_grid_is_the_untruncated_sum(rng, n):
    box = 100.0
    pos = (rng.random((6, 3)) * box).astype(np.float32)
    pos[0] = [0.0, box, -3.0]
    q = rng.normal(size=6)
    got = exact_bl3.assign_exact(pos, q[None, :], box, n)[0]
    want = _direct_exact(pos, q, box, n)
    assert np.max(np.abs(got - want)) < 1e-8 * np.max(np.abs(want))


def test_phi_is_orthonormal():
    w = np.linspace(0.0, 2 * math.pi, 97)
    assert np.max(np.abs(exact_bl3.alias_sum_exact(w) - 1.0)) < 1e-12


def test_plane_wave_closed_form_exact_kernel():
    n_grid, n_lat, box, haf, amp, m_wave = 32, 31, 1000.0, 50.0, 20.0, 3
    pos, vel = catalogs.plane_wave(n_lat, box, amp, m_wave, haf, offset=0.31)
    dl = box / n_grid
    nf = np.rint(np.fft.fftfreq(n_grid) * n_grid)
    F_avg = 0.0
    m_shifts = 16
    for s in range(m_shifts):
        shifted = pos.copy()
        shifted[:, 0] += np.float32(s * dl / m_shifts)
        _, mom_used, F = oracle.fourier_fields(shifted, vel, None, box, n_grid, kernel="bl3_exact")
        phase = np.exp(2j * math.pi * nf * s / (m_shifts * n_grid))
        F_avg = F_avg + F * phase[None, :, None, None]
    F_avg = F_avg / m_shifts
    q = oracle.mode_quantities(F_avg, mom_used, box, n_grid, haf, oracle.FLAG_NO_SHOTNOISE,
                               kernel="bl3_exact")
    k0 = 2 * math.pi * m_wave / box
    for h in (1, 2):
        z = h * k0 * amp
        want = {"p_dd": jv(h, z) ** 2, "p_pp": (haf * amp) ** 2 * jvp(h, z) ** 2,
                "p_tt": z * z * jvp(h, z) ** 2, "p_dt": z * jv(h, z) * jvp(h, z)}
        for idx in ((h * m_wave, 0, 0), (-h * m_wave, 0, 0)):
            for key, val in want.items():
                got = q[key][idx]
                assert abs(got / val - 1) < 1e-5, (h, idx, key, got, val)
