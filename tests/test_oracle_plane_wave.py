"""Closed-form pin: a single Zel'dovich plane wave.

Lattice q, x = q + A sin(k0 q_x) e_x, v = Haf A sin(k0 q_x) e_x.  At
k = h k0 e_x, with z = h k0 A and the paper's e^{+ik.r} convention,
delta = (-1)^h J_h(z), p_x = -i (-1)^h Haf A J_h'(z), theta = (-1)^h z J_h'(z)
(Eqs. 1-4 and the divergence of Sec. 2.2), so

    P_dd = J_h^2,  P_pp = (Haf A)^2 J_h'^2,  P_tt = z^2 J_h'^2,
    Re P_dt = z J_h J_h'   (positive for h = 1).

A lattice has no Poisson shot noise, so the spectra are compared without
subtraction.  The truncated BL3 window has W_t(2 pi J) ~ -0.0054 / J^2, and
the lattice comb's sidebands alias onto k at the per-cent level.  Averaging
the phase-corrected transforms over M equally spaced sub-cell translations
along x removes every alias with J not a multiple of M exactly (Eq. rawFFTed:
the alias J picks up the phase e^{-2 pi i J s/M}), leaving the deconvolved
estimate of the continuous field.  The truncated kernel jumps by phi(3) at
+-3, so W_t(w) falls only like 2 phi(3) sin(3w)/w and the surviving aliases
J in M Z leave a residual ~1/M: ~4e-4 in power at M = 64, hence the 1e-3
tolerance (a missing deconvolution is a 20 % error at k0 = 0.875 k_N, a sign
or Haf error is O(1)).
"""
import math

import numpy as np
import pytest
from scipy.special import jv, jvp

import oracle
from synth import catalogs

M_SHIFTS = 64


def _shift_averaged_modes(n_grid, n_lat, box, amp, m_wave, haf):
    pos, vel = catalogs.plane_wave(n_lat, box, amp, m_wave, haf, offset=0.31)
    dl = box / n_grid
    nf = np.rint(np.fft.fftfreq(n_grid) * n_grid)
    F_avg = 0.0
    for s in range(M_SHIFTS):
        shifted = pos.copy()
        shifted[:, 0] += np.float32(s * dl / M_SHIFTS)
        _, mom_used, F = oracle.fourier_fields(shifted, vel, None, box, n_grid)
        phase = np.exp(2j * math.pi * nf * s / (M_SHIFTS * n_grid))
        F_avg = F_avg + F * phase[None, :, None, None]
    F_avg = F_avg / M_SHIFTS
    return oracle.mode_quantities(F_avg, mom_used, box, n_grid, haf,
                                  oracle.FLAG_NO_SHOTNOISE)


@pytest.mark.parametrize("m_wave,amp,harmonics,tol", [
    (3, 20.0, (1, 2, 3), 1e-3),
    (14, 4.0, (1,), 1e-3),      # k0 = 0.875 k_N, where W_t^2 ~ 0.8
])
def test_plane_wave_closed_form(m_wave, amp, harmonics, tol):
    n_grid, n_lat, box, haf = 32, 31, 1000.0, 50.0
    q = _shift_averaged_modes(n_grid, n_lat, box, amp, m_wave, haf)
    k0 = 2 * math.pi * m_wave / box
    for h in harmonics:
        z = h * k0 * amp
        want = {"p_dd": jv(h, z) ** 2, "p_pp": (haf * amp) ** 2 * jvp(h, z) ** 2,
                "p_tt": z * z * jvp(h, z) ** 2, "p_dt": z * jv(h, z) * jvp(h, z)}
        for idx in ((h * m_wave, 0, 0), (-h * m_wave, 0, 0)):
            for key, val in want.items():
                got = q[key][idx]
                assert abs(got / val - 1) < tol, (h, idx, key, got, val)
        assert want["p_dt"] > 0 if h == 1 else True


def test_deconvolution_matters_at_this_k():
    from oracle import bl3
    assert abs(bl3.window_trunc(2 * math.pi * 14 / 32)[0] ** 2 - 1) > 0.1
