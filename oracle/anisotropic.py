"""Anisotropic (k, mu_b) spectra and the complex cross spectra of Sec. 3.

TEST INFRASTRUCTURE ONLY (see the package docstring).

mu_b is the cosine between k and a direction a, by default the bulk flow
v_b = sum w v / W (Eq. thetanoise and Sec. 3).  Per mode n != 0 with
|k| < k_N, in the paper's Fourier convention (fields sum_j w_j ... e^{+ik.r_j},
Eq. 4):

* delta_P = (1/W) sum w_j e^{ik.r_j},  p_P = (1/W) sum w_j v_j e^{ik.r_j},
  theta_P = i k.p_P / (Haf) (Sec. 2.2);
* P_dd, P_pp, P_tt as in the isotropic estimator (deconvolved, shot
  subtracted);
* the complex cross spectrum P_dt = delta_P theta_P^* / W_t^2 (Eq. rawPx); its
  real part has no shot noise, its imaginary part has the shot term
  -(k.s) C / (Haf W_t^2) with s = sum w^2 v / W^2 (k <v mu> / N of Eq. rawPx,
  weighted), subtracted unless shot noise is off;
* P_{delta p'_b} = delta_P conj(a.p'_P) / W_t^2 with p' the momentum of
  v' = v - v_b (Sec. 3, Eq. bfpp), its real part less the shot term
  (a.(sum w^2 v' / W^2)) C / W_t^2, which vanishes for unit weights.

The library stores half of the spectrum and mirrors each mode to -n; the
oracle uses the full N^3 cube and no mirroring.  p' is obtained by assigning
the particles again with v - v_b, the definition of Sec. 3.1, not by the
Fourier-space shortcut p - v_b delta.

mu bins: uniform on [-1, 1]; with a = axis / |axis| (|axis| =
sqrt(a0 a0 + a1 a1 + a2 a2) in that order), mu = (n_x a0 + n_y a1 + n_z a2) /
sqrt(n^2) and m = min(floor((mu + 1) (n_mu / 2)), n_mu - 1), clamped at 0, all
in FP64 with every operation rounded separately (the library computes the
same sequence, so the bin of every mode agrees exactly).
"""
from __future__ import annotations

import math

import numpy as np

from . import estimator as E


def unit_axis(axis):
    a = [float(x) for x in axis]
    nrm = math.sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2])
    if not nrm > 0.0:
        raise ValueError("the mu axis is zero")
    return np.array([a[0] / nrm, a[1] / nrm, a[2] / nrm])


def mu_bin(nx, ny, nz, n2, ahat, n_mu):
    """mu = k.a / |k| and its bin, in the fixed FP64 operation order."""
    dot = nx.astype(np.float64) * ahat[0]
    dot = dot + ny.astype(np.float64) * ahat[1]
    dot = dot + nz.astype(np.float64) * ahat[2]
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = dot / np.sqrt(n2.astype(np.float64))
    t = (mu + 1.0) * (0.5 * n_mu)
    m = np.floor(np.nan_to_num(t)).astype(np.int64)
    return mu, np.clip(m, 0, n_mu - 1)


def estimate_mu(pos, vel, weight=None, *, box, n_grid, haf, n_mu, axis=None,
                k_edges=None, n_bins=32, flags=0, keep_modes=False, kernel="bl3"):
    """(k, mu_b)-binned spectra; arrays of shape (n_bins, n_mu), times V.
    keep_modes adds the per-mode arrays (full N^3 cube, before binning)."""
    bulk = bool(flags & E.FLAG_BULKFLOW_SUBTRACT)
    mom, mom_used, F = E.fourier_fields(pos, vel, weight, box, n_grid, bulk, kernel)
    q = E.mode_quantities(F, mom_used, box, n_grid, haf, flags, kernel)
    W = mom["W"]
    vb = mom["sv"] / W
    ahat = unit_axis(vb if axis is None else axis)

    # p' of Sec. 3.1: the momentum of v - v_b, assigned again
    if bulk:
        mom_p, Fp = mom_used, F
    else:
        _, mom_p, Fp = E.fourier_fields(pos, vel, weight, box, n_grid, True, kernel)

    n = n_grid
    kf = 2.0 * math.pi / box
    nf = E._integer_freqs(n)
    nx, ny, nz = np.meshgrid(nf, nf, nf, indexing="ij")
    n2 = nx * nx + ny * ny + nz * nz
    kvec = kf * np.stack([nx, ny, nz]).astype(np.float64)
    w1, c1 = E.axis_tables(n, kernel)
    if flags & E.FLAG_NO_DECONVOLVE:
        w1 = np.ones(n)
    win2 = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    calias = c1[:, None, None] * c1[None, :, None] * c1[None, None, :]

    # fields in the paper's e^{+ik.r} convention
    delta_p = np.conj(q["delta"])
    mom_p_vec = np.conj(q["p"])
    theta_p = 1j * np.einsum("a...,a...->...", kvec, mom_p_vec) / haf
    cross = delta_p * np.conj(theta_p) / win2
    s_used = mom_used["s2v"] / mom_used["W"] ** 2
    sn_dt_im = -np.einsum("a...,a->...", kvec, s_used) * calias / (haf * win2)

    pprime = np.conj(Fp[1:4] / mom_p["W"])
    pb = ahat[0] * pprime[0] + ahat[1] * pprime[1] + ahat[2] * pprime[2]
    cross_b = delta_p * np.conj(pb) / win2
    s_prime = mom_p["s2v"] / mom_p["W"] ** 2
    sn_dpb = float(s_prime @ ahat) * calias / win2

    no_shot = bool(flags & E.FLAG_NO_SHOTNOISE)
    per_mode = {
        "p_dd": q["p_dd"], "p_pp": q["p_pp"], "p_tt": q["p_tt"],
        "p_dt_re": cross.real,
        "p_dt_im": cross.imag if no_shot else cross.imag - sn_dt_im,
        "p_dpb_re": cross_b.real if no_shot else cross_b.real - sn_dpb,
        "p_dpb_im": cross_b.imag,
        "sn_dd": q["sn_dd"], "sn_pp": q["sn_pp"], "sn_tt": q["sn_tt"],
        "sn_dt_im": sn_dt_im, "sn_dpb": sn_dpb * np.ones_like(n2, dtype=np.float64),
    }

    # k bins exactly as the isotropic estimator; mu bins as documented
    if k_edges is None:
        kb = E.default_bin_index(n2, n, n_bins)
        edges = kf * (n // 2) * np.arange(n_bins + 1) / n_bins
    else:
        edges = np.asarray(k_edges, dtype=np.float64)
        n_bins = len(edges) - 1
        kb = E.edges_bin_index(n2, E.edge_thresholds(edges, box), n)
    mu, mb = mu_bin(nx, ny, nz, n2, ahat, n_mu)
    sel = kb >= 0
    cell = (kb * n_mu + mb)[sel]
    ncell = n_bins * n_mu
    counts = np.bincount(cell, minlength=ncell).astype(np.int64)
    vol = box ** 3

    def mean_of(arr, scale):
        s = np.bincount(cell, weights=np.asarray(arr)[sel], minlength=ncell)
        with np.errstate(invalid="ignore", divide="ignore"):
            out = np.where(counts > 0, scale * s / counts, np.nan)
        return out.reshape(n_bins, n_mu)

    out = {"k_edges": edges, "n_modes": counts.reshape(n_bins, n_mu),
           "k_mean": mean_of(kf * np.sqrt(n2.astype(np.float64)), 1.0),
           "mu_mean": mean_of(mu, 1.0), "axis": ahat, "v_bulk": vb}
    for key, arr in per_mode.items():
        out[key] = mean_of(arr, vol)
    if keep_modes:
        out["modes"] = dict(per_mode, mu=mu, kmag=kf * np.sqrt(n2.astype(np.float64)),
                            k_bin=kb, mu_bin=mb)
    return out
