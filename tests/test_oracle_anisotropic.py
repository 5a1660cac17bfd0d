"""Pins of the oracle's (k, mu_b) spectra and complex cross spectra (Sec. 3).

* Refining shells into mu bins is additive: the mode-weighted mean over mu of
  every spectrum is the isotropic oracle's value.
* Eq. bfpp holds mode by mode: with p = p' + v_b delta (exact by linearity of
  the assignment), P_p = P_p' + 2 v_b Re P_{delta p'_b} + v_b^2 P_dd, for the
  raw spectra and, with the shot terms tr S = tr S' + 2 v_b (s'.v_b/v_b) +
  v_b^2 S_dd, for the subtracted ones.
* Eq. bfpdpx holds mode by mode: Re P_dt = Re P_dt', Im P_dt = Im P_dt' -
  k mu_b (v_b / Haf) P_dd, and P_tt = P_tt' - 2 k mu_b (v_b / Haf) Im P_dt' +
  (k mu_b v_b / Haf)^2 P_dd.
* Fig. 1: for uniform random positions with a bulk flow, the mean of the raw
  Im P_dt over realisations is the shot term -(k.s) C / (Haf W^2) (the sign
  of Eq. rawPx), and the subtracted Im P_dt has mean zero.
* Reversing the axis mirrors the mu bins and negates P_{delta p'_b}.
"""
import math

import numpy as np
import pytest

import oracle
from synth import catalogs

BOX, HAF = 1000.0, 50.0


def _catalog(seed, n=4000, vb=(120.0, -60.0, 200.0)):
    pos, vel = catalogs.zeldovich(16, BOX, 20.0, haf=HAF, seed=seed)
    vel = (vel.astype(np.float64) + np.asarray(vb)[None, :]).astype(np.float32)
    return pos, vel


def test_mu_marginal_equals_isotropic():
    pos, vel = _catalog(1)
    w = np.random.default_rng(2).uniform(0.5, 1.5, pos.shape[0]).astype(np.float32)
    for flags in (0, oracle.FLAG_BULKFLOW_SUBTRACT):
        iso = oracle.estimate(pos, vel, w, box=BOX, n_grid=16, haf=HAF, n_bins=8, flags=flags)
        ani = oracle.estimate_mu(pos, vel, w, box=BOX, n_grid=16, haf=HAF, n_mu=5, n_bins=8,
                                 flags=flags)
        cnt = ani["n_modes"]
        assert np.array_equal(cnt.sum(axis=1), iso.n_modes)
        ok = iso.n_modes > 0
        for key, iso_key in (("p_dd", "p_dd"), ("p_pp", "p_pp"), ("p_tt", "p_tt"),
                             ("p_dt_re", "p_dt"), ("sn_tt", "sn_tt")):
            marg = np.nansum(ani[key] * cnt, axis=1)[ok] / cnt.sum(axis=1)[ok]
            want = getattr(iso, iso_key)[ok]
            assert np.allclose(marg, want, rtol=1e-10, atol=1e-10 * np.abs(want).max()), (flags, key)


@pytest.mark.parametrize("flags", [oracle.FLAG_NO_SHOTNOISE, 0])
def test_bulk_flow_identities_per_mode(flags):
    pos, vel = _catalog(3)
    off = oracle.estimate_mu(pos, vel, box=BOX, n_grid=16, haf=HAF, n_mu=4, n_bins=8,
                             flags=flags, keep_modes=True)
    on = oracle.estimate_mu(pos, vel, box=BOX, n_grid=16, haf=HAF, n_mu=4, n_bins=8,
                            flags=flags | oracle.FLAG_BULKFLOW_SUBTRACT, keep_modes=True)
    a, b = off["modes"], on["modes"]
    vb = np.linalg.norm(off["v_bulk"])
    sel = (a["k_bin"] >= 0)
    kmu = (a["kmag"] * a["mu"])[sel]
    # Eq. bfpp
    lhs = a["p_pp"][sel]
    rhs = b["p_pp"][sel] + 2 * vb * b["p_dpb_re"][sel] + vb * vb * b["p_dd"][sel]
    assert np.allclose(lhs, rhs, rtol=1e-9, atol=1e-9 * np.abs(lhs).max())
    # Eq. bfpdpx (the divergence relation and the cross spectrum)
    assert np.allclose(a["p_dt_re"][sel], b["p_dt_re"][sel], atol=1e-9 * np.abs(a["p_dt_re"]).max())
    r = vb / HAF
    want_im = b["p_dt_im"][sel] - kmu * r * b["p_dd"][sel]
    assert np.allclose(a["p_dt_im"][sel], want_im, atol=1e-9 * np.abs(want_im).max())
    want_tt = b["p_tt"][sel] - 2 * kmu * r * b["p_dt_im"][sel] + (kmu * r) ** 2 * b["p_dd"][sel]
    assert np.allclose(a["p_tt"][sel], want_tt, rtol=1e-9, atol=1e-9 * np.abs(want_tt).max())


def test_imaginary_cross_shot_noise_of_a_bulk_flow():
    """Fig. 1: random positions, Gaussian velocities plus v_b = 341 km/s."""
    n_real, n_grid = 24, 16
    vb = catalogs.bulk_vector(341.0)
    raw, sub, sn = [], [], None
    for s in range(n_real):
        pos, vel = catalogs.uniform_gaussian(3000, BOX, seed=catalogs.seed_for(1, 40 + s))
        vel = (vel.astype(np.float64) + vb[None, :]).astype(np.float32)
        kw = dict(box=BOX, n_grid=n_grid, haf=HAF, n_mu=4, n_bins=4, axis=vb)
        r0 = oracle.estimate_mu(pos, vel, flags=oracle.FLAG_NO_SHOTNOISE, **kw)
        r1 = oracle.estimate_mu(pos, vel, **kw)
        raw.append(r0["p_dt_im"])
        sub.append(r1["p_dt_im"])
        sn = r1["sn_dt_im"] if sn is None else sn + r1["sn_dt_im"]
    raw, sub, sn = np.array(raw), np.array(sub), sn / n_real
    err = raw.std(axis=0, ddof=1) / math.sqrt(n_real)
    ok = np.isfinite(sn) & (err > 0)
    # the raw mean is the predicted shot term, far from zero along the flow
    assert np.all(np.abs(raw.mean(axis=0) - sn)[ok] < 5 * err[ok])
    assert np.all(np.abs(sub.mean(axis=0))[ok] < 5 * err[ok])
    big = np.abs(sn) > 10 * err
    assert big.any()
    # sign of Eq. rawPx: negative where mu_b > 0
    mu = r1["mu_mean"]
    assert np.all(sn[big & (mu > 0)] < 0) and np.all(sn[big & (mu < 0)] > 0)


def test_reversed_axis_mirrors_mu_bins():
    pos, vel = _catalog(5)
    ax = np.array([1.0, 2.3, -0.7])
    kw = dict(box=BOX, n_grid=16, haf=HAF, n_mu=7, n_bins=8)
    a = oracle.estimate_mu(pos, vel, axis=ax, **kw)
    b = oracle.estimate_mu(pos, vel, axis=-ax, **kw)
    assert np.array_equal(a["n_modes"], b["n_modes"][:, ::-1])
    for key in ("p_dd", "p_pp", "p_tt", "p_dt_re", "p_dt_im"):
        assert np.allclose(a[key], b[key][:, ::-1], equal_nan=True, rtol=1e-12, atol=1e-9), key
    for key in ("p_dpb_re", "p_dpb_im"):
        assert np.allclose(a[key], -b[key][:, ::-1], equal_nan=True, rtol=1e-12, atol=1e-9), key
