"""Helpers shared by the GPU parity tests."""
import numpy as np


def guarded_rel(gpu, orc, sn):
    """|dP| / (|P_orc| + SN): the per-bin error that stays meaningful when the
    true signal is zero (shot-noise dominated bins)."""
    gpu, orc, sn = map(np.asarray, (gpu, orc, sn))
    ok = np.isfinite(orc)
    return np.abs(gpu[ok] - orc[ok]) / (np.abs(orc[ok]) + np.abs(sn[ok]))


def compare_spectra(g, o, tol, label=""):
    """Assert GPU result dict g matches oracle Spectra o within tol (guarded)."""
    assert np.array_equal(g["n_modes"], o.n_modes), (label, g["n_modes"], o.n_modes)
    empty = o.n_modes == 0
    for key in ("k_mean", "p_pp", "p_tt", "p_dt", "p_dd", "sn_pp", "sn_tt", "sn_dd"):
        assert np.all(np.isnan(g[key][empty])), (label, key)
    assert np.allclose(g["k_mean"][~empty], o.k_mean[~empty], rtol=1e-12), label
    errs = {}
    for key, sn in (("p_pp", o.sn_pp), ("p_tt", o.sn_tt), ("p_dd", o.sn_dd),
                    ("p_dt", np.sqrt(o.sn_dd * o.sn_tt))):
        e = guarded_rel(g[key], getattr(o, key), sn)
        errs[key] = float(e.max()) if e.size else 0.0
    for key in ("sn_pp", "sn_tt", "sn_dd"):
        ov = getattr(o, key)[~empty]
        errs[key] = float(np.max(np.abs(g[key][~empty] - ov) / np.abs(ov))) if ov.size else 0.0
    print(f"{label} max guarded error: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, (label, errs)
    return errs


MU_GUARDS = {"p_dd": ("sn_dd",), "p_pp": ("sn_pp",), "p_tt": ("sn_tt",),
             "p_dt_re": ("sn_dd", "sn_tt"), "p_dt_im": ("sn_dd", "sn_tt"),
             "p_dpb_re": ("sn_dd", "sn_pp"), "p_dpb_im": ("sn_dd", "sn_pp")}


def compare_mu(g, o, tol, label=""):
    """(k, mu) cells of the library against oracle.estimate_mu: exact mode
    counts, NaN in the same empty cells, guarded errors for the spectra (the
    guard of a cross spectrum is the geometric mean of its two shot terms)."""
    assert np.array_equal(g["n_modes"], o["n_modes"]), (label, g["n_modes"], o["n_modes"])
    empty = o["n_modes"] == 0
    full = ~empty
    for key in MU_GUARDS:
        assert np.all(np.isnan(g[key][empty])), (label, key)
    assert np.allclose(g["k_mean"][full], o["k_mean"][full], rtol=1e-12), label
    assert np.allclose(g["mu_mean"][full], o["mu_mean"][full], rtol=1e-12, atol=1e-12), label
    errs = {}
    for key, guards in MU_GUARDS.items():
        sn = np.prod([np.abs(o[k]) for k in guards], axis=0) ** (1.0 / len(guards))
        errs[key] = float(np.max(guarded_rel(g[key], o[key], sn)))
    for key in ("sn_dd", "sn_pp", "sn_tt"):
        ref = np.abs(o[key][full]).max()
        errs[key] = float(np.max(np.abs(g[key][full] - o[key][full])) / ref) if ref > 0 else 0.0
    # the cross spectra's shot terms vanish identically in some cases (unit
    # weights with the bulk flow removed): compare them on their spectrum's scale
    for key, pair in (("sn_dt_im", ("sn_dd", "sn_tt")), ("sn_dpb", ("sn_dd", "sn_pp"))):
        ref = np.sqrt(np.abs(o[pair[0]][full] * o[pair[1]][full]))
        errs[key] = float(np.max(np.abs(g[key][full] - o[key][full]) / ref))
    print(f"{label} max guarded error: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, (label, errs)
    return errs
