"""Helpers shared by the GPU parity tests."""
import hashlib
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

# Run-to-run agreement of FP32 spectra of one catalog (relative to |P| +
# shot noise; FP64 grids sum exact 64-bit fixed point and agree to 1e-12).
# The atomic scatter's flush adds a cell's contributions from neighbouring
# tiles with FP32 atomics in varying order (~1e-7), and the FP32 BL3
# scatter deposits particles of one cell or z-neighbouring cells in pairs,
# rounding each pair's FP32 sum once: which particles pair follows the
# order of the LDS counter atomics of the tile's cell sort, so the
# roundings, not the accuracy, change between runs, up to ~1.1e-6 measured
# on 32^3 grids of 2e4 particles (the FP32 tolerance against the oracle is
# 3e-4).
RUN_TOL_F32 = 4e-6


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


def load_reference(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


class RefSpectra:
    """Attribute view of a stored spectrum (null -> NaN), as compare_spectra expects."""

    def __init__(self, d):
        for k, v in d.items():
            if k == "n_modes":
                setattr(self, k, np.asarray(v, dtype=np.int64))
            elif isinstance(v, list):
                setattr(self, k, np.array([np.nan if x is None else x for x in v], dtype=np.float64))
            else:
                setattr(self, k, v)


def check_fingerprint(pos, vel, fp):
    """The regenerated catalog is the recorded one: same size, FP64 velocity
    moments and mean position (to rounding), and usually the same bytes."""
    assert pos.shape[0] == fp["n_particles"]
    v = vel.astype(np.float64)
    sv = v.sum(axis=0)
    svv = (v.T @ v).ravel()
    scale = np.sqrt(np.abs(np.array(fp["sum_vv"])[[0, 4, 8]]).sum() * pos.shape[0])
    assert np.all(np.abs(sv - fp["sum_v"]) <= 1e-6 * scale), (sv, fp["sum_v"])
    assert np.allclose(svv, fp["sum_vv"], rtol=1e-9, atol=0), (svv, fp["sum_vv"])
    assert np.allclose(np.mean(pos.astype(np.float64), axis=0), fp["mean_pos"], rtol=1e-9, atol=1e-9)
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pos).tobytes())
    h.update(np.ascontiguousarray(vel).tobytes())
    same = h.hexdigest() == fp["sha256"]
    print("catalog bytes identical to the reference's:", same, flush=True)
    return same
