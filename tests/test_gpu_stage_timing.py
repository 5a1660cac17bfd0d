"""Stage timing (mps_plan_set_timing) against the untimed estimate.

With timing on, the sort's stages run as separate launches with events
between them (moments and count, scan, permute, grid clear); with timing
off, as fewer launches (the clears together before the count, the moments'
derivation and the scan in one launch).  Both must agree as two untimed
runs do: the mode counts and the moments (v_bulk, sigma_v2, n_eff) bit for
bit; the mean |k| and the shot-noise terms to 1e-13 (each workgroup's FP64
shell sums take LDS atomics in varying order: ~4e-16 measured between
untimed runs); the spectra within the run-to-run agreement of the scatter
form (1e-12 where the grid's sums do not depend on the order of the adds:
the owner-computes and halo forms and the 64-bit fixed point of FP64 grids,
~1e-13 measured; RUN_TOL_F32 for the paired FP32 atomic form).  The timed
estimate is also compared with the oracle, and its stage times must be
non-negative with a positive scatter time."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import RUN_TOL_F32, compare_spectra, guarded_rel
from synth import catalogs

pytestmark = pytest.mark.gpu

BOX = 1000.0
HAF = 50.0
# (grid, particles, precision, scatter form by the mean per 16^3 tile m)
CASES = [(64, 100_000, "f32", "atomic"),    # grids below 128^3: atomic (1563 per tile: paired)
         (128, 150_000, "f32", "gather"),   # m = 293
         (128, 250_000, "f32", "halo"),     # m = 488
         (128, 250_000, "f64", "atomic")]   # FP64, m > 384
RUN_TOL = {"atomic": RUN_TOL_F32, "gather": 1e-12, "halo": 1e-12}
ORACLE_TOL = {"f32": 3e-4, "f64": 1e-5}  # as the parity tests


def _estimate(plan, args, timing):
    plan.set_timing(timing)
    try:
        r = plan.estimate(**args)
        return r, (plan.stage_times() if timing else None)
    finally:
        plan.set_timing(False)


def _agree(a, b, tol, label):
    assert np.array_equal(a["n_modes"], b["n_modes"]), label
    for key in ("v_bulk", "sigma_v2", "n_eff"):
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), (label, key)
    full = a["n_modes"] > 0
    for key in ("k_mean", "sn_pp", "sn_tt", "sn_dd"):
        assert np.allclose(a[key][full], b[key][full], rtol=1e-13, atol=0.0), (label, key)
    for key, sn in (("p_pp", a["sn_pp"]), ("p_tt", a["sn_tt"]), ("p_dd", a["sn_dd"]),
                    ("p_dt", np.sqrt(a["sn_dd"] * a["sn_tt"]))):
        e = guarded_rel(a[key][full], b[key][full], sn[full])
        assert float(e.max()) <= tol, (label, key, float(e.max()))


@pytest.mark.parametrize("n,npart,prec,form", CASES)
def test_timing_on_equals_off(n, npart, prec, form):
    import paper_2005_06170_amd as mps
    print(f"stage timing: N={n} {prec} {form} form, {npart} particles", flush=True)
    pos, vel = catalogs.uniform_gaussian(npart, BOX, 300.0, seed=catalogs.seed_for(6, n + npart))
    args = dict(pos=torch.from_numpy(pos).cuda(), vel=torch.from_numpy(vel).cuda(), box=BOX, haf=HAF)
    plan = mps.Plan(n, prec)
    try:
        off1, _ = _estimate(plan, args, False)
        on, st = _estimate(plan, args, True)
        off2, _ = _estimate(plan, args, False)
    finally:
        plan.close()
    tol = 1e-12 if prec == "f64" else RUN_TOL[form]
    _agree(off1, on, tol, "timing off vs on")
    _agree(off1, off2, tol, "timing off twice")
    print("  stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in st.items()), flush=True)
    assert all(np.isfinite(v) and v >= 0.0 for v in st.values()), st
    assert st["scatter"] > 0.0, st
    o = oracle.estimate(pos, vel, box=BOX, n_grid=n, haf=HAF)
    compare_spectra(on, o, ORACLE_TOL[prec], f"timed N={n} {prec}")
