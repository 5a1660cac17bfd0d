"""Symmetry pins: the binned spectra are invariant under axis permutations
and integer-cell translations; negating all velocities keeps P_pp and
P_theta-theta and flips Re P_delta-theta."""
import numpy as np

import oracle
from synth import catalogs


def _est(pos, vel, **kw):
    return oracle.estimate(pos, vel, box=1000.0, n_grid=32, haf=50.0, **kw)


def test_axis_permutation_and_velocity_flip():
    pos, vel = catalogs.zeldovich(32, 1000.0, 5.0, seed=21)
    base = _est(pos, vel)
    perm = [2, 0, 1]
    rot = _est(np.ascontiguousarray(pos[:, perm]), np.ascontiguousarray(vel[:, perm]))
    for key in ("p_pp", "p_tt", "p_dt", "p_dd", "sn_pp", "sn_tt"):
        assert np.allclose(getattr(base, key), getattr(rot, key), rtol=1e-9, equal_nan=True), key
    neg = _est(pos, -vel)
    assert np.allclose(base.p_pp, neg.p_pp, rtol=1e-12, equal_nan=True)
    assert np.allclose(base.p_tt, neg.p_tt, rtol=1e-12, equal_nan=True)
    assert np.allclose(base.p_dt, -neg.p_dt, rtol=1e-12, equal_nan=True)


def test_integer_cell_translation():
    pos, vel = catalogs.uniform_gaussian(5000, 1000.0, seed=22)
    pos = (np.round(pos.astype(np.float64) * 256) / 256).astype(np.float32)
    base = _est(pos, vel)
    moved = pos.copy()
    moved[:, 0] += np.float32(2 * 1000.0 / 32)
    moved[:, 2] -= np.float32(5 * 1000.0 / 32)
    shifted = _est(moved, vel)
    for key in ("p_pp", "p_tt", "p_dt", "p_dd"):
        assert np.allclose(getattr(base, key), getattr(shifted, key), rtol=1e-9,
                           atol=1e-9 * np.nanmax(np.abs(getattr(base, key))), equal_nan=True)
