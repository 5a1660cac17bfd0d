"""The piece-by-piece form of the oracle (oracle.large, for the 512^3
reference spectra) against the direct form (oracle.estimate): the same
steps with the floating-point sums taken in another order, so the spectra
agree to rounding."""
import numpy as np
import pytest

import oracle
from oracle import large
from synth import catalogs


def _close(a, b):
    assert np.array_equal(a.n_modes, b.n_modes)
    for key in ("k_mean", "p_pp", "p_tt", "p_dt", "p_dd", "sn_pp", "sn_tt", "sn_dd"):
        x, y = getattr(a, key), getattr(b, key)
        ok = np.isfinite(y)
        assert np.array_equal(ok, np.isfinite(x)), key
        scale = np.max(np.abs(y[ok]))
        assert np.max(np.abs(x[ok] - y[ok])) <= 1e-11 * scale, (key, np.max(np.abs(x[ok] - y[ok])) / scale)
    assert np.allclose(a.v_bulk, b.v_bulk, rtol=1e-13, atol=0)


@pytest.mark.parametrize("kernel", ["bl3", "bl3q"])
@pytest.mark.parametrize("flags", [0, oracle.FLAG_BULKFLOW_SUBTRACT])
def test_matches_direct_form(kernel, flags):
    pos, vel = catalogs.zeldovich(24, 500.0, 12.0, seed=catalogs.seed_for(2, 90),
                                  bulk=catalogs.bulk_vector(51.5))
    kw = dict(box=500.0, n_grid=32, haf=50.0, n_bins=16, flags=flags, kernel=kernel)
    want = oracle.estimate(pos, vel, **kw)
    got = large.estimate_large(pos, vel, chunk=997, slab=5, **kw)   # ragged chunks and slabs
    _close(got, want)
    got = large.estimate_large(pos, vel, chunk=2999, slab=7, workers=3, **kw)   # chunks in 3 processes
    _close(got, want)


def test_weights_and_edges():
    pos, vel, w = catalogs.uniform_gaussian(6000, 300.0, seed=catalogs.seed_for(2, 91), with_weights=True)
    pos[:50, 0] = 299.999   # cells at the top of the box: blocks wrap around x = 0
    kf = 2 * np.pi / 300.0
    edges = kf * np.array([0.0, 1.5, 2.5, 4.0, 7.9])
    kw = dict(box=300.0, n_grid=16, haf=50.0, k_edges=edges)
    _close(large.estimate_large(pos, vel, w, chunk=1500, slab=3, **kw), oracle.estimate(pos, vel, w, **kw))
