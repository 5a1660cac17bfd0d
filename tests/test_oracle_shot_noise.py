"""Shot-noise pins: uniform random catalogs have zero signal.

For i.i.d. uniform positions E|F(k)|^2 / W^2 = S C(k) exactly for k != 0
(Eqs. psn, rawPp, rawPtheta), so after deconvolution and subtraction the mean
of every spectrum over seeds is zero.  With an artificial bulk flow (the
paper adds 341 km/s, Sec. 2.4.2) the directional theta shot noise of
Eq. thetanoise must still be removed exactly; the real part of the cross
spectrum has no shot noise (Eq. rawPx).
"""
import numpy as np
import pytest

import oracle
from synth import catalogs

N_SEEDS = 48


def _zscores(bulk, flags):
    n, box, npart = 16, 1000.0, 3000
    rows = {k: [] for k in ("pp", "tt", "dt", "dd")}
    for s in range(N_SEEDS):
        pos, vel = catalogs.uniform_gaussian(npart, box, 300.0, seed=1000 + s, bulk=bulk)
        est = oracle.estimate(pos, vel, box=box, n_grid=n, haf=50.0, n_bins=8, flags=flags)
        rows["pp"].append(est.p_pp / est.sn_pp)
        rows["tt"].append(est.p_tt / est.sn_tt)
        rows["dt"].append(est.p_dt / np.sqrt(est.sn_dd * est.sn_tt))
        rows["dd"].append(est.p_dd / est.sn_dd)
    out = {}
    for k, v in rows.items():
        a = np.array(v)[:, 1:]           # bin 0 is empty at this size
        mean = a.mean(0)
        err = a.std(0, ddof=1) / np.sqrt(N_SEEDS)
        out[k] = (mean / err, a.mean(), a.std(ddof=1) / np.sqrt(a.size))
    return out


@pytest.mark.parametrize("bulk,flags", [
    (None, 0),
    (catalogs.bulk_vector(341.0), 0),
    (catalogs.bulk_vector(341.0), oracle.FLAG_BULKFLOW_SUBTRACT),
])
def test_subtracted_spectra_have_zero_mean(bulk, flags):
    for key, (z, pooled, pooled_err) in _zscores(bulk, flags).items():
        assert np.max(np.abs(z)) < 4.5, (key, z)
        assert abs(pooled) < 4.0 * pooled_err, (key, pooled, pooled_err)


def test_missing_alias_factor_would_be_detected():
    # the alias sum departs from 1 by up to ~12 % at k_N; with 48 seeds the
    # pooled test above resolves a few per cent, so dropping C would fail it
    from oracle import bl3
    c = bl3.alias_sum_trunc(np.linspace(0, np.pi, 9))
    assert np.max(np.abs(c - 1)) > 0.05
