"""GPU parity of the (k, mu_b) spectra and complex cross spectra (Sec. 3)
against oracle.estimate_mu, element by element on seeded catalogs."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import compare_mu
from synth import catalogs

pytestmark = pytest.mark.gpu
TOL = {"f64": 1e-5, "f32": 3e-4}
BOX, HAF = 1000.0, 50.0


@pytest.fixture(scope="module")
def mps():
    import paper_2005_06170_amd as m
    return m


def _dev(*arrays):
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def _oracle_flags(kw):
    return ((oracle.FLAG_BULKFLOW_SUBTRACT if kw.get("bulk_flow") else 0)
            | (oracle.FLAG_NO_SHOTNOISE if kw.get("no_shotnoise") else 0)
            | (oracle.FLAG_NO_DECONVOLVE if kw.get("no_deconvolve") else 0))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", ["uniform_bulk", "zeldovich_axis_bulk_sub", "weights_edges_noshot"])
def test_mu_spectra_match_oracle(mps, prec, case):
    w = None
    axis = None
    kw = {}
    n, n_mu, n_bins, edges = 32, 6, 8, None
    if case == "uniform_bulk":
        pos, vel = catalogs.uniform_gaussian(40_000, BOX, seed=catalogs.seed_for(1, 7))
        vel = (vel.astype(np.float64) + catalogs.bulk_vector(341.0)[None, :]).astype(np.float32)
    elif case == "zeldovich_axis_bulk_sub":
        pos, vel = catalogs.zeldovich(32, BOX, 10.0, haf=HAF, seed=catalogs.seed_for(2, 3))
        vel = (vel.astype(np.float64) + catalogs.bulk_vector(51.5)[None, :]).astype(np.float32)
        axis = np.array([0.3, -1.0, 0.45])
        kw = {"bulk_flow": True}
        n_mu = 5
    else:
        pos, vel, w = catalogs.uniform_gaussian(20_000, BOX, seed=catalogs.seed_for(1, 9),
                                                with_weights=True)
        vel = (vel.astype(np.float64) + np.array([80.0, -20.0, 30.0])[None, :]).astype(np.float32)
        n = 16
        kf = 2 * np.pi / BOX
        edges = kf * np.array([0.5, 2.0, 3.5, 5.0, 7.9])
        n_bins, n_mu = 4, 7
        kw = {"no_shotnoise": True}
    o = oracle.estimate_mu(pos, vel, w, box=BOX, n_grid=n, haf=HAF, n_mu=n_mu, axis=axis,
                           k_edges=edges, n_bins=n_bins, flags=_oracle_flags(kw))
    g = mps.Plan(n, prec).estimate_mu(*_dev(pos, vel, w), box=BOX, haf=HAF, n_mu=n_mu, axis=axis,
                                      n_bins=n_bins, k_edges=edges, **kw)
    assert np.allclose(g["axis"], o["axis"], rtol=0, atol=1e-12)
    compare_mu(g, o, TOL[prec], f"{case} {prec}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_most_mu_cells(mps, prec):
    """64 mu bins, the most allowed, times 8 k bins: 512 cells, the most
    allowed (most hold a handful of modes on a 64^3 grid)."""
    pos, vel = catalogs.zeldovich(48, BOX, 10.0, haf=HAF, seed=catalogs.seed_for(2, 5))
    vel = (vel.astype(np.float64) + catalogs.bulk_vector(51.5)[None, :]).astype(np.float32)
    o = oracle.estimate_mu(pos, vel, box=BOX, n_grid=64, haf=HAF, n_mu=64, n_bins=8,
                           flags=oracle.FLAG_BULKFLOW_SUBTRACT)
    g = mps.Plan(64, prec).estimate_mu(*_dev(pos, vel), box=BOX, haf=HAF, n_mu=64, n_bins=8,
                                       bulk_flow=True)
    assert g["n_modes"].shape == (8, 64)
    compare_mu(g, o, TOL[prec], f"512 cells {prec}")


def test_mu_marginal_matches_isotropic_estimate(mps):
    """The library's own (k, mu) cells sum back to its isotropic bins."""
    pos, vel = catalogs.zeldovich(32, BOX, 10.0, haf=HAF, seed=catalogs.seed_for(2, 4))
    vel = (vel.astype(np.float64) + catalogs.bulk_vector(100.0)[None, :]).astype(np.float32)
    plan = mps.Plan(32, "f64")
    p, v = _dev(pos, vel)
    iso = plan.estimate(p, v, box=BOX, haf=HAF, n_bins=16)
    ani = plan.estimate_mu(p, v, box=BOX, haf=HAF, n_mu=8, n_bins=16)
    cnt = ani["n_modes"]
    assert np.array_equal(cnt.sum(axis=1), iso["n_modes"])
    ok = iso["n_modes"] > 0
    for key, ikey in (("p_dd", "p_dd"), ("p_pp", "p_pp"), ("p_tt", "p_tt"), ("p_dt_re", "p_dt")):
        marg = np.nansum(ani[key] * cnt, axis=1)[ok] / cnt.sum(axis=1)[ok]
        assert np.allclose(marg, iso[ikey][ok], rtol=1e-9, atol=1e-9 * np.nanmax(np.abs(iso[ikey]))), key


def test_mu_error_paths(mps):
    from paper_2005_06170_amd._lib import MpsError
    pos, vel = catalogs.uniform_gaussian(1000, BOX, seed=2)
    p, v = _dev(pos, vel)
    plan = mps.Plan(16, "f32")
    for bad in ({"n_mu": 0}, {"n_mu": 65}, {"n_mu": 32, "n_bins": 17}, {"n_mu": 4, "axis": [0.0, 0.0, 0.0]}):
        kw = {"n_bins": 8, **bad}
        with pytest.raises(MpsError) as e:
            plan.estimate_mu(p, v, box=BOX, haf=HAF, **kw)
        assert e.value.status == -1, bad
    # no bulk flow and no axis: mu_b is undefined
    z = torch.zeros_like(v)
    with pytest.raises(MpsError) as e:
        plan.estimate_mu(p, z, box=BOX, haf=HAF, n_mu=4, n_bins=8)
    assert e.value.status == -1
    # the same catalog with an explicit axis is fine
    r = plan.estimate_mu(p, z, box=BOX, haf=HAF, n_mu=4, n_bins=8, axis=[0.0, 0.0, 1.0])
    assert np.all(np.nan_to_num(r["p_pp"]) == 0.0)
