"""Sub-sample spectra on the GPU (mps_estimate_subcubes) against the oracle:
the box cut into n_div^3 cubes (Sec. 2.4.1), each estimated as a periodic
catalog, with the per-bin mean and sample standard deviation over the cubes
(Secs. 3.3, 4.1).  Same tolerances as the single-catalog parity tests."""
import numpy as np
import pytest
import torch

import oracle
from oracle import subcubes as S
from gpu_common import compare_spectra, guarded_rel
from synth import catalogs

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-5, "f32": 3e-4}
BOX = 1000.0
HAF = 50.0
KEYS = ("p_pp", "p_tt", "p_dt", "p_dd")


def _dev(*arrays):
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


@pytest.fixture(scope="module")
def mps():
    import paper_2005_06170_amd as m
    return m


@pytest.fixture(scope="module")
def zel64():
    pos, vel = catalogs.zeldovich(64, BOX, 12.0, haf=HAF, seed=catalogs.seed_for(4, 1))
    vel = vel + catalogs.bulk_vector(51.5).astype(np.float32)  # a bulk flow to remove
    return pos, vel


def _sn(o, key):
    return np.sqrt(o.sn_dd * o.sn_tt) if key == "p_dt" else getattr(o, "sn_" + key[2:])


def _compare_stats(g, want, tol, label):
    """Mean: guarded error as a spectrum.  Standard deviation: each cube is
    within tol (|P_s| + SN_s), so the spread moves by at most about that."""
    subs = [r for r in want["sub"] if r is not None]
    for key in KEYS:
        sn = np.mean([_sn(r, key) for r in subs], axis=0)
        e = guarded_rel(g["mean"][key], want["mean"][key], sn)
        scale = np.max([np.abs(getattr(r, key)) + _sn(r, key) for r in subs], axis=0)
        ok = np.isfinite(want["sdev"][key])
        d = np.abs(g["sdev"][key][ok] - want["sdev"][key][ok]) / scale[ok]
        print(label, key, "mean", float(e.max()), "sdev", float(d.max()), flush=True)
        assert e.max() <= tol and d.max() <= 2 * tol, (label, key)
    np.testing.assert_allclose(g["mean"]["v_bulk"], want["mean"]["v_bulk"], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(g["mean"]["n_eff"], want["mean"]["n_eff"], rtol=1e-12)


@pytest.mark.parametrize("bulk", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_subcubes_match_oracle(mps, zel64, prec, bulk):
    """64 sub-samples of a 64^3-particle Zel'dovich catalog with a bulk flow,
    16^3 grid per 250 Mpc/h cube."""
    pos, vel = zel64
    flags = oracle.FLAG_BULKFLOW_SUBTRACT if bulk else 0
    want = S.estimate_subcubes(pos, vel, box=BOX, n_div=4, n_grid=16, haf=HAF, flags=flags)
    g = mps.Plan(16, prec).estimate_subcubes(*_dev(pos, vel), box=BOX, haf=HAF, n_div=4, bulk_flow=bulk)
    assert np.all(g["status"] == 0)
    for s, (gs, ws) in enumerate(zip(g["sub"], want["sub"])):
        compare_spectra(gs, ws, TOL[prec], f"{prec} bulk={bulk} cube {s}")
        np.testing.assert_allclose(gs["v_bulk"], ws.v_bulk, rtol=1e-9, atol=1e-9)
        assert gs["n_eff"] == ws.n_eff  # the particle count, exactly
    _compare_stats(g, want, TOL[prec], f"{prec} bulk={bulk}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_three_cubes_per_axis_with_weights(mps, prec):
    """n_div = 3 (L / 3 not a binary fraction), weights, positions outside
    [0, L) that wrap, explicit edges."""
    pos, vel, w = catalogs.uniform_gaussian(60000, BOX, seed=catalogs.seed_for(4, 2), with_weights=True)
    pos[:100] -= BOX
    pos[100:200] += 2 * BOX
    kf = 2 * np.pi / (BOX / 3)
    edges = kf * np.array([0.5, 1.5, 2.5, 4.0, 6.0, 7.9])
    want = S.estimate_subcubes(pos, vel, w, box=BOX, n_div=3, n_grid=16, haf=HAF, k_edges=edges)
    g = mps.Plan(16, prec).estimate_subcubes(*_dev(pos, vel, w), box=BOX, haf=HAF, n_div=3, k_edges=edges)
    assert np.all(g["status"] == 0)
    for s, (gs, ws) in enumerate(zip(g["sub"], want["sub"])):
        compare_spectra(gs, ws, TOL[prec], f"{prec} n_div=3 cube {s}")
    _compare_stats(g, want, TOL[prec], f"{prec} n_div=3")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_largest_split(mps, prec):
    """n_div = 8, the largest split (512 sub-samples of 125 Mpc/h, 8^3
    grids), clustered so that the cubes hold very different counts."""
    pos, vel = catalogs.zeldovich(64, BOX, 20.0, haf=HAF, seed=catalogs.seed_for(4, 3))
    want = S.estimate_subcubes(pos, vel, box=BOX, n_div=8, n_grid=8, haf=HAF, n_bins=4)
    g = mps.Plan(8, prec).estimate_subcubes(*_dev(pos, vel), box=BOX, haf=HAF, n_div=8, n_bins=4)
    assert len(g["sub"]) == 512 and np.all(g["status"] == 0)
    for s, (gs, ws) in enumerate(zip(g["sub"], want["sub"])):
        compare_spectra(gs, ws, TOL[prec], f"{prec} n_div=8 cube {s}")
        assert gs["n_eff"] == ws.n_eff
    _compare_stats(g, want, TOL[prec], f"{prec} n_div=8")


def test_empty_cubes_report_zero_weight(mps):
    pos, vel = catalogs.uniform_gaussian(20000, BOX, seed=catalogs.seed_for(4, 3))
    pos[:, 0] *= 0.5  # x < L / 2: the cubes with m_x = 1 are empty
    want = S.estimate_subcubes(pos, vel, box=BOX, n_div=2, n_grid=8, haf=HAF)
    g = mps.Plan(8, "f64").estimate_subcubes(*_dev(pos, vel), box=BOX, haf=HAF, n_div=2)
    assert g["status"].tolist() == [0] * 4 + [-3] * 4
    assert g["sub"][4:] == [None] * 4
    for s in range(4):
        compare_spectra(g["sub"][s], want["sub"][s], TOL["f64"], f"cube {s}")
    _compare_stats(g, want, TOL["f64"], "half empty")


def test_single_cube_is_the_whole_catalog(mps):
    pos, vel = catalogs.uniform_gaussian(30000, BOX, seed=catalogs.seed_for(4, 4))
    plan = mps.Plan(16, "f64")
    g = plan.estimate_subcubes(*_dev(pos, vel), box=BOX, haf=HAF, n_div=1)
    full = plan.estimate(*_dev(pos, vel), box=BOX, haf=HAF)
    # the split reorders the particles: FP64 sums in another order
    for key in KEYS:
        sn = np.sqrt(full["sn_dd"] * full["sn_tt"]) if key == "p_dt" else full["sn_" + key[2:]]
        assert guarded_rel(g["sub"][0][key], full[key], sn).max() < 1e-10
        assert guarded_rel(g["mean"][key], full[key], sn).max() < 1e-10
        assert np.all(np.isnan(g["sdev"][key]))


def test_errors(mps):
    pos, vel = catalogs.uniform_gaussian(1000, BOX, seed=catalogs.seed_for(4, 5))
    plan = mps.Plan(8, "f32")
    bad = pos.copy()
    bad[7, 1] = np.nan
    with pytest.raises(mps.MpsError) as e:
        plan.estimate_subcubes(*_dev(bad, vel), box=BOX, haf=HAF, n_div=2)
    assert e.value.status == -2
    kn = np.pi * 8 / (BOX / 2)
    with pytest.raises(mps.MpsError) as e:  # edges above the sub-box's k_N
        plan.estimate_subcubes(*_dev(pos, vel), box=BOX, haf=HAF, n_div=2,
                               k_edges=[0.1 * kn, 0.5 * kn, 1.5 * kn])
    assert e.value.status == -1
    with pytest.raises(ValueError):
        plan.estimate_subcubes(*_dev(pos, vel), box=BOX, haf=HAF, n_div=9)
    # the plan still works after the failures
    r = plan.estimate_subcubes(*_dev(pos, vel), box=BOX, haf=HAF, n_div=2)
    assert np.all(r["status"] == 0)
