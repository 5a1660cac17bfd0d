"""Host-resident catalogs (MPS_CATALOG_HOST): every entry point copies them
to the device first and then gives what the same catalog gives from device
memory.  Results may differ only by the order of atomic additions (FP32 halo
flush, FP64 LDS adds), far below the parity tolerance."""
import numpy as np
import pytest
import torch

from gpu_common import RUN_TOL_F32, guarded_rel
from synth import catalogs

pytestmark = pytest.mark.gpu

BOX = 1000.0
HAF = 50.0


@pytest.fixture(scope="module")
def mps():
    import paper_2005_06170_amd as m
    return m


def _host(*arrays, pinned=True):
    out = []
    for a in arrays:
        t = torch.from_numpy(np.ascontiguousarray(a))
        out.append(t.pin_memory() if pinned else t)
    return out


def _close(a, b, tol, keys=("p_pp", "p_tt", "p_dd", "p_dt")):
    for key in keys:
        sn = np.sqrt(b["sn_dd"] * b["sn_tt"]) if key == "p_dt" else b["sn_" + key[2:]]
        e = guarded_rel(a[key], b[key], sn)
        assert e.size and e.max() <= tol, (key, float(e.max()))
    assert np.array_equal(a["n_modes"], b["n_modes"])


@pytest.mark.parametrize("pinned", [True, False])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_estimate_from_host_memory(mps, prec, pinned):
    pos, vel, w = catalogs.uniform_gaussian(300_000, BOX, seed=catalogs.seed_for(7, 1), with_weights=True)
    plan = mps.Plan(64, prec)
    dev = plan.estimate(*(torch.from_numpy(a).cuda() for a in (pos, vel, w)), box=BOX, haf=HAF, bulk_flow=True)
    host = plan.estimate(*_host(pos, vel, w, pinned=pinned), box=BOX, haf=HAF, bulk_flow=True)
    _close(host, dev, 1e-12 if prec == "f64" else RUN_TOL_F32)
    np.testing.assert_allclose(host["v_bulk"], dev["v_bulk"], rtol=1e-12)


def test_other_entry_points_from_host_memory(mps):
    pos, vel = catalogs.zeldovich(40, BOX, 10.0, haf=HAF, seed=catalogs.seed_for(7, 2))
    hp, hv = _host(pos, vel)
    dp, dv = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
    plan = mps.Plan(32, "f64")
    g_host = plan.assign(hp, hv, box=BOX).cpu().numpy()
    g_dev = plan.assign(dp, dv, box=BOX).cpu().numpy()
    assert np.max(np.abs(g_host - g_dev)) <= 1e-12 * np.abs(g_dev).max()
    m_host = plan.estimate_mu(hp, hv, box=BOX, haf=HAF, n_mu=4, axis=(0, 0, 1))
    m_dev = plan.estimate_mu(dp, dv, box=BOX, haf=HAF, n_mu=4, axis=(0, 0, 1))
    full = m_dev["n_modes"] > 0
    for key in ("p_pp", "p_dt_re", "p_dt_im"):
        assert np.allclose(m_host[key][full], m_dev[key][full], rtol=1e-9, atol=1e-9 * np.abs(m_dev[key][full]).max())
    s_host = mps.Plan(8, "f64").estimate_subcubes(hp, hv, box=BOX, haf=HAF, n_div=2)
    s_dev = mps.Plan(8, "f64").estimate_subcubes(dp, dv, box=BOX, haf=HAF, n_div=2)
    assert s_host["status"].tolist() == s_dev["status"].tolist()
    for a, b in zip(s_host["sub"], s_dev["sub"]):
        _close(a, b, 1e-12)


def test_server_with_host_catalogs(mps):
    """Pinned and pageable host catalogs through the server, interleaved with
    device ones, each equal to its device-memory estimate."""
    specs = [(200_000, 64, "f32", True), (50_000, 32, "f64", False), (600_000, 128, "f32", True),
             (10_000, 16, "f32", False)]
    srv = mps.Server(hbm_budget_bytes=8 << 30, max_inflight=3, small_particles=100_000)
    try:
        jobs = []
        for i, (n, grid, prec, pinned) in enumerate(specs):
            pos, vel = catalogs.uniform_gaussian(n, BOX, seed=catalogs.seed_for(7, 10 + i))
            hp, hv = _host(pos, vel, pinned=pinned)
            dp, dv = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
            t_host = srv.submit(hp, hv, box=BOX, haf=HAF, n_grid=grid, precision=prec)
            t_dev = srv.submit(dp, dv, box=BOX, haf=HAF, n_grid=grid, precision=prec)
            jobs.append((t_host, t_dev, prec, (hp, hv, dp, dv)))
        for t_host, t_dev, prec, _keep in jobs:
            _close(srv.wait(t_host, 300.0), srv.wait(t_dev, 300.0), 1e-12 if prec == "f64" else RUN_TOL_F32)
    finally:
        srv.close()


def test_mixed_host_and_device_arrays_are_rejected(mps):
    pos, vel = catalogs.uniform_gaussian(1000, BOX, seed=catalogs.seed_for(7, 20))
    with pytest.raises(ValueError):
        mps.Plan(8, "f32").estimate(torch.from_numpy(pos), torch.from_numpy(vel).cuda(), box=BOX, haf=HAF)
