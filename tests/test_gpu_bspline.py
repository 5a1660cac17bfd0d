"""B-spline assignment kernels on the GPU (MPS_KERNEL_BSPLINE(p), p = 1..6:
the comparison kernels of Secs. 2.4.1 and 2.4.3) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from oracle import bspline as B
from gpu_common import compare_mu, compare_spectra
from synth import catalogs

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-5, "f32": 3e-4}
BOX = 1000.0
HAF = 50.0
ORDERS = [1, 2, 3, 4, 5, 6]


def _dev(*arrays):
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


@pytest.fixture(scope="module")
def mps():
    import paper_2005_06170_amd as m
    return m


def _ties(n):
    """Positions on half-integer and integer grid coordinates (exact in
    float32 for L = 1000 and N = 16): where NGP's box and the odd orders'
    nearest node change."""
    d = BOX / n
    return np.array([[0.5 * d, 1.5 * d, 3.0 * d], [(n - 0.5) * d, 0.0, 2.5 * d],
                     [7.5 * d, 8.0 * d, -0.5 * d]], dtype=np.float32)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("order", ORDERS)
def test_assignment_matches_oracle(mps, prec, order):
    n = 16
    pos, vel, w = catalogs.uniform_gaussian(3000, BOX, seed=catalogs.seed_for(6, order), with_weights=True)
    pos[:3] = _ties(n)
    pos[3:40] += BOX * np.where(np.arange(37)[:, None] % 2, 1.0, -1.0).astype(np.float32)  # wrap
    plan = mps.Plan(n, prec)
    g = plan.assign(*_dev(pos, vel, w), box=BOX, kernel=f"bspline{order}").cpu().numpy().astype(np.float64)
    w64, v64 = w.astype(np.float64), vel.astype(np.float64)
    q = np.stack([w64, w64 * v64[:, 0], w64 * v64[:, 1], w64 * v64[:, 2]])
    want = B.assign(pos, q, BOX, n, order)
    scale = np.abs(want).max(axis=(1, 2, 3), keepdims=True)
    err = float(np.max(np.abs(g - want) / scale))
    print(prec, "order", order, "max grid error / max |grid|:", err, flush=True)
    assert err < (1e-12 if prec == "f64" else 2e-6), err


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("order", ORDERS)
def test_spectra_match_oracle(mps, prec, order):
    """Zel'dovich catalog with a bulk flow, removed, on a 32^3 grid."""
    pos, vel = catalogs.zeldovich(40, BOX, 10.0, haf=HAF, seed=catalogs.seed_for(6, 10 + order))
    vel = vel + catalogs.bulk_vector(51.5).astype(np.float32)
    name = f"bspline{order}"
    want = oracle.estimate(pos, vel, box=BOX, n_grid=32, haf=HAF, kernel=name,
                           flags=oracle.FLAG_BULKFLOW_SUBTRACT)
    got = mps.Plan(32, prec).estimate(*_dev(pos, vel), box=BOX, haf=HAF, kernel=name, bulk_flow=True)
    compare_spectra(got, want, TOL[prec], f"{prec} order {order}")


@pytest.mark.parametrize("order", [1, 5])
def test_weighted_ragged_edges(mps, order):
    """Weights, explicit edges and a grid of 8 (one tile)."""
    pos, vel, w = catalogs.uniform_gaussian(777, BOX, seed=catalogs.seed_for(6, 20 + order), with_weights=True)
    kf = 2 * np.pi / BOX
    edges = kf * np.array([0.0, 1.2, 2.0, 3.3, 3.99])
    name = f"bspline{order}"
    want = oracle.estimate(pos, vel, w, box=BOX, n_grid=8, haf=HAF, kernel=name, k_edges=edges)
    for prec in ("f64", "f32"):
        got = mps.Plan(8, prec).estimate(*_dev(pos, vel, w), box=BOX, haf=HAF, kernel=name, k_edges=edges)
        compare_spectra(got, want, TOL[prec], f"{prec} order {order} N=8")


def test_order_four_equals_the_untruncated_bl3_flag(mps):
    pos, vel = catalogs.uniform_gaussian(20000, BOX, seed=catalogs.seed_for(6, 30))
    for prec in ("f64", "f32"):
        plan = mps.Plan(32, prec)
        a = plan.estimate(*_dev(pos, vel), box=BOX, haf=HAF, kernel="pcs")
        b = plan.estimate(*_dev(pos, vel), box=BOX, haf=HAF, kernel="bl3_exact")
        # the same kernels and tables; only the order of atomic additions
        # (FP64 in LDS, FP32 in the halo flush) and of the per-workgroup
        # shell sums differs between runs
        for key in ("sn_pp", "sn_tt", "sn_dd", "k_mean"):
            np.testing.assert_allclose(a[key], b[key], rtol=1e-13)
        for key, sn in (("p_pp", b["sn_pp"]), ("p_tt", b["sn_tt"]), ("p_dd", b["sn_dd"]),
                        ("p_dt", np.sqrt(b["sn_dd"] * b["sn_tt"]))):
            ok = np.isfinite(b[key])
            assert np.all(np.abs(a[key][ok] - b[key][ok]) <= 1e-6 * (np.abs(b[key][ok]) + sn[ok])), key


@pytest.mark.parametrize("order", [2, 5])
def test_mu_spectra_match_oracle(mps, order):
    pos, vel = catalogs.uniform_gaussian(20000, BOX, seed=catalogs.seed_for(6, 40 + order),
                                         bulk=catalogs.bulk_vector(341.0))
    name = f"bspline{order}"
    want = oracle.estimate_mu(pos, vel, box=BOX, n_grid=16, haf=HAF, n_mu=4, kernel=name)
    got = mps.Plan(16, "f64").estimate_mu(*_dev(pos, vel), box=BOX, haf=HAF, n_mu=4, kernel=name)
    compare_mu(got, want, TOL["f64"], f"mu order {order}")


def test_kernel_flags_are_validated(mps):
    from paper_2005_06170_amd import _lib as L
    import ctypes as C
    from paper_2005_06170_amd.api import make_catalog, make_result
    pos, vel = catalogs.uniform_gaussian(100, BOX, seed=catalogs.seed_for(6, 50))
    p, v = _dev(pos, vel)
    plan = mps.Plan(8, "f32")
    # order 7 of the kernel field is the quadratic BL3 reading, valid on its
    # own but not with the exact kernel
    for flags in (L.KERNEL_BL3_EXACT | (2 << L.KERNEL_ORDER_SHIFT), L.KERNEL_BL3_EXACT | L.KERNEL_BL3_QUADRATIC,
                  1 << 8):
        cat, keep = make_catalog(p, v, box=BOX, haf=HAF, flags=flags)
        res, _ = make_result(cat.n_bins)
        st = L.lib().mps_estimate(plan.handle, C.byref(cat), C.byref(res),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == -1, (flags, st)
    r = plan.estimate(p, v, box=BOX, haf=HAF, kernel="ngp")   # the plan still works
    full = r["n_modes"] > 0
    assert full.any() and np.all(np.isfinite(r["p_pp"][full])) and np.all(np.isnan(r["p_pp"][~full]))
