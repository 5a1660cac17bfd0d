"""The quadratic-spline reading of the third-order Battle-Lemarie kernel
(MPS_KERNEL_BL3_QUADRATIC, Sec. 2.4.1) on the GPU against the oracle
(oracle.bl3_quadratic): grids, spectra in both precisions, the split of each
tap at f = 1/2, weights with ragged edges, and the bulk-flow option."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import compare_spectra
from synth import catalogs

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-5, "f32": 3e-4}
BOX = 1000.0
HAF = 50.0


def _dev(*arrays):
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


@pytest.fixture(scope="module")
def mps():
    import paper_2005_06170_amd as m
    return m


def _knots(n):
    """Coordinates on nodes and at half a cell (the split of every tap),
    exact in float32 for L = 1000 and N = 16."""
    d = BOX / n
    return np.array([[0.5 * d, 1.5 * d, 3.0 * d], [(n - 0.5) * d, 0.0, 2.5 * d],
                     [7.5 * d, 8.0 * d, -0.5 * d]], dtype=np.float32)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_assignment_matches_oracle(mps, prec):
    n = 16
    pos, vel, w = catalogs.uniform_gaussian(3000, BOX, seed=catalogs.seed_for(6, 70), with_weights=True)
    pos[:3] = _knots(n)
    pos[3:40] += BOX * np.where(np.arange(37)[:, None] % 2, 1.0, -1.0).astype(np.float32)
    g = mps.Plan(n, prec).assign(*_dev(pos, vel, w), box=BOX, kernel="bl3q").cpu().numpy().astype(np.float64)
    w64, v64 = w.astype(np.float64), vel.astype(np.float64)
    q = np.stack([w64, w64 * v64[:, 0], w64 * v64[:, 1], w64 * v64[:, 2]])
    want = oracle.assign(pos, q, BOX, n, kernel="bl3q")
    scale = np.abs(want).max(axis=(1, 2, 3), keepdims=True)
    err = float(np.max(np.abs(g - want) / scale))
    print(prec, "bl3q max grid error / max |grid|:", err, flush=True)
    assert err < (1e-12 if prec == "f64" else 2e-6), err


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n_grid", [32, 64])
def test_spectra_match_oracle(mps, prec, n_grid):
    """Zel'dovich catalog with an added bulk flow, removed; 32^3 and 64^3
    grids (one and several 16^3 tiles per axis)."""
    pos, vel = catalogs.zeldovich(40, BOX, 10.0, haf=HAF, seed=catalogs.seed_for(6, 71))
    vel = vel + catalogs.bulk_vector(51.5).astype(np.float32)
    want = oracle.estimate(pos, vel, box=BOX, n_grid=n_grid, haf=HAF, kernel="bl3q",
                           flags=oracle.FLAG_BULKFLOW_SUBTRACT)
    got = mps.Plan(n_grid, prec).estimate(*_dev(pos, vel), box=BOX, haf=HAF, kernel="bl3q", bulk_flow=True)
    compare_spectra(got, want, TOL[prec], f"{prec} bl3q N={n_grid}")


def test_weighted_ragged_edges(mps):
    """Weights, explicit edges and a grid of 8 (one 8^3 tile)."""
    pos, vel, w = catalogs.uniform_gaussian(777, BOX, seed=catalogs.seed_for(6, 72), with_weights=True)
    kf = 2 * np.pi / BOX
    edges = kf * np.array([0.0, 1.2, 2.0, 3.3, 3.99])
    want = oracle.estimate(pos, vel, w, box=BOX, n_grid=8, haf=HAF, kernel="bl3q", k_edges=edges)
    for prec in ("f64", "f32"):
        got = mps.Plan(8, prec).estimate(*_dev(pos, vel, w), box=BOX, haf=HAF, kernel="bl3q", k_edges=edges)
        compare_spectra(got, want, TOL[prec], f"{prec} bl3q N=8")


def test_rejected_with_the_exact_kernel(mps):
    import ctypes as C
    from paper_2005_06170_amd import _lib, api
    pos, vel = _dev(*catalogs.uniform_gaussian(100, BOX, seed=1))
    plan = mps.Plan(8, "f32")
    cat, keep = api.make_catalog(pos, vel, box=BOX, haf=HAF,
                                 flags=_lib.KERNEL_BL3_QUADRATIC | _lib.KERNEL_BL3_EXACT)
    res, _ = api.make_result(cat.n_bins)
    st = _lib.lib().mps_estimate(plan.handle, C.byref(cat), C.byref(res), None)
    assert st == -1, st   # MPS_E_ARG
