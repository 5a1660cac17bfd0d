"""GPU parity of the untruncated-BL3 path (kernel="bl3_exact").

The library assigns with the cubic B-spline (4 taps) and deconvolves by
sinc^4 per axis with the alias sum A(w); the oracle assigns with the
untruncated BL3 function itself (the B-spline grid filtered by c_n on the
grid, oracle.exact_bl3) and deconvolves by phi_hat with alias sum 1.  The two
agree because c_n is a periodic filter whose transform is A^(-1/2); these
tests check that equality end to end, plus the B-spline grids themselves."""
import numpy as np
import pytest
import torch

import oracle
from oracle import exact_bl3
from gpu_common import compare_mu, compare_spectra
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


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,npart", [(16, 777), (32, 5000)])
def test_bspline_grids_match_oracle(mps, prec, n, npart):
    pos, vel, w = catalogs.uniform_gaussian(npart, BOX, seed=300 + n, with_weights=True)
    pos[0] = [0.0, BOX, -1.0]
    g = mps.Plan(n, prec).assign(*_dev(pos, vel, w), box=BOX, kernel="bl3_exact")
    g = g.cpu().numpy().astype(np.float64)
    w64, v64 = w.astype(np.float64), vel.astype(np.float64)
    q = np.stack([w64, w64 * v64[:, 0], w64 * v64[:, 1], w64 * v64[:, 2]])
    want = exact_bl3.assign_pcs(pos, q, BOX, n)
    err = np.max(np.abs(g - want) / np.abs(want).max(axis=(1, 2, 3), keepdims=True))
    print(prec, n, "B-spline grid max error / max |grid|:", err, flush=True)
    assert err < (1e-12 if prec == "f64" else 2e-6), err


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", ["uniform", "zeldovich_bulk"])
def test_exact_kernel_spectra_match_oracle(mps, prec, case):
    if case == "uniform":
        pos, vel = catalogs.uniform_gaussian(60_000, BOX, seed=catalogs.seed_for(1, 21))
        kw, of = {}, 0
    else:
        pos, vel = catalogs.zeldovich(32, BOX, 10.0, haf=HAF, seed=catalogs.seed_for(2, 21))
        vel = (vel.astype(np.float64) + catalogs.bulk_vector(51.5)[None, :]).astype(np.float32)
        kw, of = {"bulk_flow": True}, oracle.FLAG_BULKFLOW_SUBTRACT
    o = oracle.estimate(pos, vel, box=BOX, n_grid=32, haf=HAF, n_bins=16, flags=of, kernel="bl3_exact")
    g = mps.Plan(32, prec).estimate(*_dev(pos, vel), box=BOX, haf=HAF, n_bins=16, kernel="bl3_exact", **kw)
    compare_spectra(g, o, TOL[prec], f"exact {case} {prec}")


def test_exact_kernel_mu_spectra_match_oracle(mps):
    pos, vel = catalogs.uniform_gaussian(40_000, BOX, seed=catalogs.seed_for(1, 22))
    vel = (vel.astype(np.float64) + catalogs.bulk_vector(341.0)[None, :]).astype(np.float32)
    o = oracle.estimate_mu(pos, vel, box=BOX, n_grid=32, haf=HAF, n_mu=4, n_bins=8, kernel="bl3_exact")
    g = mps.Plan(32, "f64").estimate_mu(*_dev(pos, vel), box=BOX, haf=HAF, n_mu=4, n_bins=8,
                                        kernel="bl3_exact")
    compare_mu(g, o, TOL["f64"], "exact mu f64")
