"""mps_estimate_static (the estimate with no device allocation, its workspace
a fixed file-scope device array) against mps_estimate on the same catalogs,
through the C ABI: two calls in a row, the second with a smaller catalog and
grid, in both precisions; and its size limits."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import guarded_rel
from synth import catalogs

pytestmark = pytest.mark.gpu

BOX = 1000.0
HAF = 50.0


@pytest.fixture(scope="module")
def lib():
    from paper_2005_06170_amd import _lib
    return _lib


def _static(lib, pos, vel, n_grid, prec, n_bins=32, flags=0, weight=None):
    from paper_2005_06170_amd import api
    cat, keep = api.make_catalog(pos, vel, weight, box=BOX, haf=HAF, n_bins=n_bins, flags=flags)
    res, arrays = api.make_result(cat.n_bins)
    st = lib.lib().mps_estimate_static(C.byref(cat), int(n_grid), int(prec), C.byref(res),
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    del keep
    return st, api.unpack_result(res, arrays, BOX, n_grid, None, cat.n_bins)


def _same(a, b, tol):
    assert np.array_equal(a["n_modes"], b["n_modes"])
    for key, sn in (("p_pp", "sn_pp"), ("p_tt", "sn_tt"), ("p_dd", "sn_dd")):
        e = guarded_rel(a[key], b[key], b[sn])
        assert e.size == 0 or e.max() <= tol, (key, e.max())
        ok = np.isfinite(b[sn])
        assert np.allclose(a[sn][ok], b[sn][ok], rtol=1e-12, atol=0), sn
    e = guarded_rel(a["p_dt"], b["p_dt"], np.sqrt(b["sn_dd"] * b["sn_tt"]))
    assert e.size == 0 or e.max() <= tol
    assert np.allclose(a["v_bulk"], b["v_bulk"], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_static_equals_plan_estimate_twice(lib, prec):
    import paper_2005_06170_amd as mps
    p = lib.MPS_F32 if prec == "f32" else lib.MPS_F64
    tol = 1e-6 if prec == "f32" else 1e-12
    # the paper-sized small case (64^3, 1e5 particles), then a smaller one
    cases = [(64, catalogs.uniform_gaussian(100_000, BOX, 300.0, seed=catalogs.seed_for(1, 60))),
             (32, catalogs.zeldovich(30, BOX, 20.0, haf=HAF, seed=catalogs.seed_for(1, 61)))]
    for n_grid, (pos, vel) in cases:
        print(prec, "static estimate", n_grid, "grid,", pos.shape[0], "particles", flush=True)
        dp, dv = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
        want = mps.Plan(n_grid, prec).estimate(dp, dv, box=BOX, haf=HAF)
        st, got = _static(lib, dp, dv, n_grid, p)
        assert st == 0, lib.ERRORS.get(st, st)
        _same(got, want, tol)


def test_static_limits(lib):
    pos, vel = catalogs.uniform_gaussian(1000, BOX, seed=3)
    dp, dv = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
    st, _ = _static(lib, dp, dv, 2 * lib.STATIC_MAX_GRID, lib.MPS_F32)  # grid above the maximum
    assert st == -8
    big = torch.zeros((lib.STATIC_MAX_PARTICLES + 1, 3), dtype=torch.float32, device="cuda")
    st, _ = _static(lib, big, big, 16, lib.MPS_F32)        # catalog above the maximum
    assert st == -8
    st, _ = _static(lib, dp.cpu(), dv.cpu(), 16, lib.MPS_F32)  # host catalogs are not staged here
    assert st == -1
