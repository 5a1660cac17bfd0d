"""The tile sort on a 512^3 grid (32,768 tiles of 16^3) takes one of two
forms by the catalog's order, decided on the device from a sample of
neighbouring particles: wave-aggregated global atomics for a catalog in
spatial order, per-workgroup LDS histograms for one in random order.  The
same particles in both orders must give the same spectra: the FP64 path's
fixed-point assignment is exact in any order, so only the FP64 moment sums
and shell sums may differ by rounding (1e-12 guarded); the FP32 path on a
sparse catalog (owner-computes scatter, fixed order) likewise.  Inputs:
seeded uniform catalogs (synth.catalogs, random order), and the same
catalog ordered by cell (x slowest), and a Zel'dovich lattice (spatial
order) shuffled."""
import numpy as np
import pytest
import torch

from synth import catalogs

pytestmark = pytest.mark.gpu

BOX, N = 1000.0, 512


@pytest.fixture(scope="module")
def mps():
    import paper_2005_06170_amd as m
    return m


def _by_cell(pos):
    c = np.floor(pos.astype(np.float64) * (N / BOX)).astype(np.int64) % N
    return np.lexsort((c[:, 2], c[:, 1], c[:, 0]))


def _compare(a, b, tol, label):
    ok = a["n_modes"] > 0
    assert np.array_equal(a["n_modes"], b["n_modes"])
    for key, sn in (("p_pp", "sn_pp"), ("p_tt", "sn_tt"), ("p_dd", "sn_dd"), ("p_dt", "sn_dd")):
        e = np.abs(a[key][ok] - b[key][ok]) / (np.abs(b[key][ok]) + np.abs(b[sn][ok]))
        print(f"{label} {key}: {e.max():.2e}", flush=True)
        assert e.max() < tol, (label, key, e.max())
    assert np.allclose(a["v_bulk"], b["v_bulk"], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_random_and_spatial_order_agree(mps, prec):
    pos, vel, w = catalogs.uniform_gaussian(2_000_000, BOX, 300.0, seed=catalogs.seed_for(5, 300), with_weights=True)
    order = _by_cell(pos)
    plan = mps.Plan(N, prec)
    res = {}
    for name, idx in (("random", np.arange(len(pos))), ("by cell", order)):
        dev = [torch.from_numpy(np.ascontiguousarray(a[idx])).cuda() for a in (pos, vel, w)]
        res[name] = plan.estimate(*dev, box=BOX, haf=50.0, bulk_flow=True)
    _compare(res["random"], res["by cell"], 1e-12, f"{prec} uniform 2M")


def test_shuffled_lattice_agrees(mps):
    pos, vel = catalogs.zeldovich(128, BOX, 3.0, haf=50.0, seed=catalogs.seed_for(5, 301))
    perm = np.random.default_rng(catalogs.seed_for(5, 302)).permutation(len(pos))
    plan = mps.Plan(N, "f64")
    a = plan.estimate(torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda(), box=BOX, haf=50.0)
    b = plan.estimate(torch.from_numpy(np.ascontiguousarray(pos[perm])).cuda(),
                      torch.from_numpy(np.ascontiguousarray(vel[perm])).cuda(), box=BOX, haf=50.0)
    _compare(b, a, 1e-12, "f64 lattice shuffled")
