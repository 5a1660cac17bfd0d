"""The tile sort's forms by the catalog's order, decided on the device from
a sample of neighbouring particles.  On grids of more than 16,384 tiles a
catalog in spatial order takes wave-aggregated global atomics; one in
random order per-workgroup LDS tile histograms on 512^3 (32,768 tiles), and
on 1024^3 the two-level sort (bucket histograms, pass A to a temporary
array in the grid's memory, pass B per bucket) when the temporary records
fit the grid, else global atomics.
The same particles in both orders must give the same spectra: the FP64
path's fixed-point assignment is exact in any order, so only the FP64
moment sums and shell sums may differ by rounding (1e-12 guarded); the FP32
path on a sparse catalog (owner-computes scatter, fixed order) likewise;
the FP32 atomic scatter adds in any order (1e-5).  Inputs: seeded uniform
catalogs (synth.catalogs or torch's generator, random order), the same
catalogs ordered by cell (x slowest), and a shuffled Zel'dovich lattice."""
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


def _device_catalog(n_part, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    pos = (torch.rand((n_part, 3), generator=g, device="cuda", dtype=torch.float64) * BOX).float().contiguous()
    vel = (torch.randn((n_part, 3), generator=g, device="cuda", dtype=torch.float64) * 300.0).float().contiguous()
    return pos, vel


def _cell_order(pos, n):
    c = torch.floor(pos.double() * (n / BOX)).long() % n
    return torch.argsort((c[:, 0] * n + c[:, 1]) * n + c[:, 2], stable=True)


def test_two_level_sort_1024(mps):
    """1024^3 grid (262,144 tiles): a random-order catalog takes the
    two-level sort (buckets of 512 tiles through a temporary array in the
    grid's memory), the same particles in cell order the one-level global
    sort; owner-computes scatter (fixed order), so the spectra agree to
    rounding."""
    n = 1024
    pos, vel = _device_catalog(4_000_000, catalogs.seed_for(5, 303))
    idx = _cell_order(pos, n)
    plan = mps.Plan(n, "f32")
    a = plan.estimate(pos, vel, box=BOX, haf=50.0)
    b = plan.estimate(pos[idx].contiguous(), vel[idx].contiguous(), box=BOX, haf=50.0)
    plan.close()
    _compare(a, b, 1e-12, "f32 1024^3 4M random vs cell order")


def test_random_order_512_atomic_scatter(mps):
    """512^3 FP32 grid with 100M particles in random order (LDS tile
    histograms) against the cell-ordered catalog (global-atomic form).
    Atomic scatter (FP32 grid atomics in any order): 1e-5 guarded."""
    n = 512
    pos, vel = _device_catalog(100_000_000, catalogs.seed_for(5, 304))
    plan = mps.Plan(n, "f32")
    a = plan.estimate(pos, vel, box=BOX, haf=50.0)
    idx = _cell_order(pos, n)
    pos, vel = pos[idx].contiguous(), vel[idx].contiguous()
    del idx
    b = plan.estimate(pos, vel, box=BOX, haf=50.0)
    plan.close()
    _compare(a, b, 1e-5, "f32 512^3 100M random vs cell order")
