"""The FP32 scatter's three forms against the oracle.

FP32 grids of N >= MPS_SCATTER_MIN_GRID with the truncated BL3 kernel choose
the scatter's form by the mean number of particles per 16^3 tile,
m = n_particles / (N/16)^3: the owner-computes form for m <=
MPS_SCATTER_GATHER_MAX_MEAN, the halo form for m <= MPS_SCATTER_HALO_MAX_MEAN,
the atomic form above (and on smaller grids).  Each
case states its form, and every switch point is checked from both sides on
the same grid: the assigned grids against oracle.assign (max |error| / max
|grid| per field < 2e-6, the FP32 assignment bound of test_gpu_parity), the
spectra against oracle.estimate (3e-4 guarded), single catalogs and the
multi-catalog launches of mps_estimate_batch (one per form and record
layout).  Inputs: seeded uniform catalogs with Gaussian velocities
(synth.catalogs) with particles placed on tile faces, edges and corners and
at the periodic wrap, and clustered catalogs whose particles sit in a few
tiles, assigned on a plan whose grid still holds a dense catalog's values."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import compare_spectra
from synth import catalogs

pytestmark = pytest.mark.gpu

BOX = 1000.0
GRID_TOL = 2e-6


@pytest.fixture(scope="module")
def mps():
    import paper_2005_06170_amd as m
    return m


def _dev(*arrays):
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def _form(n, npart):
    from paper_2005_06170_amd import _lib
    tiles = (n // 16) ** 3
    if n < _lib.SCATTER_MIN_GRID:
        return "atomic"
    if npart <= _lib.SCATTER_GATHER_MAX_MEAN * tiles:
        return "owner-computes"
    return "halo" if npart <= _lib.SCATTER_HALO_MAX_MEAN * tiles else "atomic"


def _edge_particles(pos, n):
    """Overwrite the first particles with positions on tile boundaries (16
    cells), at x = 0 and x = L, and just inside the box edges."""
    h = BOX / n
    t = 16 * h
    special = np.array([
        [0.0, 0.0, 0.0], [BOX, BOX, BOX], [-1e-4, BOX * 0.5, BOX - 1e-4],
        [t, t, t], [t - 1e-4, t, t + 1e-4], [2 * t, 3 * t - 1e-4, BOX - t],
        [t - 3 * h, t + 2 * h, t + 2.5 * h], [BOX - 2.5 * h, 0.5 * h, t - 3.5 * h],
    ], dtype=np.float32)
    pos[: len(special)] = special
    return pos


def _assign_want(pos, vel, w, n, bulk):
    w64 = np.ones(pos.shape[0]) if w is None else w.astype(np.float64)
    v64 = vel.astype(np.float64)
    if bulk:
        v64 = v64 - (w64[:, None] * v64).sum(0) / w64.sum()
    q = np.stack([w64, w64 * v64[:, 0], w64 * v64[:, 1], w64 * v64[:, 2]])
    return oracle.assign(pos, q, BOX, n)


def _grid_err(g, want):
    scale = np.abs(want).max(axis=(1, 2, 3), keepdims=True)
    return float(np.max(np.abs(g - want) / scale))


# (N, particles, weights, form): each switch point from both sides
ASSIGN_CASES = [
    (128, 5_000, True, "owner-computes"), (128, 196_000, False, "owner-computes"),
    (128, 197_500, True, "halo"), (128, 1_048_000, False, "halo"), (128, 1_049_000, True, "atomic"),
    (64, 3_000, False, "atomic"), (64, 60_000, True, "atomic"),
]


@pytest.mark.parametrize("n,npart,weights,form", ASSIGN_CASES)
def test_assign_each_side_of_each_switch(mps, n, npart, weights, form):
    assert _form(n, npart) == form
    print(f"assign N={n} {npart} particles weights={weights}: {form}", flush=True)
    pos, vel, w = catalogs.uniform_gaussian(npart, BOX, 300.0, seed=catalogs.seed_for(5, n + npart),
                                            with_weights=True)
    pos = _edge_particles(pos, n)
    w = w if weights else None
    plan = mps.Plan(n, "f32")
    g = plan.assign(*_dev(pos, vel, w), box=BOX).cpu().numpy().astype(np.float64)
    err = _grid_err(g, _assign_want(pos, vel, w, n, False))
    print(f"  max grid error / max |grid|: {err:.2e}", flush=True)
    assert err < GRID_TOL, (form, err)


@pytest.mark.parametrize("npart", [30_000, 300_000])
def test_assign_bulk_flow_grids(mps, npart):
    """The assign diagnostic's w (v - v_b) grids (owner-computes and halo forms)."""
    n = 128
    pos, vel, w = catalogs.uniform_gaussian(npart, BOX, 300.0, seed=catalogs.seed_for(5, 7), with_weights=True)
    vel = (vel.astype(np.float64) + np.array([400.0, -250.0, 120.0])).astype(np.float32)
    plan = mps.Plan(n, "f32")
    g = plan.assign(*_dev(pos, vel, w), box=BOX, bulk_flow=True).cpu().numpy().astype(np.float64)
    err = _grid_err(g, _assign_want(pos, vel, w, n, True))
    print(f"bulk-flow grids ({_form(n, npart)}): max error / max |grid| {err:.2e}", flush=True)
    assert err < GRID_TOL, err


@pytest.mark.parametrize("n_cluster,n_wrap,form", [(20_000, 5_000, "owner-computes"), (200_000, 50_000, "halo")])
def test_clustered_catalog_and_stale_grid(mps, n_cluster, n_wrap, form):
    """A few tiles hold all the particles (a Gaussian clump around one tile
    corner, a uniform block straddling the periodic wrap), most tiles and
    their neighbours are empty, and the plan's grid still holds a dense
    catalog's values: every cell must be written, zeros included."""
    n = 128
    plan = mps.Plan(n, "f32")
    dpos, dvel = catalogs.uniform_gaussian(1_200_000, BOX, 300.0, seed=catalogs.seed_for(5, 11))
    assert _form(n, dpos.shape[0]) == "atomic"
    dense = plan.assign(*_dev(dpos, dvel, None), box=BOX).cpu().numpy()
    assert np.count_nonzero(dense) > 0.99 * dense.size
    rng = np.random.default_rng(catalogs.seed_for(5, 12))
    t = 16 * BOX / n
    a = rng.normal(loc=[t, 2 * t, 3 * t], scale=0.15 * t, size=(n_cluster, 3))
    b = rng.uniform(-0.5 * t, 0.5 * t, size=(n_wrap, 3))  # straddles x, y, z = 0 = L
    pos = np.mod(np.concatenate([a, b]), BOX).astype(np.float32)
    vel = rng.normal(0.0, 300.0, size=pos.shape).astype(np.float32)
    assert _form(n, pos.shape[0]) == form
    g = plan.assign(*_dev(pos, vel, None), box=BOX).cpu().numpy().astype(np.float64)
    want = _assign_want(pos, vel, None, n, False)
    # The fixed-point unit of a tile follows a bound on sum_p |q_p| |phi|;
    # in the clump the momentum fields cancel (random velocities, up to ~10^4
    # deposits per cell), so their half-unit roundings add up to several
    # 1e-6 of the largest |grid| in any form.  Measured against the grid of
    # |q| (the scale the unit follows) the bound is that of uniform
    # catalogs, with room for the sqrt(10^4) growth of the summed roundings.
    v64 = vel.astype(np.float64)
    q_abs = np.stack([np.ones(len(pos)), np.abs(v64[:, 0]), np.abs(v64[:, 1]), np.abs(v64[:, 2])])
    scale = np.abs(oracle.assign(pos, q_abs, BOX, n)).max(axis=(1, 2, 3), keepdims=True)
    err = float(np.max(np.abs(g - want) / scale))
    print(f"clustered ({form}): max grid error / max |q| grid {err:.2e}", flush=True)
    assert err < 4e-6, err
    assert np.all(g[:, want[0] == 0.0] == 0.0)


@pytest.mark.parametrize("n,npart", [(64, 50_000), (128, 30_000), (128, 300_000), (128, 1_100_000)])
def test_estimate_matches_oracle(mps, n, npart):
    form = _form(n, npart)
    pos, vel, w = catalogs.uniform_gaussian(npart, BOX, 300.0, seed=catalogs.seed_for(5, 3 * n + npart),
                                            with_weights=True)
    pos = _edge_particles(pos, n)
    o = oracle.estimate(pos, vel, w, box=BOX, n_grid=n, haf=50.0, flags=oracle.FLAG_BULKFLOW_SUBTRACT)
    g = mps.Plan(n, "f32").estimate(*_dev(pos, vel, w), box=BOX, haf=50.0, bulk_flow=True)
    compare_spectra(g, o, 3e-4, f"N={n} {npart} particles ({form})")


def test_batch_groups_match_oracle(mps):
    """mps_estimate_batch over catalogs of every form, with and without
    weights (six multi-catalog launches), and an FP64 one, twice in a row,
    against the oracle."""
    specs = [(128, 5_000, False, "f32"), (128, 100_000, True, "f32"), (128, 200_000, False, "f32"),
             (128, 300_000, True, "f32"), (128, 140_000, True, "f32"), (64, 40_000, False, "f32"),
             (64, 20_000, True, "f32"), (128, 2_000, True, "f32"), (64, 30_000, False, "f64")]
    plans, args, wants, forms = [], [], [], []
    for i, (n, npart, weights, prec) in enumerate(specs):
        pos, vel, w = catalogs.uniform_gaussian(npart, BOX, 300.0, seed=catalogs.seed_for(5, 50 + i),
                                                with_weights=True)
        w = w if weights else None
        plans.append(mps.Plan(n, prec))
        dp, dv, dw = _dev(pos, vel, w)
        args.append(dict(pos=dp, vel=dv, weight=dw, box=BOX, haf=50.0))
        wants.append(oracle.estimate(pos, vel, w, box=BOX, n_grid=n, haf=50.0))
        forms.append((_form(n, npart) if prec == "f32" else "f64", weights))
    assert set(forms) == {(f, w) for f in ("owner-computes", "halo", "atomic") for w in (False, True)} | {("f64", False)}
    for rep in range(2):
        outs = mps.estimate_batch(plans, args)
        for (n, npart, weights, prec), g, o, f in zip(specs, outs, wants, forms):
            compare_spectra(g, o, 3e-4 if prec == "f32" else 1e-5, f"batch {rep} N={n} {npart} {f}")


def test_batch_of_many_catalogs_matches_single_estimates(mps):
    """70 catalogs in one mps_estimate_batch call (more descriptors than the
    batch workspace's first allocation holds, spread over five groups): each
    result equals the catalog's own mps_estimate.  The owner-computes and
    halo forms assign in a fixed order, so only the FP64 shell sums (LDS
    atomics) may differ, by rounding: 1e-10 guarded; the atomic form's FP32
    grid atomics add in any order: 1e-4 guarded."""
    rng = np.random.default_rng(catalogs.seed_for(5, 90))
    plans, args, forms = [], [], []
    for i in range(70):
        n = 128 if i % 5 else 64
        npart = int(rng.choice([2_000, 20_000, 150_000, 400_000])) if n == 128 else 30_000
        pos, vel, w = catalogs.uniform_gaussian(npart, BOX, 300.0, seed=catalogs.seed_for(5, 200 + i),
                                                with_weights=True)
        plans.append(mps.Plan(n, "f32"))
        dp, dv, dw = _dev(pos, vel, w if i % 3 == 0 else None)
        args.append(dict(pos=dp, vel=dv, weight=dw, box=BOX, haf=50.0))
        forms.append(_form(n, npart))
    assert len({(f, a["weight"] is not None) for f, a in zip(forms, args)}) >= 5
    outs = mps.estimate_batch(plans, args)
    for i, (p, a, g, f) in enumerate(zip(plans, args, outs, forms)):
        want = p.estimate(a["pos"], a["vel"], a["weight"], box=BOX, haf=50.0)
        assert np.array_equal(g["n_modes"], want["n_modes"]), i
        ok = want["n_modes"] > 0
        for key, sn in (("p_pp", "sn_pp"), ("p_tt", "sn_tt"), ("p_dd", "sn_dd"), ("p_dt", "sn_dd")):
            e = np.abs(g[key][ok] - want[key][ok]) / (np.abs(want[key][ok]) + np.abs(want[sn][ok]))
            assert e.max() < (1e-4 if f == "atomic" else 1e-10), (i, f, key, e.max())
    for p in plans:
        p.close()


# ------------------------------------------------------------------ FP64 grids
def _form64(n, npart):
    from paper_2005_06170_amd import _lib
    if n < _lib.SCATTER_MIN_GRID:
        return "atomic"
    return "owner-computes" if npart <= _lib.SCATTER_GATHER64_MAX_MEAN * (n // 16) ** 3 else "atomic"


@pytest.mark.parametrize("n,npart,weights,form", [(128, 3_000, True, "owner-computes"),
                                                  (128, 196_000, False, "owner-computes"),
                                                  (128, 197_500, True, "atomic")])
def test_assign_fp64_each_side_of_the_switch(mps, n, npart, weights, form):
    """FP64 grids: the owner-computes form's 64-bit fixed point (a unit of
    2^-50 of the largest deposit) against oracle.assign to 1e-12 of the
    largest |grid|, the FP64 assignment bound of test_gpu_parity."""
    assert _form64(n, npart) == form
    pos, vel, w = catalogs.uniform_gaussian(npart, BOX, 300.0, seed=catalogs.seed_for(5, 400 + npart),
                                            with_weights=True)
    pos = _edge_particles(pos, n)
    w = w if weights else None
    g = mps.Plan(n, "f64").assign(*_dev(pos, vel, w), box=BOX).cpu().numpy()
    err = _grid_err(g, _assign_want(pos, vel, w, n, False))
    print(f"f64 assign N={n} {npart} ({form}): {err:.2e}", flush=True)
    assert err < 1e-12, (form, err)


def test_fp64_clustered_stale_grid_and_estimate(mps):
    """FP64 owner-computes form on a clustered catalog over a stale grid:
    every cell written (exact zeros where the oracle has none), the grids
    within 1e-11 of the largest |q| grid (the sum of ~10^4 roundings of 2^-51
    of the largest deposit), and the spectra against oracle.estimate."""
    n = 128
    plan = mps.Plan(n, "f64")
    dpos, dvel = catalogs.uniform_gaussian(1_200_000, BOX, 300.0, seed=catalogs.seed_for(5, 411))
    assert _form64(n, dpos.shape[0]) == "atomic"
    plan.assign(*_dev(dpos, dvel, None), box=BOX)
    rng = np.random.default_rng(catalogs.seed_for(5, 412))
    t = 16 * BOX / n
    a = rng.normal(loc=[t, 2 * t, 3 * t], scale=0.15 * t, size=(20_000, 3))
    b = rng.uniform(-0.5 * t, 0.5 * t, size=(5_000, 3))
    pos = np.mod(np.concatenate([a, b]), BOX).astype(np.float32)
    vel = rng.normal(0.0, 300.0, size=pos.shape).astype(np.float32)
    assert _form64(n, pos.shape[0]) == "owner-computes"
    g = plan.assign(*_dev(pos, vel, None), box=BOX).cpu().numpy()
    want = _assign_want(pos, vel, None, n, False)
    v64 = vel.astype(np.float64)
    q_abs = np.stack([np.ones(len(pos)), np.abs(v64[:, 0]), np.abs(v64[:, 1]), np.abs(v64[:, 2])])
    scale = np.abs(oracle.assign(pos, q_abs, BOX, n)).max(axis=(1, 2, 3), keepdims=True)
    err = float(np.max(np.abs(g - want) / scale))
    print(f"f64 clustered: {err:.2e}", flush=True)
    assert err < 1e-11, err
    assert np.all(g[:, want[0] == 0.0] == 0.0)
    o = oracle.estimate(pos, vel, box=BOX, n_grid=n, haf=50.0, flags=oracle.FLAG_BULKFLOW_SUBTRACT)
    got = plan.estimate(*_dev(pos, vel, None), box=BOX, haf=50.0, bulk_flow=True)
    compare_spectra(got, o, 1e-5, "f64 clustered estimate (owner-computes)")
