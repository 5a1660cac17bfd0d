"""Batched and served estimates equal the same catalogs estimated alone,
and the oracle's spectra.

The batch entry point and the continuous-batching server run the same
kernels as mps_estimate; results may differ only by the order of the
scatter's global atomic adds (FP32 grids), far below the parity tolerance.
Five of the pool's catalogs (the ones the oracle estimates in seconds) are
also compared with oracle.estimate, in the batch and in the served mix.
"""
import threading

import numpy as np
import pytest
import torch

import oracle
from synth import catalogs
from gpu_common import RUN_TOL_F32, compare_spectra, guarded_rel

TOL = {"f64": 1e-5, "f32": 3e-4}
# pool entries small enough for the oracle
ORACLE_CHECKED = (0, 1, 3, 4, 7)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mps():
    import paper_2005_06170_amd as m
    return m


def _pool():
    """Uneven catalogs: (kind, n, grid, box, prec)."""
    specs = [("uniform", 150_000, 64, 250.0, "f32"), ("zel", 32, 128, 500.0, "f32"),
             ("uniform", 700_000, 128, 1000.0, "f32"), ("zel", 48, 64, 1000.0, "f64"),
             ("uniform", 20_000, 32, 250.0, "f64"), ("zel", 64, 256, 1000.0, "f32"),
             ("uniform", 1_000_003, 256, 500.0, "f32"), ("uniform", 5_000, 16, 100.0, "f32")]
    out = []
    for i, (kind, n, grid, box, prec) in enumerate(specs):
        if kind == "uniform":
            pos, vel = catalogs.uniform_gaussian(n, box, 300.0, seed=catalogs.seed_for(4, i))
        else:
            pos, vel = catalogs.zeldovich(n, box, 3.0 * box / 1000.0, seed=catalogs.seed_for(4, i))
        out.append(dict(pos=torch.from_numpy(pos).cuda(), vel=torch.from_numpy(vel).cuda(),
                        box=box, haf=50.0, n_bins=24, grid=grid, prec=prec, host=(pos, vel)))
    return out


@pytest.fixture(scope="module")
def pool_oracle():
    pool = _pool()
    want = {}
    for i in ORACLE_CHECKED:
        c = pool[i]
        print(f"oracle for pool catalog {i}: {c['host'][0].shape[0]} particles, {c['grid']}^3", flush=True)
        want[i] = oracle.estimate(*c["host"], box=c["box"], n_grid=c["grid"], haf=c["haf"], n_bins=c["n_bins"])
    return pool, want


def _same(a, b, tol):
    assert np.array_equal(a["n_modes"], b["n_modes"])
    for key, sn in (("p_pp", "sn_pp"), ("p_tt", "sn_tt"), ("p_dd", "sn_dd")):
        e = guarded_rel(a[key], b[key], b[sn])
        assert e.size == 0 or e.max() <= tol, (key, e.max())
    e = guarded_rel(a["p_dt"], b["p_dt"], np.sqrt(b["sn_dd"] * b["sn_tt"]))
    assert e.size == 0 or e.max() <= tol


def _alone(mps, c):
    return mps.Plan(c["grid"], c["prec"]).estimate(c["pos"], c["vel"], box=c["box"], haf=c["haf"],
                                                   n_bins=c["n_bins"])


def test_batch_equals_alone(mps, pool_oracle):
    pool, want = pool_oracle
    alone = [_alone(mps, c) for c in pool]
    plans = [mps.Plan(c["grid"], c["prec"]) for c in pool]
    cats = [dict(pos=c["pos"], vel=c["vel"], box=c["box"], haf=c["haf"], n_bins=c["n_bins"]) for c in pool]
    batch = mps.estimate_batch(plans, cats)
    for a, b, c in zip(batch, alone, pool):
        _same(a, b, RUN_TOL_F32 if c["prec"] == "f32" else 1e-12)
    for i in ORACLE_CHECKED:
        compare_spectra(batch[i], want[i], TOL[pool[i]["prec"]], f"batch catalog {i}")


def test_server_mix_equals_alone(mps, pool_oracle):
    pool, want = pool_oracle
    alone = [_alone(mps, c) for c in pool]
    srv = mps.Server(hbm_budget_bytes=24 << 30, max_inflight=3, small_particles=400_000)
    order = list(range(len(pool))) * 3
    rng = np.random.default_rng(3)
    rng.shuffle(order)
    tickets = [None] * len(order)
    errors = []

    def submit(part):
        try:
            for j in part:
                c = pool[order[j]]
                tickets[j] = srv.submit(c["pos"], c["vel"], box=c["box"], haf=c["haf"], n_grid=c["grid"],
                                        precision=c["prec"], n_bins=c["n_bins"])
        except Exception as exc:  # pragma: no cover - reported below
            errors.append(exc)

    threads = [threading.Thread(target=submit, args=(range(k, len(order), 3),)) for k in range(3)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for j, t in enumerate(tickets):
        got = srv.wait(t, timeout_s=120.0)
        c = pool[order[j]]
        _same(got, alone[order[j]], RUN_TOL_F32 if c["prec"] == "f32" else 1e-12)
        if order[j] in ORACLE_CHECKED:
            compare_spectra(got, want[order[j]], TOL[c["prec"]], f"served catalog {order[j]}")
    srv.close()


def test_server_waits_for_the_producing_stream(mps):
    """A catalog written on a side stream by work still in flight at submit
    time: the request's kernels wait for that stream (mps_submit records an
    event on it), so the result equals the estimate of the finished catalog."""
    pos, vel = catalogs.uniform_gaussian(400_000, 500.0, 300.0, seed=catalogs.seed_for(4, 50))
    src_p, src_v = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
    want = mps.Plan(64, "f32").estimate(src_p, src_v, box=500.0, haf=50.0, n_bins=16)
    srv = mps.Server(hbm_budget_bytes=4 << 30, max_inflight=2)
    side = torch.cuda.Stream()
    a = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    for rep in range(3):
        dst_p = torch.zeros_like(src_p)
        dst_v = torch.zeros_like(src_v)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            for _ in range(8):           # keep the side stream busy first
                a = torch.tanh(a @ a * 1e-3)
            dst_p.copy_(src_p)
            dst_v.copy_(src_v)
            t = srv.submit(dst_p, dst_v, box=500.0, haf=50.0, n_grid=64, n_bins=16, stream=side)
        got = srv.wait(t, timeout_s=120.0)
        torch.cuda.synchronize()
        _same(got, want, RUN_TOL_F32)
    srv.close()


def test_server_admission_errors(mps):
    from paper_2005_06170_amd._lib import MpsError
    pos, vel = catalogs.uniform_gaussian(100_000, 100.0, seed=5)
    p, v = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
    srv = mps.Server(hbm_budget_bytes=64 << 20, max_inflight=1)
    with pytest.raises(MpsError) as e:                    # 256^3 grids need > 64 MiB
        srv.submit(p, v, box=100.0, haf=50.0, n_grid=256)
    assert e.value.status == -8
    with pytest.raises(MpsError) as e:
        srv.submit(p, v, box=-1.0, haf=50.0, n_grid=32)
    assert e.value.status == -1
    t = srv.submit(p, v, box=100.0, haf=50.0, n_grid=32)  # fits
    out = srv.wait(t, timeout_s=60.0)
    assert out["n_modes"].sum() > 0
    srv.close()
