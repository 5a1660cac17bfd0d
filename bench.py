#!/usr/bin/env python3
"""Benchmark: catalogs/s of the momentum power spectrum estimator on one MI355X.

Workload: a 512^3-particle Zel'dovich catalog (lattice displaced by a Gaussian
field with P(k) = A k^-1.5 exp(-k/0.5), rms displacement 8 Mpc/h, v = 50 Psi)
in a 1000 Mpc/h box, estimated on a 512^3 grid: moments, tile sort, BL3
assignment, three FFT passes, fused deconvolution/shot-noise/binning of
P_pp, P_theta-theta, P_delta-theta and P_dd into 32 linear bins, finalize.
One step = one full estimate with the catalog already resident in HBM.

`value` is the FP32-grid path's catalogs/s; the plain FP64-grid path is timed
beside it (`fp64`).  Per-stage device times come from HIP events recorded on
the stream the stages run on.  The CPU oracle is timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# The FP32 scatter is bound by the LDS atomic unit, not HBM.  Each 64-bit
# ds_add_u64 lane carries two 32-bit fixed-point deposits; the LDS pipe
# accepts one 64-lane instruction per 4 clocks per CU (16 lanes/clk/CU), so
# the peak is 256 CUs x 16 lanes x 2 deposits x 2.4 GHz.  The probe's
# measured ds_add_u64 ceiling (9.44 lanes/clk/CU) is reported beside it.
LDS_DEPOSIT_PEAK = 256 * 16 * 2 * 2.4e9
LDS_DEPOSIT_PROBE = 256 * 9.44 * 2 * 2.4e9
DEPOSITS_PER_PARTICLE = 216 * 4
# HBM bytes per dispatch of the 512^3 scatter as measured by rocprofv3
# (FETCH_SIZE and WRITE_SIZE, one counter per run, calibrated by a 1 GiB
# device copy), with the SHA-256 (first 16 hex digits) of the kernel source
# the counters were taken on.  Reported only while that source is unchanged.
SCATTER_TRAFFIC = {"bytes": 3.505e9 + 8.179e9, "read_bytes": 3.505e9, "write_bytes": 8.179e9,
                   "source": "paper_2005_06170_amd/csrc/particles.hip", "source_sha16": "8b2dc287af87a091",
                   "profile": "profiles/estimate_512_f32_hbm_traffic.md"}


def _sha16(path):
    import hashlib
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def scatter_traffic():
    """The measured traffic with its provenance, or None when the kernel
    source has changed since the counters were taken."""
    t = SCATTER_TRAFFIC
    if t["source_sha16"] is None or _sha16(t["source"]) != t["source_sha16"]:
        return None
    return dict(t)
N_GRID = 512
N_LAT = 512
BOX = 1000.0
HAF = 50.0
RMS = 8.0


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(n_grid, n_part, real):
    """HBM bytes each stage must move at minimum (records in, grids out)."""
    n3 = n_grid ** 3
    grid = 4 * n3 * real                     # four real (or N/2-complex) grids
    rec = 24                                 # sorted record of an unweighted catalog (x, y, z, vx, vy, vz)
    inp = 24                                 # float32 pos + vel
    half = n_grid // 2
    # x pass reads only (ky, kz-block) items that intersect |n| < N/2
    return {
        "moments+count": n_part * inp,
        "permute": n_part * (inp + rec),
        "clear": grid,
        "scatter": n_part * rec + grid,      # records in, grids out once
        "fft_z": 2 * grid,
        "fft_y": 2 * grid,
        "fft_x+bin": grid * math.pi / 4,     # pencils inside the k_N disc
    }


def time_path(mps, torch, pos, vel, prec, steps, warmup, kernel="bl3", n_mu=0):
    """Time `steps` estimates (n_mu > 0: the (k, mu_b) estimate with that many
    mu bins along the z axis)."""
    plan = mps.Plan(N_GRID, prec)
    plan.reserve(pos.shape[0])
    kw = dict(box=BOX, haf=HAF, n_bins=32, kernel=kernel)

    def run():
        if n_mu:
            return plan.estimate_mu(pos, vel, n_mu=n_mu, axis=(0.0, 0.0, 1.0), **kw)
        return plan.estimate(pos, vel, **kw)

    for _ in range(warmup):
        run()
    plan.set_timing(True)
    stages = []
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        out = run()
        lat.append(time.perf_counter() - t1)
        stages.append(plan.stage_times())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.set_timing(False)
    plan.close()
    avg = {k: float(np.mean([s[k] for s in stages])) for k in stages[0]}
    return wall, np.array(lat), avg, out


def time_subcubes(mps, torch, pos, vel, prec, steps, warmup):
    """The sub-sample workload: the catalog cut into 4^3 cubes of 250 Mpc/h,
    each estimated on a 128^3 grid (the spacing of the 512^3 grid)."""
    plan = mps.Plan(N_GRID // 4, prec)

    def run():
        return plan.estimate_subcubes(pos, vel, box=BOX, haf=HAF, n_div=4)

    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.close()
    return wall


def time_spt(mps, n_k=1024, n_table=256, reps=5):
    """One-loop SPT predictions at n_k wavenumbers in [0.005, 1] h/Mpc from an
    n_table-node table of the catalogs' power law (wall clock per call,
    including the host breakpoints and the copies)."""
    tk = np.geomspace(1e-3, 4.0, n_table)
    tp = 2e3 * tk ** -1.5 * np.exp(-tk / 0.5)
    ks = np.geomspace(0.005, 1.0, n_k)
    mps.spt_one_loop(ks, tk, tp)
    t0 = time.perf_counter()
    for _ in range(reps):
        mps.spt_one_loop(ks, tk, tp)
    dt = (time.perf_counter() - t0) / reps
    return {"n_k": n_k, "n_table": n_table, "ms_per_call": 1e3 * dt, "predictions_per_s": n_k / dt}


def batch_workload(mps, torch, seed_config=4, n_cat=64, reps=5, sequential=True):
    """The batched form: 64 catalogs of uneven sizes (particle counts
    log-uniform in [1e5, 4e6], grids from {64, 128, 256}^3, boxes from
    {250, 500, 1000} Mpc/h, half uniform with Gaussian velocities, half
    Zel'dovich power-law lattices with rms displacement 3 Mpc/h x L/1000),
    FP32 grids.  Times one mps_estimate_batch call over all 64 (after a
    warm-up call, mean of `reps`) against 64 mps_estimate calls in sequence
    (plans created beforehand in both; sequential=False skips the latter)."""
    from synth import catalogs
    rng = np.random.default_rng(catalogs.seed_for(seed_config))
    cats = []
    for i in range(n_cat):
        n = int(round(np.exp(rng.uniform(np.log(1e5), np.log(4e6)))))
        grid = int(rng.choice([64, 128, 256]))
        box = float(rng.choice([250.0, 500.0, 1000.0]))
        if i % 2 == 0:
            pos, vel = catalogs.uniform_gaussian(n, box, 300.0, seed=catalogs.seed_for(seed_config, 100 + i))
        else:
            nl = max(2, int(round(n ** (1.0 / 3.0))))
            pos, vel = catalogs.zeldovich(nl, box, 3.0 * box / 1000.0, haf=HAF,
                                          seed=catalogs.seed_for(seed_config, 100 + i))
        cats.append(dict(pos=torch.from_numpy(pos).cuda(), vel=torch.from_numpy(vel).cuda(),
                         box=box, haf=HAF, grid=grid))
    plans = [mps.Plan(c["grid"], "f32") for c in cats]
    for p, c in zip(plans, cats):
        p.reserve(c["pos"].shape[0])
    args = [dict(pos=c["pos"], vel=c["vel"], box=c["box"], haf=c["haf"]) for c in cats]
    mps.estimate_batch(plans, args)  # warm-up (tables, bins)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mps.estimate_batch(plans, args)
    t_batch = (time.perf_counter() - t0) / reps
    t_seq = float("nan")
    if sequential:
        t0 = time.perf_counter()
        for _ in range(reps):
            for p, a in zip(plans, args):
                p.estimate(a["pos"], a["vel"], box=a["box"], haf=a["haf"])
        t_seq = (time.perf_counter() - t0) / reps
    for p in plans:
        p.close()
    n_part = sum(int(c["pos"].shape[0]) for c in cats)
    return {"catalogs": n_cat, "particles": n_part, "batch_ms": 1e3 * t_batch, "sequential_ms": 1e3 * t_seq,
            "batch_catalogs_per_s": n_cat / t_batch, "sequential_catalogs_per_s": n_cat / t_seq}


def resolution_study(mps, pos, vel, n_lo=N_GRID // 2):
    """The aliasing check of Sec. 2.4.3 on the synthetic catalog: estimates on
    N^3 and (2N)^3 grids in the same k bins (32 linear bins up to the k_N of
    the N^3 grid), FP32.  Per kernel and spectrum: the lower edge (in units
    of k_N) of the first bin where |P_N / P_2N - 1| exceeds 1 %, and the
    largest deviation below 0.5 k_N and 0.7 k_N."""
    kn = math.pi * n_lo / BOX
    edges = kn * np.arange(33) / 32
    out = {}
    for kernel in ("bl3", "bl3q", "pqs", "ngp"):
        res = []
        for n in (n_lo, 2 * n_lo):
            plan = mps.Plan(n, "f32")
            res.append(plan.estimate(pos, vel, box=BOX, haf=HAF, k_edges=edges, kernel=kernel))
            plan.close()
        lo, hi = res
        out[kernel] = {}
        for key in ("p_pp", "p_tt", "p_dt", "p_dd"):
            with np.errstate(invalid="ignore", divide="ignore"):
                dev = np.abs(lo[key] / hi[key] - 1.0)
            kc = lo["k_mean"] / kn
            ok = np.isfinite(dev)
            bad = np.nonzero(ok & (dev > 0.01))[0]
            out[kernel][key] = {
                "k_over_kN_1pct": float(edges[bad[0]] / kn) if bad.size else None,
                "max_dev_below_0.5kN": float(np.max(dev[ok & (kc < 0.5)])),
                "max_dev_below_0.7kN": float(np.max(dev[ok & (kc < 0.7)]))}
        _log(f"resolution study {kernel}: {out[kernel]}")
    return {"grids": [n_lo, 2 * n_lo], "precision": "f32", "k_N": kn, "by_kernel": out}


def cpu_baseline():
    """The oracle on 1/8 of the workload, stage by stage: a 256^3-particle
    Zel'dovich catalog of the same construction on a 256^3 grid, 8x fewer
    particles and cells.  The assignment runs the oracle's chunked form
    (oracle/large.py) on a fork pool of one worker per host thread (at most
    16, the host share of one GPU), the FFT on as many threads; the moments
    and the per-mode and binning steps are single-threaded numpy.  Every
    stage scales linearly with particles or cells except the FFT (N log N:
    x8 x 9/8).  Runs before anything touches the GPU, so that the pool forks
    a process without GPU state."""
    import multiprocessing as mp

    import scipy.fft

    from oracle import estimator as E
    from oracle import large
    from synth import catalogs
    n = 256
    threads = min(16, os.cpu_count() or 1)
    pos, vel = catalogs.zeldovich(n, BOX, RMS, haf=HAF, seed=catalogs.seed_for(3, 1))
    t = {}
    t0 = time.perf_counter()
    w = np.ones(pos.shape[0])
    mom = E.moments(vel.astype(np.float64), w)
    t["moments"] = time.perf_counter() - t0
    v = vel.astype(np.float64)
    charges = np.stack([w, v[:, 0], v[:, 1], v[:, 2]])
    t0 = time.perf_counter()
    chunk = 1 << 16  # particles per pool task (a few x planes each)
    grids = large.assign_chunked(pos, charges, BOX, n, chunk=chunk, workers=threads)
    t["assign"] = time.perf_counter() - t0
    del charges
    t0 = time.perf_counter()
    F = scipy.fft.fftn(grids, axes=(1, 2, 3), workers=threads)
    t["fft"] = time.perf_counter() - t0
    del grids
    t0 = time.perf_counter()
    q = E.mode_quantities(F, mom, BOX, n, HAF)
    E.bin_modes(q, BOX, n, n_bins=32)
    t["per_mode_and_bin"] = time.perf_counter() - t0
    fft_scale = 8.0 * math.log(512) / math.log(256)
    scaled = {k: val * (fft_scale if k == "fft" else 8.0) for k, val in t.items()}
    total = sum(scaled.values())
    return {"value": 1.0 / total, "unit": "catalogs/s", "cores": threads, "kind": "oracle",
            "sample": (f"oracle stages on a 256^3-particle Zel'dovich catalog on a 256^3 grid (1/8 of the "
                       f"particles and cells), scaled x8 (FFT x{fft_scale:.1f}); the assignment on {threads} "
                       f"fork-pool workers, the FFT on {threads} threads, the moments and per-mode steps on one"),
            "stage_s_sample": t, "stage_s_scaled": scaled, "start_method": mp.get_start_method(allow_none=True),
            "threads_by_stage": {"moments": 1, "assign": threads, "fft": threads, "per_mode_and_bin": 1}}


def reference_errors(out, pos_np, vel_np):
    """Per-bin guarded error |dP| / (|P_orc| + SN) of one estimate of the
    benchmark catalog against the oracle's reference spectra of it
    (tests/golden/zeldovich512_rms8.json), and whether the catalog is the
    one the reference was computed for."""
    path = os.path.join(ROOT, "tests", "golden", "zeldovich512_rms8.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        var = json.load(f)["variants"]["as_generated"]
    ref = {k: np.array([np.nan if x is None else x for x in v], dtype=np.float64)
           for k, v in var["spectra"].items() if isinstance(v, list) and k not in ("v_bulk",)}
    fp = var["fingerprint"]
    v64 = vel_np.astype(np.float64)
    same = (pos_np.shape[0] == fp["n_particles"]
            and np.allclose((v64.T @ v64).ravel(), fp["sum_vv"], rtol=1e-9, atol=0))
    errs = {}
    for key, sn in (("p_pp", ref["sn_pp"]), ("p_tt", ref["sn_tt"]), ("p_dd", ref["sn_dd"]),
                    ("p_dt", np.sqrt(ref["sn_dd"] * ref["sn_tt"]))):
        ok = np.isfinite(ref[key])
        e = np.abs(out[key][ok] - ref[key][ok]) / (np.abs(ref[key][ok]) + np.abs(sn[ok]))
        errs[key] = float(e.max())
    errs["n_modes_equal"] = bool(np.array_equal(out["n_modes"], ref["n_modes"].astype(np.int64)))
    errs["catalog_matches_reference"] = bool(same)
    return errs


def serving_pool(torch, catalogs):
    """Device-resident request pool: eight particle counts log-spaced over
    [1e6, 5e8]; the 1e6 and 1e7 ones are Zel'dovich lattices (100^3 and
    215^3, host-generated, lattice order), the other six uniform catalogs
    with Gaussian velocities (generated on the device, random order)."""
    sizes = [10 ** 6, 3 * 10 ** 6, 10 ** 7, 3 * 10 ** 7, 6 * 10 ** 7, 134217728, 2.5e8, 5e8]
    pool = []
    for i, n in enumerate(sizes):
        n = int(n)
        if i % 2 == 0 and n <= 3 * 10 ** 7:
            nl = int(round(n ** (1.0 / 3.0)))
            pos, vel = catalogs.zeldovich(nl, BOX, 3.0, haf=HAF, seed=catalogs.seed_for(5, i))
            p, v = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
            kind = f"zeldovich {nl}^3"
        else:
            g = torch.Generator(device="cuda").manual_seed(catalogs.seed_for(5, i))
            p = torch.rand((n, 3), generator=g, device="cuda") * BOX
            v = torch.randn((n, 3), generator=g, device="cuda") * 300.0
            kind = f"uniform {n}"
        pool.append((p.contiguous(), v.contiguous()))
        _log(f"pool catalog {i}: {kind}")
    torch.cuda.synchronize()
    return pool


def serve_stream(mps, torch, pool, prec, rate, duration, seed, inflight=3, budget_gb=200.0, label=""):
    """Poisson arrivals at `rate` requests/s for `duration` s through the
    continuous-batching server; each request draws a grid from
    {128, 256, 512, 1024}^3 and a pool catalog.  Latency is submit -> result
    on the host.  Returns catalogs/s over the whole stream (last result
    included), p50/p99 latency and the offered rate."""
    import threading
    rng = np.random.default_rng(seed)
    grids = [128, 256, 512, 1024]
    n_req = max(1, int(rate * duration))
    gaps = rng.exponential(1.0 / rate, n_req)
    picks = [(int(rng.integers(len(pool))), grids[int(rng.integers(len(grids)))]) for _ in range(n_req)]
    srv = mps.Server(hbm_budget_bytes=int(budget_gb * 2 ** 30), max_inflight=inflight,
                     small_particles=4_000_000)
    for g in grids:   # plans resident before the stream starts
        srv.wait(srv.submit(*pool[0], box=BOX, haf=HAF, n_grid=g, precision=prec), 600.0)
    lat = [None] * n_req
    done_t = [None] * n_req
    tickets = [None] * n_req
    t_sub = [None] * n_req
    ready = threading.Semaphore(0)

    def collect():
        for j in range(n_req):
            ready.acquire()
            srv.wait(tickets[j], 600.0)
            done_t[j] = time.perf_counter()
            lat[j] = done_t[j] - t_sub[j]
            if j % 100 == 0:
                _log(f"serving {label} {prec} at {rate:g}/s: {j}/{n_req} done")

    th = threading.Thread(target=collect)
    th.start()
    t0 = time.perf_counter()
    nxt = t0
    for j, (ci, g) in enumerate(picks):
        nxt += gaps[j]
        d = nxt - time.perf_counter()
        if d > 0:
            time.sleep(d)
        t_sub[j] = time.perf_counter()
        tickets[j] = srv.submit(*pool[ci], box=BOX, haf=HAF, n_grid=g, precision=prec)
        ready.release()
    th.join()
    elapsed = max(done_t) - t0
    srv.close()
    lat_ms = np.array(lat) * 1e3
    return {"catalogs_per_s": n_req / elapsed, "p50_ms": float(np.percentile(lat_ms, 50)),
            "p99_ms": float(np.percentile(lat_ms, 99)), "offered_rate": rate, "requests": n_req,
            "elapsed_s": elapsed}


P99_BOUND_MS = 1000.0


def serving_section(mps, torch, args):
    """Config 5 in the default run: the FP32 and FP64 streams at the offered
    rate, then the FP32 capacity point: the highest offered rate (tried in
    increasing order) at which p99 stays under P99_BOUND_MS and the server
    keeps up (served rate >= 95 % of offered)."""
    from synth import catalogs
    pool = serving_pool(torch, catalogs)
    out = {"pool": "8 device-resident catalogs, 1e6-5e8 particles (Zel'dovich lattices 100^3 and 215^3, "
                   "6 uniform in random order), grids uniform in {128,256,512,1024}^3",
           "p99_bound_ms": P99_BOUND_MS}
    for prec in ("f32", "f64"):
        out[prec] = serve_stream(mps, torch, pool, prec, args.rate, args.duration, catalogs.seed_for(5, 90),
                                 inflight=args.inflight, budget_gb=args.budget_gb, label="stream")
        _log(f"serving {prec}: {out[prec]}")
    cap = None
    tried = []
    for rate in args.capacity_rates:
        r = serve_stream(mps, torch, pool, "f32", rate, args.capacity_duration, catalogs.seed_for(5, 91),
                         inflight=args.inflight, budget_gb=args.budget_gb, label="capacity")
        tried.append(r)
        _log(f"capacity f32 at {rate}/s: {r}")
        if r["p99_ms"] <= P99_BOUND_MS and r["catalogs_per_s"] >= 0.95 * rate:
            cap = rate
        else:
            break
    out["capacity_f32"] = {"highest_rate_within_bound": cap, "tried": tried}
    del pool
    torch.cuda.empty_cache()
    return out


def serving(args):
    """Only the serving stream (--serving): FP32 (and FP64) at --rate."""
    import torch
    import paper_2005_06170_amd as mps
    from synth import catalogs
    pool = serving_pool(torch, catalogs)
    out = {}
    for prec in ("f32",) + (() if args.no_fp64 else ("f64",)):
        out[prec] = serve_stream(mps, torch, pool, prec, args.rate, args.duration, catalogs.seed_for(5, 90),
                                 inflight=args.inflight, budget_gb=args.budget_gb)
        _log(f"{prec}: {out[prec]}")
    if args.host_catalogs:
        # the same pool from page-locked host memory: each request's catalog
        # crosses PCIe on its worker's stream (MPS_CATALOG_HOST)
        _log("moving the pool to pinned host memory")
        pool = [(p.cpu().pin_memory(), v.cpu().pin_memory()) for p, v in pool]
        torch.cuda.empty_cache()
        out["f32_host"] = serve_stream(mps, torch, pool, "f32", args.rate, args.duration,
                                       catalogs.seed_for(5, 90), inflight=args.inflight, budget_gb=args.budget_gb)
        _log(f"f32_host: {out['f32_host']}")
    line = {"metric": "serving: catalogs/s and p50/p99 latency, Poisson arrivals", "value": out["f32"]["catalogs_per_s"],
            "unit": "catalogs/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "poisson_stream_grids_128-1024_particles_1e6-5e8", "rate": args.rate,
                       "duration_s": args.duration, "inflight": args.inflight, "budget_gb": args.budget_gb},
            "serving": out}
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the kernel, (k, mu_b) and sub-sample variants and the N vs 2N study")
    ap.add_argument("--shuffle", action="store_true",
                    help="permute particle order randomly (no spatial coherence)")
    ap.add_argument("--serving", action="store_true",
                    help="run the Poisson serving stream instead of the 512^3 benchmark")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the Poisson serving stream of the default run")
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--duration", type=float, default=20.0)
    ap.add_argument("--capacity-rates", type=float, nargs="*", default=[30.0, 40.0, 60.0],
                    help="offered rates tried in order for the FP32 capacity point")
    ap.add_argument("--capacity-duration", type=float, default=10.0)
    ap.add_argument("--inflight", type=int, default=3)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--host-catalogs", action="store_true",
                    help="serving: also run the stream with the pool in pinned host memory")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, copy 1 GiB device-to-device once (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (--gpus 1): independent catalogs need no "
              "communication between GPUs, and a sharded single catalog is not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.serving:
        serving(args)
        return

    cpu = None
    if not args.no_cpu_baseline:
        _log("timing the CPU oracle sample (before the GPU is touched)")
        cpu = cpu_baseline()
        _log(f"oracle: {cpu['value']:.5f} catalogs/s; stages {cpu['stage_s_sample']}")

    import torch
    import paper_2005_06170_amd as mps
    from synth import catalogs

    _log("generating the 512^3 Zel'dovich catalog")
    t0 = time.perf_counter()
    pos_np, vel_np = catalogs.zeldovich(N_LAT, BOX, RMS, haf=HAF, seed=catalogs.seed_for(3))
    if args.shuffle:
        perm = np.random.default_rng(1).permutation(pos_np.shape[0])
        pos_np, vel_np = pos_np[perm], vel_np[perm]
    _log(f"catalog ready in {time.perf_counter() - t0:.1f} s; uploading")
    pos = torch.from_numpy(pos_np).cuda()
    vel = torch.from_numpy(vel_np).cuda()
    n_part = pos.shape[0]

    _log("timing the FP32 path")
    wall, lat, stages, out32 = time_path(mps, torch, pos, vel, "f32", args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    _log(f"f32: {ms_step:.2f} ms/step; stages {stages}")

    fp64 = None
    precision = None
    if not args.no_fp64:
        _log("timing the FP64 path")
        steps64 = max(3, args.steps // 4)
        wall64, lat64, stages64, out64 = time_path(mps, torch, pos, vel, "f64", steps64, 1)
        fp64 = {"catalogs_per_s": steps64 / wall64, "ms_per_step": 1e3 * wall64 / steps64,
                "stage_ms": stages64}
        _log(f"f64: {1e3 * wall64 / steps64:.2f} ms/step")
        # precision study: per-bin error of each path against the oracle's
        # reference spectra of this catalog, and FP32 against FP64 grids,
        # all as |dP| / (|P| + SN)
        precision = {"f32_vs_oracle": reference_errors(out32, pos_np, vel_np),
                     "f64_vs_oracle": reference_errors(out64, pos_np, vel_np),
                     "reference": "tests/golden/zeldovich512_rms8.json"}
        _log(f"against the oracle: {precision}")
        precision["f32_vs_f64"] = {}
        for key, sn in (("p_pp", out64["sn_pp"]), ("p_tt", out64["sn_tt"]), ("p_dd", out64["sn_dd"]),
                        ("p_dt", np.sqrt(out64["sn_dd"] * out64["sn_tt"]))):
            ok = np.isfinite(out64[key])
            e = np.abs(out32[key][ok] - out64[key][ok]) / (np.abs(out64[key][ok]) + np.abs(sn[ok]))
            precision["f32_vs_f64"][key] = float(e.max())
        _log(f"FP32 vs FP64 max guarded per-bin error: {precision['f32_vs_f64']}")
    del pos_np, vel_np

    variants = None
    if not args.no_variants:
        variants = {}
        steps_v = max(3, args.steps // 4)
        for name, kw in (("bl3_exact_f32", {"kernel": "bl3_exact"}), ("bl3q_f32", {"kernel": "bl3q"}),
                         ("pqs_f32", {"kernel": "pqs"}),
                         ("ngp_f32", {"kernel": "ngp"}), ("mu16_f32", {"n_mu": 16})):
            _log(f"timing variant {name}")
            wall_v, _, stages_v, _ = time_path(mps, torch, pos, vel, "f32", steps_v, 1, **kw)
            variants[name] = {"catalogs_per_s": steps_v / wall_v, "ms_per_step": 1e3 * wall_v / steps_v,
                              "stage_ms": stages_v}
        _log("timing variant subcubes_4x4x4_128_f32")
        wall_v = time_subcubes(mps, torch, pos, vel, "f32", steps_v, 1)
        variants["subcubes_4x4x4_128_f32"] = {"catalogs_per_s": steps_v / wall_v,
                                              "ms_per_step": 1e3 * wall_v / steps_v,
                                              "sub_catalogs_per_s": 64 * steps_v / wall_v}
        _log("timing the one-loop SPT predictions")
        variants["spt_one_loop_f64"] = time_spt(mps)
        _log("timing the batched form (64 uneven catalogs)")
        variants["batch64_f32"] = batch_workload(mps, torch)
        _log(f"batch64: {variants['batch64_f32']}")

    aliasing = None
    if not args.no_variants:
        _log("resolution study (N vs 2N)")
        aliasing = resolution_study(mps, pos, vel)

    abytes = algorithmic_bytes(N_GRID, n_part, 4)
    per_stage = {}
    for k, ms in stages.items():
        entry = {"ms": ms}
        if k in abytes and ms > 0:
            gbs = abytes[k] / (ms * 1e-3) / 1e9
            entry.update({"algorithmic_GB": abytes[k] / 1e9, "GB_s": gbs, "frac_hbm": gbs / HBM_PEAK_GBS})
        per_stage[k] = entry
    dom = max((k for k in stages if k in abytes), key=lambda k: stages[k])
    if dom == "scatter":
        dep_rate = DEPOSITS_PER_PARTICLE * n_part / (stages[dom] * 1e-3)
        roofline = {"kernel": dom, "bound": "alu", "achieved": dep_rate / 1e12,
                    "peak": LDS_DEPOSIT_PEAK / 1e12, "unit": "Tdeposit/s",
                    "frac": dep_rate / LDS_DEPOSIT_PEAK,
                    "traffic": scatter_traffic() if n_part == N_LAT ** 3 else None,
                    "traffic_algorithmic": abytes[dom],
                    "probe_ceiling": LDS_DEPOSIT_PROBE / 1e12,
                    "frac_of_probe_ceiling": dep_rate / LDS_DEPOSIT_PROBE,
                    "hbm_frac": per_stage[dom].get("frac_hbm")}
    else:
        dom_gbs = abytes[dom] / (stages[dom] * 1e-3) / 1e9
        roofline = {"kernel": dom, "bound": "hbm", "achieved": dom_gbs, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS, "traffic": None}

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        _log("copied 1 GiB device-to-device (counter calibration)")

    serving_out = None
    if not args.no_serving:
        del pos, vel
        torch.cuda.empty_cache()
        _log("serving streams (config 5)")
        serving_out = serving_section(mps, torch, args)

    line = {
        "metric": "catalogs/sec (P_pp,P_\u03b8\u03b8,P_\u03b4\u03b8) at 512^3 grid, 134M particles; p50/p99 latency",
        "value": args.steps / wall,
        "unit": "catalogs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "zeldovich_512^3_particles_512^3_grid", "n_grid": N_GRID,
                   "n_particles": n_part, "box_mpc_h": BOX, "rms_disp_mpc_h": RMS, "haf": HAF,
                   "n_bins": 32, "particle_order": "shuffled" if args.shuffle else "lattice"},
        "latency_ms": ({"p50": serving_out["f32"]["p50_ms"], "p99": serving_out["f32"]["p99_ms"],
                        "source": f"serving stream, FP32, Poisson arrivals at {args.rate:g}/s"}
                       if serving_out else None),
        "estimate_latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                "p99": float(np.percentile(lat, 99) * 1e3),
                                "source": "back-to-back single estimates of the 512^3 catalog"},
        "fp64": fp64,
        "precision": precision,
        "serving": serving_out,
        "variants": variants,
        "resolution_study": aliasing,
        "stages": per_stage,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
