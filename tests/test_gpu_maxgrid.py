"""The largest grid a plan accepts, 1024^3 (its own FFT, fused x pass and
scatter instances in both precisions).  The oracle cannot transform a grid
this size, so the checks are exact closed forms and properties:

* the FFT of plane-wave grids: one mode of height N^3 / 2 per field (two on
  the kz = 0 plane) and nothing elsewhere;
* the Zel'dovich plane wave (200^3 lattice, k0 = 2 pi 4 / L) estimated with
  the untruncated BL3 kernel, whose window vanishes at every alias of k0:
  all four spectra against their closed forms (Bessel functions of
  z = k0 A), as at 512^3;
* exact shell mode counts against an integer count;
* the FP32 path against the FP64 path on a clustered catalog;
* the largest catalog a plan accepts, 2^31 - 1 particles (uniform, on a
  128^3 grid: 4.2M particles per 16^3 tile): N times the density shot term
  (V C(k) / (N W^2(k)) per bin for unit weights) equals that of a 10^6
  particle catalog on the same grid, so the FP64 moment sums hold all
  2^31 - 1 particles, and FP32 matches FP64.
"""
import math

import numpy as np
import pytest
import torch
from scipy.special import jv, jvp

import oracle
from gpu_common import guarded_rel
from synth import catalogs

pytestmark = pytest.mark.gpu

N = 1024
BOX = 1000.0
HAF = 50.0


@pytest.fixture(scope="module")
def mps():
    import paper_2005_06170_amd as m
    return m


def _release():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_maxgrid_fft_of_plane_waves(mps, prec):
    dt = torch.float32 if prec == "f32" else torch.float64
    waves = [(3, 0, 5), (-7, 12, 511), (0, 0, 1), (37, -200, 0)]   # the last on the kz = 0 plane
    i = torch.arange(N, device="cuda", dtype=torch.float64)
    grids = torch.empty((4, N, N, N), device="cuda", dtype=dt)
    for f, (a, b, c) in enumerate(waves):
        ph = (a * i[:, None, None] + b * i[None, :, None] + c * i[None, None, :]) % N
        grids[f] = torch.cos(ph * (2 * math.pi / N)).to(dt)
        del ph
    plan = mps.Plan(N, prec)
    spec = plan.fft(grids)
    half = N ** 3 / 2
    worst_peak, worst_rest = 0.0, 0.0
    for f, (a, b, c) in enumerate(waves):
        peaks = [(a % N, b % N, c)] + ([((-a) % N, (-b) % N, 0)] if c == 0 else [])
        for p in peaks:
            v = complex(spec[f, p[0], p[1], p[2]].cpu().numpy())
            worst_peak = max(worst_peak, abs(v - half) / half)
            spec[f, p[0], p[1], p[2]] = 0
        worst_rest = max(worst_rest, float(spec[f].abs().max()) / half)
    print(prec, "1024^3 plane-wave FFT: peak error", worst_peak, "largest other mode", worst_rest, flush=True)
    tol = 1e-12 if prec == "f64" else 2e-6
    assert worst_peak < tol and worst_rest < tol, (worst_peak, worst_rest)
    del spec, grids
    plan.close()
    _release()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_maxgrid_plane_wave_closed_form(mps, prec):
    m_wave, amp = 4, 1.0
    pos, vel = catalogs.plane_wave(200, BOX, amp, m_wave, HAF)
    kf = 2 * math.pi / BOX
    edges = np.array([math.sqrt(15.5) * kf, math.sqrt(16.5) * kf])   # n^2 = 16 only
    plan = mps.Plan(N, prec)
    r = plan.estimate(torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda(), box=BOX, haf=HAF,
                      k_edges=edges, no_shotnoise=True, kernel="bl3_exact")
    plan.close()
    _release()
    assert int(r["n_modes"][0]) == 6
    z = m_wave * kf * amp
    frac = BOX ** 3 * 2.0 / 6.0
    want = {"p_pp": (HAF * amp) ** 2 * jvp(1, z) ** 2, "p_tt": z * z * jvp(1, z) ** 2,
            "p_dd": jv(1, z) ** 2, "p_dt": z * jv(1, z) * jvp(1, z)}
    errs = {k: abs(float(r[k][0]) / (frac * v) - 1) for k, v in want.items()}
    print(prec, "plane wave at 1024^3: relative error", errs, flush=True)
    assert max(errs.values()) < (3e-5 if prec == "f64" else 1e-4), errs


@pytest.fixture(scope="module")
def clustered():
    pos, vel = catalogs.zeldovich(256, BOX, 8.0, haf=HAF, seed=catalogs.seed_for(3, 2))
    return torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()


def test_maxgrid_mode_counts(mps, clustered):
    plan = mps.Plan(N, "f32")
    res = plan.estimate(*clustered, box=BOX, haf=HAF)
    plan.close()
    _release()
    nf = np.rint(np.fft.fftfreq(N) * N).astype(np.int64)
    n2yz = nf[:, None] ** 2 + nf[None, :] ** 2
    want = np.zeros(32, dtype=np.int64)
    for nx in nf:                       # one plane at a time: 1024^3 int64 would be 8 GiB
        b = oracle.default_bin_index(n2yz + nx * nx, N, 32)
        want += np.bincount(b[b >= 0], minlength=32)
    assert np.array_equal(res["n_modes"], want), (res["n_modes"], want)


def test_maxgrid_fp32_matches_fp64(mps, clustered):
    outs = {}
    for p in ("f32", "f64"):
        plan = mps.Plan(N, p)
        outs[p] = plan.estimate(*clustered, box=BOX, haf=HAF, bulk_flow=True)
        plan.close()
        _release()
    a, b = outs["f32"], outs["f64"]
    errs = {}
    for key, sn in (("p_pp", b["sn_pp"]), ("p_tt", b["sn_tt"]), ("p_dd", b["sn_dd"]),
                    ("p_dt", np.sqrt(b["sn_dd"] * b["sn_tt"]))):
        errs[key] = float(guarded_rel(a[key], b[key], sn).max())
    print("1024^3 FP32 vs FP64 max guarded per-bin error:", errs, flush=True)
    assert max(errs.values()) <= 3e-4, errs


def test_max_particle_count(mps):
    n_part = 2 ** 31 - 1
    g = torch.Generator(device="cuda").manual_seed(catalogs.seed_for(3, 5))
    pos = torch.rand((n_part, 3), generator=g, device="cuda") * BOX
    vel = torch.randn((n_part, 3), generator=g, device="cuda") * 300.0
    n_small = 10 ** 6
    outs = {}
    for p in ("f32", "f64"):
        plan = mps.Plan(128, p)
        outs[p] = plan.estimate(pos, vel, box=BOX, haf=HAF, n_bins=16)
        if p == "f64":
            small = plan.estimate(pos[:n_small].contiguous(), vel[:n_small].contiguous(),
                                  box=BOX, haf=HAF, n_bins=16)
        plan.close()
        _release()
    del pos, vel
    _release()
    a, b = outs["f32"], outs["f64"]
    ok = b["n_modes"] > 0
    # unit weights: S_dd = W_2 / W^2 = 1 / N, so N sn_dd depends on the grid only
    for r in (a, b):
        np.testing.assert_allclose(r["sn_dd"][ok] * n_part, small["sn_dd"][ok] * n_small, rtol=1e-12)
    assert np.array_equal(a["n_modes"], b["n_modes"])
    errs = {}
    for key, sn in (("p_pp", b["sn_pp"]), ("p_tt", b["sn_tt"]), ("p_dd", b["sn_dd"]),
                    ("p_dt", np.sqrt(b["sn_dd"] * b["sn_tt"]))):
        errs[key] = float(guarded_rel(a[key], b[key], sn).max())
    print("2^31 - 1 particles on 128^3, FP32 vs FP64 max guarded per-bin error:", errs, flush=True)
    assert max(errs.values()) <= 3e-4, errs
