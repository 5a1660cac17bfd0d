"""Parity at the benchmark's full size, in the launch configuration bench.py
times: a 512^3 grid with 512^3 = 134,217,728 particles (Zel'dovich lattice,
rms displacement 8 Mpc/h, L = 1000 Mpc/h).  The oracle cannot estimate this
catalog in seconds, so the checks are

* assigned grid values on sampled nodes, each summed directly over the
  particles by the oracle (FP32 and FP64 grids);
* transformed modes on sampled wave vectors, each a direct DFT of the same
  grid;
* exact mode counts per shell against a brute-force integer count;
* every binned spectrum, FP64 and FP32 grids, against the oracle's
  reference spectra of this catalog (tests/golden/zeldovich512_rms8.json,
  computed by the oracle in FP64 on the CPU; the catalog's fingerprint is
  checked first);
* the FP32 path against the FP64 path bin by bin;
* invariance of all spectra under a translation by whole cells;
* the 8M-particle plane-wave control (200^3 lattice on the 512^3 grid)
  against its closed form (Eqs. 1-4 and the divergence of Sec. 2.2).
"""
import math

import numpy as np
import pytest
import torch
from scipy.special import jv, jvp

import oracle
from gpu_common import RefSpectra, check_fingerprint, compare_spectra, guarded_rel, load_reference
from synth import catalogs

pytestmark = pytest.mark.gpu

N = 512
BOX = 1000.0
HAF = 50.0


@pytest.fixture(scope="module")
def mps():
    import paper_2005_06170_amd as m
    return m


@pytest.fixture(scope="module")
def zel512():
    print("generating the 512^3 Zel'dovich catalog", flush=True)
    pos, vel = catalogs.zeldovich(N, BOX, 8.0, haf=HAF, seed=catalogs.seed_for(3))
    return pos, vel


@pytest.fixture(scope="module")
def zel512_dev(zel512):
    pos, vel = zel512
    return torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()


def _blocks(grid0, rng):
    """Sampled nodes: 3^3 blocks at the densest and the most negative node of
    the density grid, across the periodic corner, and at a random spot."""
    n = grid0.shape[0]
    centres = [np.array(np.unravel_index(int(torch.argmax(grid0)), grid0.shape)),
               np.array(np.unravel_index(int(torch.argmin(grid0)), grid0.shape)),
               np.zeros(3, dtype=np.int64),
               rng.integers(0, n, 3)]
    off = np.stack(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1], indexing="ij"), -1).reshape(-1, 3)
    return [(c[None, :] + off) % n for c in centres]


def _near(cell, nodes, n):
    """Particles whose cell is within reach (taps -2..3) of any of the nodes
    of a block that starts at nodes[0] and is contiguous modulo n."""
    lo = nodes[0]
    keep = np.ones(cell.shape[0], dtype=bool)
    for a in range(3):
        # reach is [lo - 3, hi + 2]
        span = (nodes[:, a] - lo[a]) % n
        d = (cell[:, a] - (lo[a] - 3)) % n
        keep &= d <= span.max() + 5
    return keep


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fullsize_spectra_match_the_oracle_reference(mps, zel512, zel512_dev, prec):
    """All 32 bins of P_pp, P_tt, P_dt, P_dd and the shot terms at the
    benchmark's size against the oracle: FP64 grids within 1e-5, FP32 grids
    within 3e-4 (guarded), mode counts exact."""
    doc = load_reference("zeldovich512_rms8.json")
    var = doc["variants"]["as_generated"]
    check_fingerprint(*zel512, var["fingerprint"])
    got = mps.Plan(N, prec).estimate(*zel512_dev, box=BOX, haf=HAF, n_bins=doc["estimate"]["n_bins"])
    errs = compare_spectra(got, RefSpectra(var["spectra"]), 1e-5 if prec == "f64" else 3e-4, f"{prec} 512^3 reference")
    print(prec, "512^3 max guarded per-bin error against the oracle:", errs, flush=True)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fullsize_assignment_on_sampled_nodes(mps, zel512, zel512_dev, prec):
    pos, vel = zel512
    plan = mps.Plan(N, prec)
    plan.reserve(pos.shape[0])
    grid = plan.assign(*zel512_dev, box=BOX)
    scale = grid.abs().amax(dim=(1, 2, 3)).double().cpu().numpy()
    rng = np.random.default_rng(11)
    cell, _ = oracle.cell_and_fraction(pos, BOX, N)
    worst = 0.0
    for nodes in _blocks(grid[0], rng):
        idx = torch.from_numpy(nodes).cuda()
        got = grid[:, idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
        sub = _near(cell, nodes, N)
        v64 = vel[sub].astype(np.float64)
        q = np.stack([np.ones(v64.shape[0]), v64[:, 0], v64[:, 1], v64[:, 2]])
        want = oracle.assign_cells(pos[sub], q, BOX, N, nodes)
        err = float(np.max(np.abs(got - want) / scale[:, None]))
        print(prec, "block at", nodes[13], "particles", int(sub.sum()),
              "max error / max |grid|:", err, flush=True)
        worst = max(worst, err)
    del grid
    plan.close()
    # FP32 grids: per-cell fixed point, unit = bound / 2^31 per tile
    assert worst < (1e-12 if prec == "f64" else 2e-6), worst


def _dft_mode(g, n_vec):
    """Direct DFT of one real N^3 grid at integer wave vector n (e^{-i})."""
    n = g.shape[0]
    e = [np.exp(-2j * math.pi * n_vec[a] * np.arange(n) / n) for a in range(3)]
    return complex(e[0] @ ((g @ e[2]) @ e[1]))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fullsize_fft_on_sampled_modes(mps, zel512_dev, prec):
    plan = mps.Plan(N, prec)
    plan.reserve(zel512_dev[0].shape[0])
    grid = plan.assign(*zel512_dev, box=BOX)
    fields = {f: grid[f].double().cpu().numpy() for f in (0, 3)}
    spec = plan.fft(grid)
    modes = [(1, 0, 0), (0, 0, 1), (3, 5, 7), (-100, 37, 200), (255, -256, 13), (-7, 130, 255)]
    for f, g in fields.items():
        norm = math.sqrt(float(np.sum(g * g)))     # rms |F| over all modes
        worst = 0.0
        for m in modes:
            want = _dft_mode(g, m)
            got = complex(spec[f, m[0] % N, m[1] % N, m[2]].cpu().numpy())
            # rounding errors scale with the mode itself where it is large
            # (the long-wavelength modes of the clustered fields) and with
            # the rms elsewhere
            worst = max(worst, abs(got - want) / (norm + abs(want)))
        print(prec, "field", f, "max |dF| / (rms |F| + |F|):", worst, flush=True)
        assert worst < (1e-12 if prec == "f64" else 2e-5), (f, worst)
    del grid, spec
    plan.close()


def test_fullsize_mode_counts(mps, zel512_dev):
    res = mps.Plan(N, "f32").estimate(*zel512_dev, box=BOX, haf=HAF)
    nf = np.rint(np.fft.fftfreq(N) * N).astype(np.int64)
    n2 = (nf[:, None, None] ** 2 + nf[None, :, None] ** 2) + nf[None, None, :] ** 2
    b = oracle.default_bin_index(n2, N, 32)
    want = np.bincount(b[b >= 0], minlength=32)
    assert np.array_equal(res["n_modes"], want), (res["n_modes"], want)


def test_fullsize_fp32_matches_fp64(mps, zel512_dev):
    """The precision study at 512^3: per-bin guarded error of the FP32 path
    against the FP64 path."""
    outs = {p: mps.Plan(N, p).estimate(*zel512_dev, box=BOX, haf=HAF) for p in ("f32", "f64")}
    a, b = outs["f32"], outs["f64"]
    errs = {}
    for key, sn in (("p_pp", b["sn_pp"]), ("p_tt", b["sn_tt"]), ("p_dd", b["sn_dd"]),
                    ("p_dt", np.sqrt(b["sn_dd"] * b["sn_tt"]))):
        e = guarded_rel(a[key], b[key], sn)
        errs[key] = float(e.max())
    print("512^3 FP32 vs FP64 max guarded per-bin error:", errs, flush=True)
    assert max(errs.values()) <= 3e-4, errs


@pytest.mark.parametrize("kernel", ["pqs", "ngp"])
def test_fullsize_bspline_fp32_matches_fp64(mps, zel512_dev, kernel):
    """The comparison kernels at 512^3: FP32 grids against FP64 grids."""
    outs = {p: mps.Plan(N, p).estimate(*zel512_dev, box=BOX, haf=HAF, kernel=kernel) for p in ("f32", "f64")}
    a, b = outs["f32"], outs["f64"]
    errs = {}
    for key, sn in (("p_pp", b["sn_pp"]), ("p_tt", b["sn_tt"]), ("p_dd", b["sn_dd"]),
                    ("p_dt", np.sqrt(b["sn_dd"] * b["sn_tt"]))):
        errs[key] = float(guarded_rel(a[key], b[key], sn).max())
    print(kernel, "512^3 FP32 vs FP64 max guarded per-bin error:", errs, flush=True)
    assert max(errs.values()) <= 3e-4, errs


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fullsize_translation_by_whole_cells(mps, zel512, prec):
    """Moving every particle by whole cells leaves every spectrum unchanged.
    Positions are first rounded to multiples of 2^-14 Mpc/h, so that below
    L = 1000 < 2^10 both they and their shifts by whole cells (multiples of
    L/N = 125/64) are exact in float32."""
    pos, vel = zel512
    q = np.rint(pos.astype(np.float64) * 2.0 ** 14) / 2.0 ** 14 % BOX
    shift = np.array([7, -3, 130]) * (BOX / N)
    base = q.astype(np.float32)
    moved = ((q + shift) % BOX).astype(np.float32)
    assert np.array_equal(moved.astype(np.float64), (q + shift) % BOX)
    plan = mps.Plan(N, prec)
    v = torch.from_numpy(vel).cuda()
    r0 = plan.estimate(torch.from_numpy(base).cuda(), v, box=BOX, haf=HAF)
    r1 = plan.estimate(torch.from_numpy(moved).cuda(), v, box=BOX, haf=HAF)
    errs = {}
    for key, sn in (("p_pp", r0["sn_pp"]), ("p_tt", r0["sn_tt"]), ("p_dd", r0["sn_dd"]),
                    ("p_dt", np.sqrt(r0["sn_dd"] * r0["sn_tt"]))):
        errs[key] = float(guarded_rel(r1[key], r0[key], sn).max())
    print(prec, "translation: max guarded change", errs, flush=True)
    # u = x N / L is rounded in FP64 either way: a particle within ~1e-13 of
    # a cell edge may change cell, a change of order 1e-10 in a spectrum
    assert max(errs.values()) < (1e-8 if prec == "f64" else 3e-4), errs


def test_fullsize_subcubes(mps, zel512, zel512_dev):
    """The 64 sub-samples of the benchmark catalog: 4^3 cubes of 250 Mpc/h,
    each on a 128^3 grid (the 512^3 grid's spacing).  Particle counts per
    cube are exact; one sampled cube matches the oracle; FP32 matches FP64 on
    every cube and on the mean and spread."""
    pos, vel = zel512
    cube, local = oracle.subcubes.split(pos, BOX, 4)
    counts = np.bincount(cube, minlength=64).astype(np.float64)
    res = {}
    for prec in ("f64", "f32"):
        plan = mps.Plan(128, prec)
        res[prec] = plan.estimate_subcubes(*zel512_dev, box=BOX, haf=HAF, n_div=4)
        plan.close()
        assert np.all(res[prec]["status"] == 0)
        assert [r["n_eff"] for r in res[prec]["sub"]] == counts.tolist()
    c = 37
    sel = cube == c
    print("oracle on cube", c, "with", int(sel.sum()), "particles", flush=True)
    want = oracle.estimate(local[sel], vel[sel], box=BOX / 4, n_grid=128, haf=HAF)
    for prec in ("f64", "f32"):
        compare_spectra(res[prec]["sub"][c], want, 1e-5 if prec == "f64" else 3e-4, f"{prec} cube {c}")
    a, b = res["f32"], res["f64"]
    worst = {}
    for key, sk in (("p_pp", "sn_pp"), ("p_tt", "sn_tt"), ("p_dd", "sn_dd"), ("p_dt", None)):
        for s in range(64):
            sn = b["sub"][s][sk] if sk else np.sqrt(b["sub"][s]["sn_dd"] * b["sub"][s]["sn_tt"])
            e = float(guarded_rel(a["sub"][s][key], b["sub"][s][key], sn).max())
            worst[key] = max(worst.get(key, 0.0), e)
        sn = b["mean"][sk] if sk else np.sqrt(b["mean"]["sn_dd"] * b["mean"]["sn_tt"])
        worst[key + " mean"] = float(guarded_rel(a["mean"][key], b["mean"][key], sn).max())
        ok = np.isfinite(b["sdev"][key])
        worst[key + " sdev"] = float(np.max(np.abs(a["sdev"][key][ok] - b["sdev"][key][ok])
                                            / (np.abs(b["mean"][key][ok]) + np.abs(sn[ok]))))
    print("sub-cubes FP32 vs FP64 max guarded error:", worst, flush=True)
    assert max(worst.values()) <= 3e-4, worst


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kernel", ["bl3_exact", "bl3"])
def test_plane_wave_control_512(mps, prec, kernel):
    """200^3-particle plane wave (k0 = 2 pi 4 / L, A = 1 Mpc/h) on the 512^3
    grid.  The shell [sqrt(15.5), sqrt(16.5)] k_f holds the 6 modes with
    n^2 = 16, two of which carry the wave, so the shell mean is V (2/6) P_wave.

    With the untruncated kernel every spectrum matches the closed form: its
    window vanishes at every alias of k0 (a CPU evaluation of the transform at
    k0 gives |delta| and |p_x| within 2e-6 and 1e-8 of it).  The six-tap
    truncation leaves window tails ~1/J^2 at the aliases k0 + 2 k_N J, where
    the lattice's comb carries Bessel sidebands J_h(k_x A) of order 0.1: the
    density at k0 picks up a few per cent (3.9e-2 in |delta| by the same CPU
    evaluation) while the momentum, which has no comb, stays within 2e-4.  For
    that kernel only P_pp and P_tt are compared with the closed form."""
    m_wave, amp = 4, 1.0
    pos, vel = catalogs.plane_wave(200, BOX, amp, m_wave, HAF)
    kf = 2 * math.pi / BOX
    edges = np.array([math.sqrt(15.5) * kf, math.sqrt(16.5) * kf])   # n^2 = 16 only
    r = mps.Plan(N, prec).estimate(torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda(),
                                   box=BOX, haf=HAF, k_edges=edges, no_shotnoise=True, kernel=kernel)
    assert int(r["n_modes"][0]) == 6
    z = m_wave * kf * amp
    frac = BOX ** 3 * 2.0 / 6.0
    want = {"p_pp": (HAF * amp) ** 2 * jvp(1, z) ** 2, "p_tt": z * z * jvp(1, z) ** 2}
    if kernel == "bl3_exact":
        want.update({"p_dd": jv(1, z) ** 2, "p_dt": z * jv(1, z) * jvp(1, z)})
    errs = {k: abs(float(r[k][0]) / (frac * v) - 1) for k, v in want.items()}
    print(prec, kernel, "plane wave at 512^3: relative error", errs, flush=True)
    assert r["p_dt"][0] > 0
    tol = 1e-3 if kernel == "bl3" else (3e-5 if prec == "f64" else 1e-4)
    assert max(errs.values()) < tol, errs


@pytest.mark.parametrize("kernel", ["bl3", "bl3q"])
def test_aliasing_n_vs_2n_within_the_printed_bounds(mps, zel512_dev, kernel):
    """Sec. 2.4.3: the same catalog on 256^3 and 512^3 grids (BL3 in both
    readings of its order, FP32 as timed), 32 linear bins up to the k_N of
    the 256^3 grid, against the
    paper's bounds for its N-body sample (tests/golden/paper_claims.json):
    below 0.2 % up to 0.5 k_N, below 0.5 % up to 0.7 k_N, and no 1 %
    departure below the lowest of its per-spectrum thresholds (0.74 k_N).
    The paper qualifies its third bound (under 5 % close to k_N) with
    "generally"; on this lattice-based catalog the last bins below k_N
    depart by up to ~12 %, so that figure is printed, not asserted."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")))
    g = g["aliasing_n_vs_2n_bl3"]
    pos, vel = zel512_dev
    kn = math.pi * (N // 2) / BOX
    edges = kn * np.arange(33) / 32
    res = []
    for n in (N // 2, N):
        plan = mps.Plan(n, "f32")
        res.append(plan.estimate(pos, vel, box=BOX, haf=HAF, k_edges=edges, kernel=kernel))
        plan.close()
    lo, hi = res
    kc = lo["k_mean"] / kn
    first = min(g["one_percent_threshold_over_kN"].values())
    worst = {}
    for key in ("p_pp", "p_tt", "p_dt", "p_dd"):
        dev = np.abs(lo[key] / hi[key] - 1.0)
        ok = np.isfinite(dev)
        worst[key] = (dev[ok & (kc <= 0.5)].max(), dev[ok & (kc <= 0.7)].max(),
                      dev[ok & (kc < first)].max(), dev[ok].max())
        print(kernel, key, "max below 0.5 k_N %.2e, 0.7 k_N %.2e, %.2f k_N %.2e, k_N %.2e" % (
            worst[key][0], worst[key][1], first, worst[key][2], worst[key][3]), flush=True)
    for key, (a, b, c, _) in worst.items():
        assert a < g["max_relative_difference_at_0p5_kN"], key
        assert b < g["max_relative_difference_below_0p7_kN"], key
        assert c < 0.01, key
