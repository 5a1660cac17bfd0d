"""Plain FP64 CPU oracle of the FFT momentum power spectrum estimator.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may call this module.  It shares no code, table
or constant generator with the GPU library.

What it computes (J. Pan, "Estimating power spectrum of discrete cosmic
momentum field with fast Fourier transform"):

* momentum p = (1 + delta) v (Eq. 1); Fourier estimator
  p_hat(k) = (1/N) sum_j v_j e^{i k.r_j} (Eq. 4), generalised to weights
  w_j (N -> sum w, N^2 -> (sum w)^2);
* shot noise sigma_v^2 / N of P_p (Eq. psn), the directional shot noise
  k^2 <v^2 mu^2> / ((Haf)^2 N) of P_theta (Eqs. rawPtheta, thetanoise), and
  no real-part shot noise for P_delta-theta (Eq. rawPx);
* the grid sampled through an assignment window with alias sum
  sum_J W^2(k + 2 k_N J) (Eqs. rawFFTed, rawPp);
* momentum divergence theta_p = i k.p / (Haf) (Sec. 2.2);
* bulk-flow removal v' = v - v_b, v_b = sum v / N (Sec. 3.1).

Every step is written in its most direct form: a direct 3D tap loop over the
6^3 kernel taps, a full complex FFT (scipy.fft.fftn, e^{-i k.x}), and a
per-mode estimator over the whole N^3 cube.  Readings where the paper is
silent follow these conventions:

* grid nodes sit at g * dL; u = x * (N / L) in FP64; cell floor(u) mod N;
* BL3 truncated to six taps j - f, j = -2..3 (oracle.bl3);
* deconvolution divides by W_t(k)^2 of the truncated kernel; the shot term is
  scaled by the truncated kernel's alias sum C_t(k);
* the FFT sign is e^{-i k.x}, so theta_hat = -i k.p_hat / (Haf) keeps the sign
  of Re P_delta-theta; only the real part of the cross spectrum is binned;
* bins are half-open shells [k_b, k_{b+1}); DC and |k| >= k_N are excluded;
  the default is 32 linear bins on [0, k_N) decided by an exact integer
  comparison;
* outputs are V = L^3 times the paper's volume-normalised spectra.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.fft

from . import bl3, bl3_quadratic

FLAG_BULKFLOW_SUBTRACT = 1
FLAG_NO_SHOTNOISE = 2
FLAG_NO_DECONVOLVE = 4


# ----------------------------------------------------------------- moments
def moments(vel, weight):
    """FP64 sums entering the shot-noise and bulk-flow terms.

    Returns W = sum w, W2 = sum w^2, sv = sum w v, s2v = sum w^2 v,
    s2vv = sum w^2 v v^T (Eqs. rawppnoise, thetanoise; bulk flow Sec. 3.1).
    numpy's float64 sums are pairwise.
    """
    v = np.asarray(vel, dtype=np.float64)
    w = np.asarray(weight, dtype=np.float64)
    w2 = w * w
    return {
        "W": float(np.sum(w)),
        "W2": float(np.sum(w2)),
        "sv": np.sum(w[:, None] * v, axis=0),
        "s2v": np.sum(w2[:, None] * v, axis=0),
        "s2vv": np.einsum("j,ja,jb->ab", w2, v, v),
    }


# -------------------------------------------------------------- assignment
def cell_and_fraction(pos, box: float, n_grid: int):
    """Grid coordinate u = x N / L (FP64), cell floor(u) mod N, fraction f."""
    u = np.asarray(pos, dtype=np.float64) * (n_grid / box)
    uf = np.floor(u)
    frac = u - uf
    cell = (uf - n_grid * np.floor(uf / n_grid)).astype(np.int64)
    cell = np.clip(cell, 0, n_grid - 1)
    return cell, frac


KERNELS = ("bl3", "bl3q", "bl3_exact", "ngp", "cic", "tsc", "pcs", "pqs", "bspline6",
           "bspline1", "bspline2", "bspline3", "bspline4", "bspline5")


def assign(pos, charges, box: float, n_grid: int, kernel: str = "bl3"):
    """Assign charges q[c, j] of particles j to 4 periodic grids with BL3.

    kernel "bl3" (default) is the six-tap truncated function described below;
    "bl3q" is the same six-tap assignment with the quadratic-spline reading of
    the function (oracle.bl3_quadratic); "bl3_exact" is the untruncated cubic
    function (oracle.exact_bl3); the B-spline kernels ("ngp" .. "bspline6")
    are in oracle.bspline.

    Each particle deposits q * phi(jx - fx) phi(jy - fy) phi(jz - fz) on node
    (cell + (jx, jy, jz)) mod N for every tap j in {-2..3}^3 (Eq. rawFFTed with
    the truncated BL3 window).  Returns float64 array (n_charge, N, N, N)
    indexed [c, x, y, z].
    """
    if kernel == "bl3_exact":
        from . import exact_bl3
        return exact_bl3.assign_exact(pos, charges, box, n_grid)
    from . import bspline
    if bspline.order_of(kernel):
        return bspline.assign(pos, charges, box, n_grid, bspline.order_of(kernel))
    if kernel not in ("bl3", "bl3q"):
        raise ValueError(f"unknown kernel {kernel!r}")
    fn = bl3 if kernel == "bl3" else bl3_quadratic
    charges = np.atleast_2d(np.asarray(charges, dtype=np.float64))
    cell, frac = cell_and_fraction(pos, box, n_grid)
    wts = [fn.tap_weights(frac[:, a]) for a in range(3)]   # (6, n) each
    n = n_grid
    grids = np.zeros((charges.shape[0], n * n * n))
    for ix, jx in enumerate(bl3.TAPS):
        gx = (cell[:, 0] + jx) % n
        for iy, jy in enumerate(bl3.TAPS):
            gy = (cell[:, 1] + jy) % n
            wxy = wts[0][ix] * wts[1][iy]
            for iz, jz in enumerate(bl3.TAPS):
                gz = (cell[:, 2] + jz) % n
                flat = (gx * n + gy) * n + gz
                wxyz = wxy * wts[2][iz]
                for c in range(charges.shape[0]):
                    grids[c] += np.bincount(flat, weights=charges[c] * wxyz,
                                            minlength=n ** 3)
    return grids.reshape(charges.shape[0], n, n, n)


# -------------------------------------------------------------- binning
def assign_cells(pos, charges, box: float, n_grid: int, cells):
    """Assigned grid values at the listed nodes only, from the definition.

    G_c(g) = sum_p q_{c,p} phi_t(g_x - u_x) phi_t(g_y - u_y) phi_t(g_z - u_z)
    with u = x N / L, the separation taken periodically and phi_t the BL3
    function on its support (-3, 3] (Eq. rawFFTed with the BL3 window of
    Sec. 2.4.1).  Each node is a direct sum over the particles, with no tap
    decomposition; `cells` is an (m, 3) integer array; returns (n_charge, m).
    """
    charges = np.atleast_2d(np.asarray(charges, dtype=np.float64))
    cells = np.atleast_2d(np.asarray(cells, dtype=np.int64))
    cell, frac = cell_and_fraction(pos, box, n_grid)
    out = np.zeros((charges.shape[0], cells.shape[0]))
    half = n_grid // 2
    for i, g in enumerate(cells):
        # integer part of g - u, wrapped to [-N/2, N/2); g - u = d - f
        d = (g[None, :] - cell + half) % n_grid - half
        near = np.all((d >= -2) & (d <= 3), axis=1)
        if not near.any():
            continue
        sep = d[near].astype(np.float64) - frac[near]
        phi3 = (bl3.phi_trunc(sep[:, 0]) * bl3.phi_trunc(sep[:, 1])
                * bl3.phi_trunc(sep[:, 2]))
        out[:, i] = charges[:, near] @ phi3
    return out


def default_bin_index(n2, n_grid: int, n_bins: int = 32):
    """Linear bins of width k_N / n_bins on [0, k_N) by exact integers.

    Mode with integer |n|^2 = n2 lies in bin b iff
    (b * N/2)^2 <= n_bins^2 * n2 < ((b+1) * N/2)^2.
    Returns -1 for DC and for |k| >= k_N.
    """
    n2 = np.asarray(n2, dtype=np.int64)
    half = n_grid // 2
    scaled = n_bins * n_bins * n2
    b = np.floor(np.sqrt(scaled.astype(np.float64)) / half).astype(np.int64)
    # repair the float estimate so that (b h)^2 <= scaled < ((b+1) h)^2 exactly
    b = np.where((b * half) ** 2 > scaled, b - 1, b)
    b = np.where(((b + 1) * half) ** 2 <= scaled, b + 1, b)
    valid = (n2 > 0) & (n2 < half * half) & (b < n_bins)
    return np.where(valid, b, -1)


def edge_thresholds(k_edges, box: float):
    """FP64 thresholds t_b = (k_b / k_f)^2 compared with the integer |n|^2."""
    kf = 2.0 * math.pi / box
    e = np.asarray(k_edges, dtype=np.float64)
    return (e / kf) * (e / kf)


def edges_bin_index(n2, thresholds, n_grid: int):
    """Bin b iff t_b <= n2 < t_{b+1}; DC and n2 >= (N/2)^2 excluded (-1)."""
    n2 = np.asarray(n2, dtype=np.int64)
    half = n_grid // 2
    x = n2.astype(np.float64)
    b = np.searchsorted(thresholds, x, side="right") - 1
    nb = len(thresholds) - 1
    valid = (n2 > 0) & (n2 < half * half) & (b >= 0) & (b < nb)
    return np.where(valid, b, -1)


# -------------------------------------------------------------- estimator
@dataclass
class Spectra:
    k_edges: np.ndarray
    k_mean: np.ndarray
    p_pp: np.ndarray
    p_tt: np.ndarray
    p_dt: np.ndarray
    p_dd: np.ndarray
    sn_pp: np.ndarray
    sn_tt: np.ndarray
    sn_dd: np.ndarray
    n_modes: np.ndarray
    v_bulk: np.ndarray
    sigma_v2: float
    n_eff: float
    extra: dict = field(default_factory=dict)


def _integer_freqs(n_grid: int):
    return np.rint(np.fft.fftfreq(n_grid) * n_grid).astype(np.int64)


def fourier_fields(pos, vel, weight, box, n_grid, bulk_flow=False, kernel="bl3"):
    """Moments and full complex FFTs of the four assigned fields.

    Returns (mom, mom_used, F) with F[c] = FFT of the grid of charge c in
    (w, w v_x, w v_y, w v_z), using v - v_b when bulk_flow is set (the
    regridded field p' = p - (1 + delta) v_b of Sec. 3.1).
    """
    pos = np.asarray(pos)
    vel = np.asarray(vel, dtype=np.float64)
    n_p = pos.shape[0]
    w = (np.ones(n_p) if weight is None
         else np.asarray(weight, dtype=np.float64))
    mom = moments(vel, w)
    v_used = vel
    if bulk_flow:
        v_bulk = mom["sv"] / mom["W"]
        v_used = vel - v_bulk[None, :]
    mom_used = moments(v_used, w)
    charges = np.stack([w, w * v_used[:, 0], w * v_used[:, 1], w * v_used[:, 2]])
    grids = assign(pos, charges, box, n_grid, kernel)
    F = scipy.fft.fftn(grids, axes=(1, 2, 3), workers=-1)
    return mom, mom_used, F


def axis_tables(n_grid: int, kernel: str = "bl3"):
    """Per-axis window W(w)^2 and alias sum C(w) at w = 2 pi n / N."""
    nf = _integer_freqs(n_grid)
    omega = 2.0 * math.pi * nf / n_grid
    if kernel == "bl3_exact":
        # orthonormal phi: the alias sum of phi_hat^2 is 1
        return bl3.phi_hat(omega) ** 2, np.ones(n_grid)
    from . import bspline
    if bspline.order_of(kernel):
        return bspline.axis_tables(n_grid, bspline.order_of(kernel))
    fn = bl3_quadratic if kernel == "bl3q" else bl3
    return fn.window_trunc(omega) ** 2, fn.alias_sum_trunc(omega)


def mode_quantities(F, mom_used, box, n_grid, haf, flags=0, kernel="bl3", xs=None):
    """Per-mode estimator values over the full N^3 cube.

    Returns a dict of arrays with shape (N, N, N): integer n2, |k|, and the
    deconvolved, shot-subtracted P_dd, P_pp, P_tt, Re P_dt plus the shot terms.
    With xs (a slice of x indices, for grids too large to hold every per-mode
    array at once) only the modes F[:, xs] are evaluated, shape (len, N, N).
    """
    n = n_grid
    W = mom_used["W"]
    xs = slice(None) if xs is None else xs
    delta = F[0, xs] / W
    p = F[1:4, xs] / W
    nf = _integer_freqs(n)
    kf = 2.0 * math.pi / box
    nx, ny, nz = np.meshgrid(nf[xs], nf, nf, indexing="ij")
    kvec = kf * np.stack([nx, ny, nz]).astype(np.float64)
    n2 = nx * nx + ny * ny + nz * nz
    kmag = kf * np.sqrt(n2.astype(np.float64))

    w1, c1 = axis_tables(n, kernel)
    if flags & FLAG_NO_DECONVOLVE:
        w1 = np.ones(n)
    win2 = w1[xs, None, None] * w1[None, :, None] * w1[None, None, :]
    calias = c1[xs, None, None] * c1[None, :, None] * c1[None, None, :]

    s_dd = mom_used["W2"] / W ** 2
    s_ab = mom_used["s2vv"] / W ** 2
    s_pp = float(np.trace(s_ab))
    ksk = np.einsum("a...,ab,b...->...", kvec, s_ab, kvec)

    kp = np.einsum("a...,a...->...", kvec, p)
    theta = -1j * kp / haf

    sn_dd = s_dd * calias / win2
    sn_pp = s_pp * calias / win2
    sn_tt = ksk * calias / (haf * haf * win2)
    raw_dd = np.abs(delta) ** 2 / win2
    raw_pp = np.sum(np.abs(p) ** 2, axis=0) / win2
    raw_tt = np.abs(theta) ** 2 / win2
    raw_dt = np.real(delta * np.conj(theta)) / win2
    if flags & FLAG_NO_SHOTNOISE:
        p_dd, p_pp, p_tt = raw_dd, raw_pp, raw_tt
    else:
        p_dd, p_pp, p_tt = raw_dd - sn_dd, raw_pp - sn_pp, raw_tt - sn_tt
    return {"n2": n2, "kmag": kmag, "p_dd": p_dd, "p_pp": p_pp, "p_tt": p_tt,
            "p_dt": raw_dt, "sn_dd": sn_dd, "sn_pp": sn_pp, "sn_tt": sn_tt,
            "delta": delta, "p": p, "theta": theta}


BINNED = ("kmag", "p_pp", "p_tt", "p_dt", "p_dd", "sn_pp", "sn_tt", "sn_dd")


def bin_sums(q, box, n_grid, k_edges=None, n_bins=32):
    """Mode counts and sums of the per-mode quantities in |k| shells.
    Returns (edges, counts, {name: sums})."""
    n = n_grid
    kf = 2.0 * math.pi / box
    k_nyq = kf * (n // 2)
    if k_edges is None:
        idx = default_bin_index(q["n2"], n, n_bins)
        edges = k_nyq * np.arange(n_bins + 1) / n_bins
    else:
        edges = np.asarray(k_edges, dtype=np.float64)
        n_bins = len(edges) - 1
        idx = edges_bin_index(q["n2"], edge_thresholds(edges, box), n)
    sel = idx >= 0
    b = idx[sel]
    counts = np.bincount(b, minlength=n_bins).astype(np.int64)
    sums = {key: np.bincount(b, weights=q[key][sel], minlength=n_bins) for key in BINNED}
    return edges, counts, sums


def bin_means(edges, counts, sums, box):
    """Shell means from bin_sums; spectra multiplied by V = L^3."""
    vol = box ** 3

    def mean_of(s, scale):
        with np.errstate(invalid="ignore", divide="ignore"):
            return np.where(counts > 0, scale * s / counts, np.nan)

    out = {"k_edges": edges, "n_modes": counts, "k_mean": mean_of(sums["kmag"], 1.0)}
    for key in BINNED[1:]:
        out[key] = mean_of(sums[key], vol)
    return out


def bin_modes(q, box, n_grid, k_edges=None, n_bins=32):
    """Average per-mode quantities in |k| shells; multiply by V = L^3."""
    return bin_means(*bin_sums(q, box, n_grid, k_edges, n_bins), box)


def estimate(pos, vel, weight=None, *, box, n_grid, haf, k_edges=None,
             n_bins=32, flags=0, keep_modes=False, kernel="bl3"):
    """Binned P_pp, P_theta-theta, Re P_delta-theta and P_dd of one catalog."""
    if n_grid < 8 or n_grid & (n_grid - 1):
        raise ValueError("n_grid must be a power of two >= 8")
    bulk = bool(flags & FLAG_BULKFLOW_SUBTRACT)
    mom, mom_used, F = fourier_fields(pos, vel, weight, box, n_grid, bulk, kernel)
    q = mode_quantities(F, mom_used, box, n_grid, haf, flags, kernel)
    out = bin_modes(q, box, n_grid, k_edges, n_bins)
    W = mom["W"]
    extra = {"moments": mom, "moments_used": mom_used}
    if keep_modes:
        extra["modes"] = q
        extra["F"] = F
    return Spectra(
        k_edges=out["k_edges"], k_mean=out["k_mean"], p_pp=out["p_pp"],
        p_tt=out["p_tt"], p_dt=out["p_dt"], p_dd=out["p_dd"],
        sn_pp=out["sn_pp"], sn_tt=out["sn_tt"], sn_dd=out["sn_dd"],
        n_modes=out["n_modes"], v_bulk=mom["sv"] / W,
        sigma_v2=float(np.trace(mom_used["s2vv"]) / mom_used["W2"]),
        n_eff=W * W / mom["W2"], extra=extra)
