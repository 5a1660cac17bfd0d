"""The oracle's estimator for catalogs and grids too large for the direct
form's intermediate arrays (512^3 grids with 512^3 particles).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The steps and the arithmetic are those of oracle.estimator.estimate, taken
piece by piece so that memory stays bounded:

* moments: oracle.estimator.moments over the whole catalog;
* assignment (Eq. rawFFTed with the truncated BL3 function, Sec. 2.4.1):
  particles ordered by their x cell and taken in chunks; each chunk deposits
  q phi(jx - fx) phi(jy - fy) phi(jz - fz) on node (cell + j) mod N for the
  taps j in {-2..3}^3 into a block of x planes just wide enough for it, and
  the block is added into the periodic grid (the direct form's np.bincount
  over the whole grid, restricted to the planes the chunk reaches);
* bulk flow (Sec. 3.1): the grids of w (v - v_b) are assigned, as in the
  direct form;
* FFT: scipy.fft.fftn of each field, FP64, e^{-i k.x};
* per mode and binning: oracle.estimator.mode_quantities over slabs of x
  indices, shell sums accumulated over the slabs (oracle.estimator.bin_sums),
  then the means (oracle.estimator.bin_means).

Only the order in which floating-point sums are accumulated differs from the
direct form; tests/test_oracle_large.py checks the two agree to ~1e-12.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from . import bl3, bl3_quadratic
from . import estimator as E

KERNELS = {"bl3": bl3, "bl3q": bl3_quadratic}


_SHARED = {}


def _chunk_block(c0):
    """Deposits of the particles order[c0 : c0 + chunk] into a block of the
    x planes they reach: returns (first plane, block (n_charge, span, N, N))."""
    sh = _SHARED
    fn, n, taps = KERNELS[sh["kernel"]], sh["n"], KERNELS[sh["kernel"]].TAPS
    idx = sh["order"][c0:c0 + sh["chunk"]]
    cl, fr = sh["cell"][idx], sh["frac"][idx]
    q = sh["charges"][:, idx]
    nq = q.shape[0]
    x0 = int(cl[:, 0].min()) + int(taps[0])
    span = int(cl[:, 0].max()) + int(taps[-1]) - x0 + 1
    wts = [fn.tap_weights(fr[:, a]) for a in range(3)]
    block = np.zeros((nq, span * n * n))
    for ix, jx in enumerate(taps):
        lx = cl[:, 0] + jx - x0                      # plane in the block, unwrapped
        for iy, jy in enumerate(taps):
            gy = (cl[:, 1] + jy) % n
            wxy = wts[0][ix] * wts[1][iy]
            for iz, jz in enumerate(taps):
                gz = (cl[:, 2] + jz) % n
                flat = (lx * n + gy) * n + gz
                wxyz = wxy * wts[2][iz]
                for k in range(nq):
                    block[k] += np.bincount(flat, weights=q[k] * wxyz, minlength=span * n * n)
    return x0, block.reshape(nq, span, n, n)


def assign_chunked(pos, charges, box: float, n_grid: int, kernel: str = "bl3", chunk: int = 1 << 22,
                   workers: int = 1):
    """The four assigned grids (n_charge, N, N, N), accumulated chunk by chunk
    (see the module docstring).  charges has shape (n_charge, n_particles).
    With workers > 1 the chunks' blocks are computed in forked processes; they
    are added in chunk order either way, so the result does not depend on it."""
    n = n_grid
    cell, frac = E.cell_and_fraction(pos, box, n)
    order = np.argsort(cell[:, 0], kind="stable")
    nq = charges.shape[0]
    grids = np.zeros((nq, n, n, n))
    _SHARED.update(kernel=kernel, n=n, order=order, cell=cell, frac=frac, charges=charges, chunk=chunk)
    starts = list(range(0, order.shape[0], chunk))

    def add(x0, block):
        for lp in range(block.shape[1]):
            grids[:, (x0 + lp) % n] += block[:, lp]

    try:
        if workers > 1 and len(starts) > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(workers) as pool:
                for x0, block in pool.imap(_chunk_block, starts):
                    add(x0, block)
        else:
            for c0 in starts:
                add(*_chunk_block(c0))
    finally:
        _SHARED.clear()
    return grids


def estimate_large(pos, vel, weight=None, *, box, n_grid, haf, k_edges=None, n_bins=32, flags=0,
                   kernel="bl3", chunk=1 << 22, slab=16, workers=1):
    """Binned spectra of one catalog as oracle.estimate returns them (an
    oracle.estimator.Spectra), computed piece by piece."""
    if n_grid < 8 or n_grid & (n_grid - 1):
        raise ValueError("n_grid must be a power of two >= 8")
    n_p = pos.shape[0]
    vel = np.asarray(vel, dtype=np.float64)
    w = np.ones(n_p) if weight is None else np.asarray(weight, dtype=np.float64)
    mom = E.moments(vel, w)
    v_used = vel
    if flags & E.FLAG_BULKFLOW_SUBTRACT:
        v_used = vel - (mom["sv"] / mom["W"])[None, :]
    mom_used = E.moments(v_used, w)
    charges = np.stack([w, w * v_used[:, 0], w * v_used[:, 1], w * v_used[:, 2]])
    del v_used
    grids = assign_chunked(pos, charges, box, n_grid, kernel, chunk, workers)
    del charges
    F = np.empty((4, n_grid, n_grid, n_grid), dtype=np.complex128)
    for c in range(4):
        F[c] = scipy.fft.fftn(grids[c], workers=-1)
    del grids
    counts, sums, edges = None, None, None
    for x0 in range(0, n_grid, slab):
        q = E.mode_quantities(F, mom_used, box, n_grid, haf, flags, kernel, xs=slice(x0, x0 + slab))
        edges, cnt, sm = E.bin_sums(q, box, n_grid, k_edges, n_bins)
        if counts is None:
            counts, sums = cnt, sm
        else:
            counts = counts + cnt
            sums = {k: sums[k] + sm[k] for k in sums}
    out = E.bin_means(edges, counts, sums, box)
    W = mom["W"]
    return E.Spectra(
        k_edges=out["k_edges"], k_mean=out["k_mean"], p_pp=out["p_pp"], p_tt=out["p_tt"],
        p_dt=out["p_dt"], p_dd=out["p_dd"], sn_pp=out["sn_pp"], sn_tt=out["sn_tt"], sn_dd=out["sn_dd"],
        n_modes=out["n_modes"], v_bulk=mom["sv"] / W,
        sigma_v2=float(np.trace(mom_used["s2vv"]) / mom_used["W2"]),
        n_eff=W * W / mom["W2"], extra={"moments": mom, "moments_used": mom_used})
