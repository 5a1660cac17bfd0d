"""Spectra of sub-samples: the catalog cut into n_div^3 equal cubes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's sub-samples (Sec. 2.4.1) cut the periodic box of side L evenly
into 4 x 4 x 4 non-overlapping cubes of side L / 4.  Their spectra, with and
without each sub-sample's own bulk flow removed, are averaged and compared
with the full sample (Sec. 3.3), and their scatter gives the error bars of
Sec. 4.1.  Readings:

* each sub-sample is estimated as a catalog of its own in a periodic box of
  side L_s = L / n_div (the same estimator as the full box, bins relative to
  the sub-box's own k_N unless edges are given);
* the split, in FP64 with every operation rounded separately:
  u = x (n_div / L), g = floor(u), index m = g - n_div floor(g / n_div)
  clamped to [0, n_div - 1], position within the cube x' = x - g L_s,
  stored as float32 (round to nearest); sub-cube number
  s = (m_x n_div + m_y) n_div + m_z; velocities and weights are unchanged;
* mean and spread over the sub-cubes that hold particles: the mean, and the
  sample standard deviation with divisor m - 1 (NaN for m < 2).
"""
from __future__ import annotations

import numpy as np

from . import estimator as E


def split(pos, box: float, n_div: int):
    """Sub-cube number of every particle and its float32 position in it."""
    if n_div < 1:
        raise ValueError("n_div must be >= 1")
    x = np.asarray(pos, dtype=np.float64)
    u = x * (n_div / box)
    g = np.floor(u)
    m = g - n_div * np.floor(g / n_div)
    m = np.clip(m, 0, n_div - 1).astype(np.int64)
    sub_box = box / n_div
    local = (x - g * sub_box).astype(np.float32)
    s = (m[:, 0] * n_div + m[:, 1]) * n_div + m[:, 2]
    return s, local


def subcatalogs(pos, vel, weight, box: float, n_div: int):
    """The n_div^3 sub-catalogs (pos', vel, weight or None), in sub-cube
    order, each keeping the original order of its particles."""
    s, local = split(pos, box, n_div)
    out = []
    for c in range(n_div ** 3):
        sel = np.nonzero(s == c)[0]
        out.append((local[sel], np.asarray(vel)[sel],
                    None if weight is None else np.asarray(weight)[sel]))
    return out


def spread(values):
    """Mean and sample standard deviation (divisor m - 1) along axis 0."""
    v = np.asarray(values, dtype=np.float64)
    m = v.shape[0]
    mean = np.sum(v, axis=0) / m if m > 0 else np.full(v.shape[1:], np.nan)
    if m < 2:
        return mean, np.full(v.shape[1:], np.nan)
    return mean, np.sqrt(np.sum((v - mean) ** 2, axis=0) / (m - 1))


SPECTRA = ("k_mean", "p_pp", "p_tt", "p_dt", "p_dd", "sn_pp", "sn_tt", "sn_dd")


def estimate_subcubes(pos, vel, weight=None, *, box, n_div, n_grid, haf, k_edges=None,
                      n_bins=32, flags=0, kernel="bl3"):
    """Per-sub-cube spectra (None for an empty sub-cube) and their mean and
    standard deviation per bin over the non-empty ones."""
    sub_box = box / n_div
    per = []
    for p, v, w in subcatalogs(pos, vel, weight, box, n_div):
        if p.shape[0] == 0:
            per.append(None)
            continue
        per.append(E.estimate(p, v, w, box=sub_box, n_grid=n_grid, haf=haf, k_edges=k_edges,
                              n_bins=n_bins, flags=flags, kernel=kernel))
    used = [r for r in per if r is not None]
    mean, sdev = {}, {}
    for key in SPECTRA:
        mean[key], sdev[key] = spread([getattr(r, key) for r in used])
    for key in ("sigma_v2", "n_eff"):
        mean[key], sdev[key] = (float(a) for a in spread([getattr(r, key) for r in used]))
    mean["v_bulk"], sdev["v_bulk"] = spread([r.v_bulk for r in used])
    return {"sub": per, "mean": mean, "sdev": sdev, "sub_box": sub_box}
