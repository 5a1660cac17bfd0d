"""Assignment with the untruncated BL3 function (the exact kernel).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The BL3 function is phi(x) = sum_n c_n beta3(x - n) (Sec. 2.4.1; c_n the
Fourier coefficients of A(w)^(-1/2), oracle.bl3).  Assigning a particle with
phi is therefore, exactly, the cubic B-spline assignment (taps j = -1..2 with
weights beta3(j - f)) followed on the periodic grid by the discrete filter
c_n along each axis:

    G_phi(g) = sum_p q_p prod_a phi(g_a - u_a)
             = sum_m c_mx c_my c_mz G_beta(g - m).

The window of phi is phi_hat(w) = sinc^4(w/2) / sqrt(A(w)) and, phi being
orthonormal, its alias sum sum_J phi_hat(w + 2 pi J)^2 is exactly 1.  This
module builds G_phi literally in that way; it does not use the equivalent
Fourier-space shortcut.
"""
from __future__ import annotations

import numpy as np

from . import bl3
from . import estimator as E

PCS_TAPS = np.arange(-1, 3)   # taps j = -1..2 relative to floor(u)


def assign_pcs(pos, charges, box: float, n_grid: int):
    """Cubic B-spline assignment: weight beta3(j - f) per axis, taps -1..2."""
    charges = np.atleast_2d(np.asarray(charges, dtype=np.float64))
    cell, frac = E.cell_and_fraction(pos, box, n_grid)
    wts = [np.stack([bl3.bspline3(j - frac[:, a]) for j in PCS_TAPS]) for a in range(3)]
    n = n_grid
    grids = np.zeros((charges.shape[0], n * n * n))
    for ix, jx in enumerate(PCS_TAPS):
        gx = (cell[:, 0] + jx) % n
        for iy, jy in enumerate(PCS_TAPS):
            gy = (cell[:, 1] + jy) % n
            wxy = wts[0][ix] * wts[1][iy]
            for iz, jz in enumerate(PCS_TAPS):
                gz = (cell[:, 2] + jz) % n
                flat = (gx * n + gy) * n + gz
                wxyz = wxy * wts[2][iz]
                for c in range(charges.shape[0]):
                    grids[c] += np.bincount(flat, weights=charges[c] * wxyz, minlength=n ** 3)
    return grids.reshape(charges.shape[0], n, n, n)


def periodic_filter(n_grid: int):
    """K[r] = sum of c_m over all |m| <= N_FILTER with m = r mod N."""
    c = bl3.filter_coefficients()
    k = np.zeros(n_grid)
    for m in range(-bl3.N_FILTER, bl3.N_FILTER + 1):
        k[m % n_grid] += c[abs(m)]
    return k


def apply_filter(grids, n_grid: int):
    """Periodic convolution with c_n along x, y and z (direct sums)."""
    k = periodic_filter(n_grid)
    out = np.asarray(grids, dtype=np.float64)
    for axis in (1, 2, 3):
        acc = np.zeros_like(out)
        for r in range(n_grid):
            if k[r] != 0.0:
                acc += k[r] * np.roll(out, r, axis=axis)
        out = acc
    return out


def assign_exact(pos, charges, box: float, n_grid: int):
    """Grids of the untruncated BL3 assignment, (n_charge, N, N, N)."""
    return apply_filter(assign_pcs(pos, charges, box, n_grid), n_grid)


def window_exact(w):
    """phi_hat(w): the window of the untruncated kernel."""
    return bl3.phi_hat(w)


def alias_sum_exact(w, j_max: int = 200):
    """sum_{|J| <= j_max} phi_hat(w + 2 pi J)^2, which is 1 for orthonormal phi."""
    w = np.asarray(w, dtype=np.float64)
    total = np.zeros(w.shape)
    for j in range(-j_max, j_max + 1):
        total = total + bl3.phi_hat(w + 2.0 * np.pi * j) ** 2
    return total
