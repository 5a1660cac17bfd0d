"""Seeded synthetic catalogs shared by the tests, the benchmark and the oracle.

This module holds input generators only: none of the estimator's arithmetic.
All catalogs are produced in FP64 with numpy's PCG64 and handed out as
float32 arrays (positions in Mpc/h, velocities in km/s), positions wrapped
into [0, L).  Particle order is lattice order for lattice-based catalogs (x
slowest, z fastest) and generation order otherwise.

The paper measures on a Gadget-2 dark-matter simulation (1024^3 particles in a
1000 Mpc/h box); these generators stand in for it with the shapes the paper
uses: uniform "randomised" samples that keep a velocity distribution
(Sec. 2.4.2), Zel'dovich-displaced lattices with a power-law spectrum, and a
single plane wave whose spectra have a closed form.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft

SEED_BASE = 2005061700


def seed_for(config: int, index: int = 0) -> int:
    """Default seed of catalog `index` of configuration `config`."""
    return SEED_BASE + 100 * config + index


def uniform_gaussian(n: int, box: float, sigma_v: float = 300.0, seed: int = 0,
                     bulk=None, with_weights: bool = False):
    """Uniform periodic positions, i.i.d. Gaussian velocities (sigma_v per axis).

    bulk: optional 3-vector added to every velocity (an artificial bulk flow).
    with_weights: also return uniform(0.5, 1.5) float32 weights.
    Returns (pos, vel) or (pos, vel, weight).
    """
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)) * box
    vel = rng.normal(0.0, sigma_v, (n, 3))
    if bulk is not None:
        vel = vel + np.asarray(bulk, dtype=np.float64)[None, :]
    out = (_wrap32(pos, box), np.ascontiguousarray(vel, dtype=np.float32))
    if with_weights:
        out = out + (rng.uniform(0.5, 1.5, n).astype(np.float32),)
    return out


def _wrap32(pos, box):
    p = np.ascontiguousarray(np.mod(pos, box), dtype=np.float32)
    # rounding to float32 can land exactly on L; that is a legal periodic
    # coordinate, but keep generated catalogs inside [0, L)
    p[p >= np.float32(box)] = 0.0
    return p


def lattice(n_lattice: int, box: float, offset: float = 0.5):
    """Lattice points q = (i + offset) L / n_l, x slowest, z fastest; (n_l^3, 3)."""
    q1 = (np.arange(n_lattice) + offset) * (box / n_lattice)
    qx, qy, qz = np.meshgrid(q1, q1, q1, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel(), qz.ravel()], axis=1)


def gaussian_displacement(n_lattice: int, box: float, rms_disp: float,
                          slope: float = -1.5, k_cut: float = 0.5,
                          seed: int = 0, workers: int = -1):
    """Zel'dovich displacement Psi = -grad inv-laplacian delta on the lattice.

    delta is a Gaussian random field with P(k) = A k^slope exp(-k / k_cut),
    drawn as white noise coloured by sqrt(P); DC and Nyquist modes are zeroed
    and A is fixed so that the realised rms |Psi| equals rms_disp.
    Returns float64 array (3, n_l, n_l, n_l).
    """
    n = n_lattice
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    dk = scipy.fft.rfftn(white, workers=workers)
    del white
    kf = 2.0 * math.pi / box
    k1 = kf * np.fft.fftfreq(n, 1.0 / n)
    kz1 = kf * np.arange(n // 2 + 1)
    kx = k1[:, None, None]
    ky = k1[None, :, None]
    kz = kz1[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    kk = np.sqrt(k2)
    amp = np.sqrt(kk ** slope * np.exp(-kk / k_cut))
    amp[0, 0, 0] = 0.0
    amp[n // 2, :, :] = 0.0
    amp[:, n // 2, :] = 0.0
    amp[:, :, n // 2] = 0.0
    dk *= amp
    del amp
    psi = np.empty((3, n, n, n))
    for a, ka in enumerate((kx, ky, kz)):
        psi[a] = scipy.fft.irfftn(1j * ka * dk / k2, s=(n, n, n), workers=workers)
    rms = math.sqrt(float(np.mean(np.sum(psi * psi, axis=0))))
    psi *= rms_disp / rms
    return psi


def zeldovich(n_lattice: int, box: float, rms_disp: float, haf: float = 50.0,
              slope: float = -1.5, k_cut: float = 0.5, seed: int = 0,
              bulk=None, workers: int = -1):
    """Lattice displaced by a Zel'dovich field; v = Haf * Psi (+ bulk).

    Returns float32 (pos, vel), each (n_l^3, 3), in lattice order.
    """
    psi = gaussian_displacement(n_lattice, box, rms_disp, slope, k_cut, seed,
                                workers)
    disp = psi.reshape(3, -1).T
    del psi
    pos = _wrap32(lattice(n_lattice, box) + disp, box)
    vel = haf * disp
    if bulk is not None:
        vel = vel + np.asarray(bulk, dtype=np.float64)[None, :]
    return pos, np.ascontiguousarray(vel, dtype=np.float32)


def zeldovich_sampled(n_lattice: int, box: float, rms_disp: float, fraction: float,
                      haf: float = 50.0, seed: int = 0, bulk=None):
    """A clustered catalog with Poisson shot noise: each particle of a
    Zel'dovich catalog (as zeldovich()) is kept with probability `fraction`
    (independent draws; the lattice's own sub-Poisson discreteness is then
    diluted to about (1 - fraction) of the Poisson level).

    Returns float32 (pos, vel) in lattice order.
    """
    pos, vel = zeldovich(n_lattice, box, rms_disp, haf=haf, seed=seed, bulk=bulk)
    keep = np.random.default_rng(seed + 1).random(pos.shape[0]) < fraction
    return np.ascontiguousarray(pos[keep]), np.ascontiguousarray(vel[keep])


def plane_wave(n_lattice: int, box: float, amp: float, m_wave: int,
               haf: float = 50.0, offset: float = 0.5):
    """Single Zel'dovich plane wave along x on a lattice.

    x = q + A sin(k0 q_x) e_x and v = Haf A sin(k0 q_x) e_x with
    k0 = 2 pi m_wave / L and lattice q = (i + offset) L / n_l.
    Returns float32 (pos, vel).
    """
    q = lattice(n_lattice, box, offset)
    k0 = 2.0 * math.pi * m_wave / box
    s = amp * np.sin(k0 * q[:, 0])
    pos = q.copy()
    pos[:, 0] += s
    vel = np.zeros_like(q)
    vel[:, 0] = haf * s
    return _wrap32(pos, box), np.ascontiguousarray(vel, dtype=np.float32)


def bulk_vector(speed: float, direction=(1.0, 2.0, 2.0)):
    """A bulk-flow vector of the given speed along `direction`."""
    d = np.asarray(direction, dtype=np.float64)
    return speed * d / np.linalg.norm(d)
