"""Pins of the oracle's transform and shell binning.

The transform is checked against a direct O(N^6) DFT and Parseval's
identity; shell counts against a brute-force integer square root.
"""
import math

import numpy as np

import oracle
from synth import catalogs


def test_fourier_fields_equal_direct_dft(rng):
    n, box = 8, 80.0
    pos = (rng.random((30, 3)) * box).astype(np.float32)
    vel = rng.normal(0, 100, (30, 3)).astype(np.float32)
    _, _, F = oracle.fourier_fields(pos, vel, None, box, n)
    charges = np.stack([np.ones(30), vel[:, 0], vel[:, 1], vel[:, 2]]).astype(np.float64)
    G = oracle.assign(pos, charges, box, n)
    g = np.arange(n)
    gx, gy, gz = np.meshgrid(g, g, g, indexing="ij")
    for c in range(4):
        for nvec in [(0, 0, 0), (1, 0, 0), (0, 3, 5), (7, 2, 4), (4, 4, 4)]:
            phase = np.exp(-2j * math.pi * (nvec[0] * gx + nvec[1] * gy + nvec[2] * gz) / n)
            direct = np.sum(G[c] * phase)
            assert abs(direct - F[c][nvec]) < 1e-10 * np.sum(np.abs(G[c]))


def test_parseval(rng):
    n, box = 16, 100.0
    pos = (rng.random((300, 3)) * box).astype(np.float32)
    vel = rng.normal(0, 100, (300, 3)).astype(np.float32)
    _, _, F = oracle.fourier_fields(pos, vel, None, box, n)
    charges = np.stack([np.ones(300), vel[:, 0], vel[:, 1], vel[:, 2]]).astype(np.float64)
    G = oracle.assign(pos, charges, box, n)
    for c in range(4):
        lhs = np.sum(np.abs(F[c]) ** 2)
        rhs = n ** 3 * np.sum(G[c] ** 2)
        assert abs(lhs - rhs) < 1e-11 * rhs


def _brute_counts(n, n_bins):
    half = n // 2
    width = half // n_bins if half >= n_bins else None
    counts = np.zeros(n_bins, np.int64)
    rng_ = range(-half, half)
    for a in rng_:
        for b in rng_:
            for c in rng_:
                n2 = a * a + b * b + c * c
                if n2 == 0 or n2 >= half * half:
                    continue
                r = math.isqrt(n2)        # floor(|n|)
                counts[r // width] += 1
    return counts


def test_default_bin_counts_match_lattice_point_count(rng):
    for n in (16, 64):
        pos, vel = catalogs.uniform_gaussian(2000, 1000.0, seed=3)
        s = oracle.estimate(pos, vel, box=1000.0, n_grid=n, haf=50.0, n_bins=n // 2 if n == 16 else 32)
        want = _brute_counts(n, n // 2 if n == 16 else 32)
        assert np.array_equal(s.n_modes, want)
    # bin 1 at N = 64 holds |n|^2 in {1, 2, 3}: 6 + 12 + 8 modes; bin 0 is empty
    assert want[0] == 0 and want[1] == 26


def test_user_edges_against_float_shells():
    n, box = 32, 500.0
    kf = 2 * math.pi / box
    edges = np.array([0.0, 0.031, 0.05, 0.11, 0.17, 0.2])
    pos, vel = catalogs.uniform_gaussian(1000, box, seed=4)
    s = oracle.estimate(pos, vel, box=box, n_grid=n, haf=50.0, k_edges=edges)
    half = n // 2
    want = np.zeros(len(edges) - 1, np.int64)
    ks = []
    for a in range(-half, half):
        for b in range(-half, half):
            for c in range(-half, half):
                n2 = a * a + b * b + c * c
                if n2 == 0 or n2 >= half * half:
                    continue
                k = kf * math.sqrt(n2)
                for i in range(len(edges) - 1):
                    if edges[i] <= k < edges[i + 1]:
                        want[i] += 1
                        ks.append((i, k))
    assert np.array_equal(s.n_modes, want)
    kmean = [np.mean([k for i, k in ks if i == b]) for b in range(len(want))]
    assert np.allclose(s.k_mean, kmean, rtol=1e-13)
