"""Pins of the oracle's BL3 assignment (Eq. rawFFTed with the BL3 window).

Brute force: every (particle, node) pair evaluated from the periodic
displacement with the truncated kernel phi_t, no tap bookkeeping.  Lattice
constancy and integer-cell translation are exact properties of any
shift-invariant assignment.
"""
import numpy as np
import scipy.fft

import oracle
from oracle import bl3


def _brute_force(pos, q, box, n):
    pos = np.asarray(pos, dtype=np.float64)
    u = pos * (n / box)
    g = np.arange(n)
    out = np.zeros((n, n, n))
    for j in range(len(pos)):
        w = []
        for a in range(3):
            d = g - u[j, a]
            # periodic image of the displacement in (-n/2, n/2]
            d = d - n * np.ceil((d - n / 2) / n)
            w.append(bl3.phi_trunc(d))
        out += q[j] * w[0][:, None, None] * w[1][None, :, None] * w[2][None, None, :]
    return out


def test_matches_brute_force_small_grids(rng):
    for n in (8, 10, 16):
        box = 100.0
        pos = (rng.random((25, 3)) * box).astype(np.float32)
        # on-node, at x = L and negative coordinates are all legal
        pos[0] = [0.0, 50.0, 12.5]
        pos[1] = [box, 0.0, -25.0]
        pos[2] = [-3.0, 99.999, 37.5]
        q = rng.normal(size=25)
        got = oracle.assign(pos, q[None, :], box, n)[0]
        want = _brute_force(pos, q, box, n)
        assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want)), n


def test_lattice_is_constant_field():
    n = 16
    box = 1000.0
    q1 = (np.arange(n) + 0.37) * (box / n)
    qx, qy, qz = np.meshgrid(q1, q1, q1, indexing="ij")
    pos = np.stack([qx.ravel(), qy.ravel(), qz.ravel()], 1)
    g = oracle.assign(pos, np.ones((1, n ** 3)), box, n)[0]
    assert np.std(g) < 1e-12 * np.mean(g)
    F = scipy.fft.fftn(g)
    F[0, 0, 0] = 0
    assert np.max(np.abs(F)) < 1e-9 * np.mean(g) * n ** 3


def test_integer_cell_translation_rolls_grid(rng):
    n, box = 16, 1000.0          # dL = 62.5 is exact in binary
    # coordinates on a 1/1024 lattice so that the float32 shift is exact
    pos = (np.round(rng.random((200, 3)) * (box - 300) * 1024) / 1024).astype(np.float32)
    q = rng.normal(size=(2, 200))
    g0 = oracle.assign(pos, q, box, n)
    shifted = pos.copy()
    shifted[:, 1] += np.float32(3 * box / n)
    g1 = oracle.assign(shifted, q, box, n)
    assert np.allclose(np.roll(g0, 3, axis=2), g1, rtol=0, atol=1e-12)


def test_total_mass_is_product_of_tap_sums(rng):
    n, box = 12, 50.0
    pos = (rng.random((40, 3)) * box).astype(np.float32)
    w = rng.random(40)
    g = oracle.assign(pos, w[None, :], box, n)[0]
    _, frac = oracle.cell_and_fraction(pos, box, n)
    per_axis = [np.sum(bl3.tap_weights(frac[:, a]), axis=0) for a in range(3)]
    assert abs(g.sum() - np.sum(w * per_axis[0] * per_axis[1] * per_axis[2])) < 1e-11


def test_cell_index_wraps_periodically():
    pos = np.array([[0.0, -0.1, 1000.0], [999.99, -1000.0, 2500.0]], np.float32)
    cell, frac = oracle.cell_and_fraction(pos, 1000.0, 64)
    assert cell.min() >= 0 and cell.max() < 64
    assert cell[0, 2] == 0 and cell[1, 1] == 0 and cell[1, 2] == 32
    assert np.all((frac >= 0) & (frac < 1))


def test_single_node_sums_match_brute_force(rng):
    """oracle.assign_cells (a per-node sum over particles, used to check the
    library at full size on sampled nodes) equals the brute force at every
    node of small grids, including wrapped particles."""
    for n in (8, 16):
        box = 100.0
        pos = (rng.random((40, 3)) * box).astype(np.float32)
        pos[0] = [0.0, 50.0, 12.5]
        pos[1] = [box, 0.0, -25.0]
        pos[2] = [-3.0, 99.999, 37.5]
        q = rng.normal(size=(2, 40))
        g = np.arange(n)
        cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
        got = oracle.assign_cells(pos, q, box, n, cells)
        for c in range(2):
            want = _brute_force(pos, q[c], box, n).reshape(-1)
            assert np.max(np.abs(got[c] - want)) < 1e-12 * np.max(np.abs(want)), (n, c)
