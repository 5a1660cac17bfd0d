"""Pins of the sub-sample split (Sec. 2.4.1: the box cut into 4 x 4 x 4 equal
cubes) and of the statistics over sub-samples (Secs. 3.3, 4.1)."""
import math

import numpy as np
import pytest

import oracle
from oracle import subcubes as S

BOX = 1000.0
HAF = 50.0


def _quantised_uniform(rng, n, hi):
    """Positions on multiples of 2^-14 in [0, hi): with hi + BOX < 2^10 every
    sum with a multiple of 250 below 1000 is exact in float32."""
    return (np.floor(rng.random((n, 3)) * hi * 2.0 ** 14) / 2.0 ** 14).astype(np.float32)


def test_hand_placed_particles():
    # worked by hand: L = 1000, n_div = 4, L_s = 250
    pos = np.array([[260.5, 0.25, 999.75],    # cube (1, 0, 3) at (10.5, 0.25, 249.75)
                    [-10.0, 1000.0, 500.0],   # wraps: cube (3, 0, 2) at (240, 0, 0)
                    [749.5, 250.0, 0.0]],     # cube (2, 1, 0) at (249.5, 0, 0)
                   dtype=np.float32)
    s, local = S.split(pos, BOX, 4)
    assert s.tolist() == [1 * 16 + 0 * 4 + 3, 3 * 16 + 0 * 4 + 2, 2 * 16 + 1 * 4 + 0]
    assert local.dtype == np.float32
    np.testing.assert_array_equal(local, np.array([[10.5, 0.25, 249.75], [240.0, 0.0, 0.0],
                                                   [249.5, 0.0, 0.0]], dtype=np.float32))


@pytest.mark.parametrize("n_div", [1, 2, 3, 4])
def test_split_is_a_partition(n_div):
    rng = np.random.default_rng(5)
    pos = (rng.random((20000, 3)) * 1.2 * BOX - 0.1 * BOX).astype(np.float32)  # some outside [0, L)
    s, local = S.split(pos, BOX, n_div)
    assert s.min() >= 0 and s.max() < n_div ** 3
    ls = BOX / n_div
    # within the cube up to the rounding of u (a local position a hair below 0
    # is the same point of the periodic sub-box as 0)
    assert local.min() > -1e-9 * ls and local.max() < ls * (1 + 1e-7)
    # the cube index and the local position give back the periodic position
    m = np.stack([s // (n_div * n_div), (s // n_div) % n_div, s % n_div], axis=1)
    back = (local.astype(np.float64) + m * ls) % BOX
    want = pos.astype(np.float64) % BOX
    d = np.abs(back - want)
    d = np.minimum(d, BOX - d)
    assert d.max() < 1e-4, d.max()
    subs = S.subcatalogs(pos, pos, None, BOX, n_div)
    assert sum(p.shape[0] for p, _, _ in subs) == pos.shape[0]


def test_whole_box_is_one_subcube():
    rng = np.random.default_rng(6)
    pos = (rng.random((3000, 3)) * BOX).astype(np.float32)
    vel = (rng.normal(0, 300, (3000, 3))).astype(np.float32)
    r = S.estimate_subcubes(pos, vel, box=BOX, n_div=1, n_grid=8, haf=HAF)
    full = oracle.estimate(pos, vel, box=BOX, n_grid=8, haf=HAF)
    for key in ("p_pp", "p_tt", "p_dt", "p_dd"):
        np.testing.assert_array_equal(getattr(r["sub"][0], key), getattr(full, key))


def test_translation_by_one_cube_permutes_the_subsamples():
    """Shifting every particle by L / n_div along y moves sub-sample
    (a, b, c) to (a, b + 1 mod n, c) unchanged."""
    n_div = 2
    rng = np.random.default_rng(7)
    pos = _quantised_uniform(rng, 4000, BOX)
    vel = rng.normal(0, 300, (4000, 3)).astype(np.float32)
    moved = pos.astype(np.float64)
    moved[:, 1] = (moved[:, 1] + BOX / n_div) % BOX
    moved = moved.astype(np.float32)
    a = S.estimate_subcubes(pos, vel, box=BOX, n_div=n_div, n_grid=8, haf=HAF)
    b = S.estimate_subcubes(moved, vel, box=BOX, n_div=n_div, n_grid=8, haf=HAF)
    for s in range(n_div ** 3):
        i, j, k = s // 4, (s // 2) % 2, s % 2
        t = (i * n_div + (j + 1) % n_div) * n_div + k
        for key in ("p_pp", "p_tt", "p_dt", "p_dd", "sn_tt"):
            np.testing.assert_array_equal(getattr(b["sub"][t], key), getattr(a["sub"][s], key))


def test_replicated_catalog_gives_identical_subsamples():
    """64 copies of one 250 Mpc/h catalog, one per cube: every sub-sample is
    that catalog, the mean is its spectrum and the spread is zero."""
    rng = np.random.default_rng(8)
    base = _quantised_uniform(rng, 500, BOX / 4)
    vel = rng.normal(0, 300, (500, 3)).astype(np.float32)
    w = rng.uniform(0.5, 2.0, 500).astype(np.float32)
    shifts = np.stack(np.meshgrid(*[np.arange(4)] * 3, indexing="ij"), -1).reshape(-1, 3) * (BOX / 4)
    pos = np.concatenate([base + sh.astype(np.float32) for sh in shifts])
    assert np.array_equal(pos.astype(np.float64),
                          np.concatenate([base.astype(np.float64) + sh for sh in shifts]))
    r = S.estimate_subcubes(pos, np.tile(vel, (64, 1)), np.tile(w, 64), box=BOX, n_div=4,
                            n_grid=8, haf=HAF, flags=oracle.FLAG_BULKFLOW_SUBTRACT)
    one = oracle.estimate(base, vel, w, box=BOX / 4, n_grid=8, haf=HAF,
                          flags=oracle.FLAG_BULKFLOW_SUBTRACT)
    for key in ("p_pp", "p_tt", "p_dt", "p_dd"):
        for sub in r["sub"]:
            np.testing.assert_array_equal(getattr(sub, key), getattr(one, key))
        np.testing.assert_allclose(r["mean"][key], getattr(one, key), rtol=1e-14, equal_nan=True)
        sd = r["sdev"][key]
        assert np.all((sd[np.isfinite(sd)] < 1e-9 * np.nanmax(np.abs(getattr(one, key)))))


def test_spread_closed_forms():
    a, b = np.array([1.0, -2.0, 5.0]), np.array([3.0, 2.0, 5.0])
    mean, sd = S.spread([a, b])
    np.testing.assert_allclose(mean, [2.0, 0.0, 5.0])
    np.testing.assert_allclose(sd, [math.sqrt(2.0), 2.0 * math.sqrt(2.0), 0.0])
    mean, sd = S.spread([a])
    np.testing.assert_array_equal(mean, a)
    assert np.all(np.isnan(sd))
    # 1, 2, ..., 10: mean 5.5, sample variance 55 / 6
    mean, sd = S.spread(np.arange(1.0, 11.0))
    assert mean == 5.5 and abs(sd - math.sqrt(55.0 / 6.0)) < 1e-14


def test_empty_subcubes_are_skipped():
    rng = np.random.default_rng(9)
    pos = (rng.random((3000, 3)) * [BOX / 2, BOX, BOX]).astype(np.float32)  # x < L / 2 only
    vel = rng.normal(0, 300, (3000, 3)).astype(np.float32)
    r = S.estimate_subcubes(pos, vel, box=BOX, n_div=2, n_grid=8, haf=HAF)
    assert [sub is None for sub in r["sub"]] == [False] * 4 + [True] * 4
    mean, _ = S.spread([sub.p_pp for sub in r["sub"][:4]])
    np.testing.assert_array_equal(r["mean"]["p_pp"], mean)
