"""Pins of the oracle's spectral angle criterion (Section 4.1 lists the
spectral angle mapper among the dissimilarities HSEG can use).

The ranked value is D = 1 - sign(c) c^2 with c the cosine of the angle
between the two regions' mean spectra, i.e. sin^2(theta) up to 90 degrees
and 2 - sin^2(theta) beyond. The pins are independent of the oracle's code:
hand-computed closed forms, trigonometry, scipy's cosine distance, exact
power-of-two scale invariance, a pure-Python rational-arithmetic HSEG, and a
tie-only special case whose merge order follows from the tie-break alone."""
import math

import numpy as np
import pytest
from scipy.spatial import distance

import oracle
from oracle import oracle as orc
from paper_2106_12942_amd import synth
from tests import pybrute
from tests.invariants import check_partition_levels


def sam(a, b):
    return orc.criterion_sam(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64))


@pytest.mark.parametrize("a,b,want", [
    ([3.0, 4.0], [4.0, 3.0], 49.0 / 625.0),       # cos = 24/25: sin^2 = 49/625
    ([1.0, 0.0], [0.0, 1.0], 1.0),                # orthogonal
    ([1.0, 1.0], [2.0, 2.0], 0.0),                # parallel
    ([1.0, 0.0], [-1.0, 0.0], 2.0),               # opposite
    ([3.0, 4.0], [-4.0, -3.0], 2.0 - 49.0 / 625.0),
    ([1.0, 2.0, 2.0], [2.0, 1.0, -2.0], 1.0),     # orthogonal in 3 bands
    ([1.0, 2.0, 2.0], [2.0, 2.0, 1.0], 1.0 - 64.0 / 81.0),
    ([0.0, 0.0, 0.0], [5.0, 1.0, 2.0], 1.0),      # a zero spectrum counts as orthogonal
    ([7.5], [-0.25], 2.0),                        # one band: only 0 or 2
    ([7.5], [0.25], 0.0),
])
def test_hand_computed_values(a, b, want):
    got = sam(a, b)
    assert abs(got - want) <= 1e-15 * max(1.0, want), (got, want)
    assert sam(b, a) == got  # symmetric, bit for bit


def test_matches_trigonometry_over_the_half_turn():
    for deg in np.linspace(0.0, 180.0, 181):
        t = math.radians(deg)
        a = [2.0, 0.0]
        b = [3.0 * math.cos(t), 3.0 * math.sin(t)]
        want = math.sin(t) ** 2 if deg <= 90.0 else 2.0 - math.sin(t) ** 2
        assert abs(sam(a, b) - want) < 1e-12, deg


def test_matches_scipy_cosine_distance():
    rng = np.random.default_rng(5)
    for B in (1, 2, 3, 7, 64, 100, 257):
        for _ in range(20):
            a = rng.normal(size=B) * 10.0 ** rng.integers(-3, 4)
            b = rng.normal(size=B) + (rng.random() < 0.5) * a  # some nearly parallel pairs
            c = 1.0 - distance.cosine(a, b)
            want = 1.0 - math.copysign(c * c, c)
            assert abs(sam(a, b) - want) < 1e-12, (B, want)


def test_scale_invariance_is_exact_for_powers_of_two():
    # the counts cancel: scaling either sum vector by 2^k changes no rounding
    rng = np.random.default_rng(8)
    for B in (3, 50, 220):
        a = synth.quantise_f32(rng.uniform(-1000, 1000, size=B)).astype(np.float64)
        b = synth.quantise_f32(rng.uniform(-1000, 1000, size=B)).astype(np.float64)
        d = sam(a, b)
        for ka, kb in ((1, 0), (0, 5), (7, 3), (-4, 9)):
            assert sam(a * 2.0 ** ka, b * 2.0 ** kb) == d


def test_bounds_and_zero_on_the_diagonal():
    rng = np.random.default_rng(9)
    for _ in range(200):
        B = int(rng.integers(1, 40))
        a = rng.uniform(-5, 5, size=B)
        b = rng.uniform(-5, 5, size=B)
        d = sam(a, b)
        assert 0.0 <= d <= 2.0
        assert sam(a, a) <= 4e-16 * B  # parallel up to rounding
        assert abs(sam(a, -a) - 2.0) <= 4e-16 * B
        for k in (3.0, 5.0, 7.0):  # parallel with rounding either way: never below 0
            assert 0.0 <= sam(a, k * a) <= 4e-16 * B


GRID = [
    dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=12, rnb_levels=2, section_regions=3),
    dict(connectivity=8, seam_connectivity=8, spclust_wght=0.21, spclust_max=30, rnb_levels=1),
    dict(connectivity=4, seam_connectivity=4, spclust_wght=1.0, spclust_max=40, rnb_levels=2, section_regions=4),
    dict(connectivity=8, seam_connectivity=8, spclust_wght=0.0, spclust_max=0, rnb_levels=2, section_regions=5),
]


@pytest.mark.parametrize("t", range(12))
def test_hseg_matches_rational_python_hseg(t):
    """Whole merge loop against pybrute in exact rational arithmetic (its
    decisions are the mathematically exact ones) and in canonical FP64 (its
    values must then be bit-identical), both oracle modes."""
    p = GRID[t % len(GRID)]
    rng = np.random.default_rng(100 + t)
    H, W = int(rng.integers(3, 7)), int(rng.integers(3, 7))
    B = int(rng.integers(1, 6))
    cube = synth.random_cube(H, W, B, seed=60 + t, kind="continuous" if t % 3 else "integer")
    counts = [max(2, H * W // 2), 2]
    res = oracle.rhseg(cube, **p, target_regions=2, level_counts=counts, criterion="sam")
    brute = oracle.rhseg(cube, **p, target_regions=2, level_counts=counts, criterion="sam", brute=True)
    assert np.array_equal(res.log, brute.log) and np.array_equal(res.labels, brute.labels)
    snaps, log = pybrute.rhseg(cube, **p, target_regions=2, level_counts=counts, criterion="sam")
    got = [(int(m["lo"]), int(m["hi"]), int(m["kind"]), int(m["r_after"]), float(m["d2"])) for m in res.log]
    assert got == [tuple(x) for x in log]
    for i in range(2):
        assert np.array_equal(res.labels[i], np.array(snaps[i]))
    check_partition_levels(res.labels, counts)
    if t % 3:  # tie-free continuous data: exact rational decisions agree
        _, xlog = pybrute.rhseg(cube, **p, target_regions=2, level_counts=counts, criterion="sam", exact=True)
        assert [g[:4] for g in got] == [tuple(x[:4]) for x in xlog]
        assert all(abs(g[4] - float(x[4])) <= 1e-12 for g, x in zip(got, xlog))


def test_spectral_stage_is_exercised():
    # the rational comparison above decides weighted adjacent-vs-spectral
    # choices; make sure the grid really produces non-adjacent merges
    cube = synth.random_cube(6, 6, 4, seed=61, kind="continuous")
    res = oracle.rhseg(cube, **GRID[1], target_regions=2, level_counts=[2], criterion="sam")
    kinds = res.log["kind"]
    assert 0 < kinds.sum() < len(kinds)


@pytest.mark.parametrize("H,W,conn", [(4, 5, 4), (3, 7, 8), (1, 9, 4)])
def test_all_ties_grow_region_zero_in_raster_order(H, W, conn):
    """One positive band: every pair has angle 0, so every D is 0 and the
    (D, lo, hi) tie-break alone orders the merges. Region 0 always has the
    smallest key, and its smallest-labelled neighbour is the next pixel in
    raster order, so after m merges region 0 holds pixels 0..m and every other
    pixel is alone; with D = 0 the spectral stage never wins (0 < w^2 * 0 is
    false)."""
    rng = np.random.default_rng(H * 100 + W)
    cube = rng.integers(1, 50, size=(H, W, 1)).astype(np.float32)
    counts = [H * W - 1, H * W // 2, 1]
    res = oracle.rhseg(cube, connectivity=conn, spclust_wght=0.7, spclust_max=H * W, target_regions=1,
                       level_counts=counts, criterion="sam")
    assert (res.log["d2"] == 0.0).all() and (res.log["kind"] == 0).all()
    assert [(int(m["lo"]), int(m["hi"])) for m in res.log] == [(0, k) for k in range(1, H * W)]
    idx = np.arange(H * W).reshape(H, W)
    for lvl, k in enumerate(counts):
        m = H * W - k
        assert np.array_equal(res.labels[lvl], np.where(idx <= m, 0, idx))


def test_unknown_criterion_rejected():
    cube = synth.random_cube(3, 3, 2, seed=1)
    with pytest.raises(KeyError):
        oracle.rhseg(cube, criterion="sid")
