"""Pins of the oracle's two-merge reading of the HSEG step list (Section
4.1): each iteration merges the best adjacent pair (step 2), then -- on the
partition that merge left, when the spectral stage is on at its region count
-- the best non-adjacent pair if it is below w^2 times step 2's value
(step 3). The paper's future-work list also asks for several merges per step;
this is the reading its own step list allows.

Independent pins: a hand-computed 1 x 4 case whose two readings differ, the
pure-Python HSEG (rational and canonical FP64) in the same reading, the
reduction to one merge per iteration without a spectral stage, Ward's SSE
identity, and the structure of the merge log."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2106_12942_amd import synth
from tests import pybrute
from tests.invariants import check_partition_levels, sse_of_partition

ROW = np.array([[[0.0], [5.0], [5.25], [0.125]]], dtype=np.float32)


def d2(a, b):
    """Equation 1 squared for regions given as lists of 1-band pixel values."""
    ni, nj = len(a), len(b)
    mi, mj = Fraction(sum(Fraction(x) for x in a), ni), Fraction(sum(Fraction(x) for x in b), nj)
    return float(Fraction(ni * nj, ni + nj) * (mi - mj) ** 2)


def recs(res):
    return [(int(m["lo"]), int(m["hi"]), int(m["kind"]), int(m["r_after"]), float(m["d2"])) for m in res.log]


def run_row(w, two, brute=False):
    return recs(oracle.rhseg(ROW, connectivity=4, spclust_wght=w, spclust_max=10, target_regions=1,
                             level_counts=[1], two_merges=two, brute=brute))


@pytest.mark.parametrize("brute", [False, True])
def test_hand_case_full_weight(brute):
    # step 2 merges (1,2) at 0.03125; (0,3) is then non-adjacent at 0.0078125 < 1 * 0.03125,
    # so step 3 merges it in the same iteration; one merge per iteration takes (0,3) first
    want = [(1, 2, 0, 3, d2([5.0], [5.25])), (0, 3, 1, 2, d2([0.0], [0.125])),
            (0, 1, 0, 1, d2([0.0, 0.125], [5.0, 5.25]))]
    got = run_row(1.0, True, brute)
    assert [g[:4] for g in got] == [x[:4] for x in want]
    assert all(abs(g[4] - x[4]) <= 1e-15 * x[4] for g, x in zip(got, want))
    assert [g[:4] for g in run_row(1.0, False, brute)] == [(0, 3, 1, 3), (1, 2, 0, 2), (0, 1, 0, 1)]


@pytest.mark.parametrize("brute", [False, True])
def test_hand_case_quarter_weight(brute):
    # w^2 = 1/4: step 3 needs D2 < 0.0078125 and (0,3) is exactly that, so it waits; in the next
    # iteration step 2 merges (1,3) [{1,2} and 3] and no non-adjacent pair is left. One merge
    # per iteration instead merges (0,3) in iteration 2, against that iteration's adjacent minimum.
    want = [(1, 2, 0, 3, d2([5.0], [5.25])), (1, 3, 0, 2, d2([5.0, 5.25], [0.125])),
            (0, 1, 0, 1, d2([0.0], [5.0, 5.25, 0.125]))]
    got = run_row(0.5, True, brute)
    assert [g[:4] for g in got] == [x[:4] for x in want]
    assert all(abs(g[4] - x[4]) <= 1e-15 * x[4] for g, x in zip(got, want))
    assert [g[:4] for g in run_row(0.5, False, brute)] == [(1, 2, 0, 3), (0, 3, 1, 2), (0, 1, 0, 1)]


@pytest.mark.parametrize("brute", [False, True])
@pytest.mark.parametrize("kmax,target,want", [
    # step 2 brings R from 4 to 3 = spclust_max: step 3 runs at once and merges (0,3)
    (3, 1, [(1, 2, 0, 3), (0, 3, 1, 2), (0, 1, 0, 1)]),
    # spclust_max 2: no step 3 at R = 3; then step 2 merges (1,3) and no non-adjacent pair is left
    (2, 1, [(1, 2, 0, 3), (1, 3, 0, 2), (0, 1, 0, 1)]),
    # stop count 3: step 2 reaches it, so step 3 does not run
    (10, 3, [(1, 2, 0, 3)]),
])
def test_hand_case_boundaries(kmax, target, want, brute):
    res = oracle.rhseg(ROW, connectivity=4, spclust_wght=1.0, spclust_max=kmax, target_regions=target,
                       level_counts=[target], two_merges=True, brute=brute)
    assert [g[:4] for g in recs(res)] == want


GRID = [
    dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=12, rnb_levels=2, section_regions=3),
    dict(connectivity=8, seam_connectivity=8, spclust_wght=0.21, spclust_max=30, rnb_levels=1),
    dict(connectivity=4, seam_connectivity=4, spclust_wght=1.0, spclust_max=40, rnb_levels=2, section_regions=4),
    dict(connectivity=8, seam_connectivity=4, spclust_wght=0.8, spclust_max=9, rnb_levels=3, section_regions=2),
]


@pytest.mark.parametrize("crit", ["bsmse", "sam"])
@pytest.mark.parametrize("t", range(10))
def test_matches_python_hseg(t, crit):
    p = GRID[t % len(GRID)]
    rng = np.random.default_rng(300 + t)
    H, W = int(rng.integers(4, 8)), int(rng.integers(4, 8))
    B = int(rng.integers(1, 5))
    cube = synth.random_cube(H, W, B, seed=80 + t, kind="continuous" if t % 3 else "integer")
    counts = [max(2, H * W // 2), max(2, H * W // 4), 2]
    counts = sorted(set(counts), reverse=True)
    kw = dict(p, target_regions=2, level_counts=counts, criterion=crit, two_merges=True)
    res = oracle.rhseg(cube, **kw)
    brute = oracle.rhseg(cube, **kw, brute=True)
    assert np.array_equal(res.log, brute.log) and np.array_equal(res.labels, brute.labels)
    snaps, log = pybrute.rhseg(cube, **kw)
    assert recs(res) == [tuple(x) for x in log]
    for i in range(len(counts)):
        assert np.array_equal(res.labels[i], np.array(snaps[i]))
    check_partition_levels(res.labels, counts)
    if t % 3:  # tie-free: the rational decisions agree
        _, xlog = pybrute.rhseg(cube, **kw, exact=True)
        assert [g[:4] for g in recs(res)] == [tuple(x[:4]) for x in xlog]


def test_log_structure_and_sse_identity():
    """Every non-adjacent merge directly follows the adjacent merge of its
    iteration and is below w^2 times its value; the merged D2 values add up
    to each level's SSE (Ward's identity, whatever the merge order)."""
    sc = synth.voronoi_scene(24, 20, 6, K=7, sigma=25.0, seed=9)
    w = 0.6
    counts = [150, 60, 12, 3]  # the top pass starts at 4 x 40 = 160 regions
    res = oracle.rhseg(sc.cube, connectivity=4, seam_connectivity=8, spclust_wght=w, spclust_max=150,
                       rnb_levels=2, section_regions=40, target_regions=3, level_counts=counts, two_merges=True)
    log = res.log
    w2 = float(np.float32(w)) ** 2
    n1 = 0
    for k in range(len(log)):
        if log["kind"][k] == 1:
            n1 += 1
            assert k > 0 and log["kind"][k - 1] == 0
            assert log["d2"][k] < w2 * log["d2"][k - 1]
            assert log["r_after"][k] == log["r_after"][k - 1] - 1
    assert n1 > 10
    cube = sc.cube.astype(np.float64)
    csum = np.concatenate([[0.0], np.cumsum(log["d2"])])
    H, W = sc.cube.shape[:2]
    for i, c in enumerate(counts):
        assert len(np.unique(res.labels[i])) == c
        assert abs(csum[H * W - c] - sse_of_partition(cube, res.labels[i])) <= 1e-9 * (1 + csum[H * W - c])


@pytest.mark.parametrize("kw", [dict(spclust_wght=0.0, spclust_max=50), dict(spclust_wght=0.5, spclust_max=0)])
def test_without_spectral_stage_equals_one_merge(kw):
    cube = synth.random_cube(9, 7, 3, seed=4)
    p = dict(connectivity=8, seam_connectivity=8, rnb_levels=2, section_regions=5, target_regions=2,
             level_counts=[20, 2], **kw)
    a = oracle.rhseg(cube, **p, two_merges=True)
    b = oracle.rhseg(cube, **p)
    assert np.array_equal(a.log, b.log) and np.array_equal(a.labels, b.labels)
