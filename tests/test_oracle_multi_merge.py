"""Pins of the oracle's several-merges-per-step mode, the future-work item of
Section 6.2 (several region merges per step, fewer steps for merging
identical regions), read as: a step whose one-merge winner has the value 0
merges a greedy disjoint set of zero-valued pairs -- adjacent pairs by
(lo, hi), then, with the spectral stage on at the step's start, non-adjacent
pairs by (lo, hi) -- one after another until the pass's stop count; any other
step is one merge. The second and later merges of a step carry kind + 2.

Independent pins: hand-computed strips whose one-merge and multi-merge logs
differ, the pure-Python HSEG in the same mode (which finds each merge of a
step afresh from the label map instead of from one ranked list), the
reduction to the one-merge reading on tie-free cubes, the agreement of the
partitions between zero storms with the one-merge reading, Ward's SSE
identity and the structure of the log."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2106_12942_amd import synth
from tests import pybrute
from tests.invariants import check_partition_levels, sse_of_partition


def recs(res):
    return [(int(m["lo"]), int(m["hi"]), int(m["kind"]), int(m["r_after"]), float(m["d2"])) for m in res.log]


def strip(values):
    return np.array([[[float(v)] for v in values]], dtype=np.float32)


def run(cube, multi, brute=False, target=1, w=0.5, kmax=10):
    return oracle.rhseg(cube, connectivity=4, spclust_wght=w, spclust_max=kmax, target_regions=target,
                        level_counts=[target], multi_merge=multi, brute=brute)


# 1 x 6 strip x = 1 1 1 7 1 1, w = 0.5, spectral stage on throughout (spclust_max 10).
#  step 1, R=6: adjacent (0,1)=(1,2)=(4,5)=0, (2,3)=(3,4)=1/2*36=18 -> winner (0,1) at 0.
#     zero pairs ranked: adjacent (0,1),(1,2),(4,5); non-adjacent (0,2),(0,4),(0,5),(1,4),(1,5),
#     (2,4),(2,5). Greedy: (0,1) taken, (1,2) skipped (1 taken), (4,5) taken, every non-adjacent
#     pair touches 0, 1, 4 or 5 -> merges (0,1) and (4,5).
#  step 2, R=4: {0,1} n2 mean 1, {2} 1, {3} 7, {4,5} n2 mean 1. Adjacent (0,2)=0, (2,3)=18,
#     (3,4)=2/3*36=24 -> winner (0,2) at 0; non-adjacent zeros (0,4), (2,4) both touch a taken
#     region -> one merge (0,2).
#  step 3, R=3: {0,1,2} n3, {3}, {4,5} n2. Adjacent (0,3)=3/4*36=27, (3,4)=24; non-adjacent
#     (0,4)=0 < w^2*24 -> non-adjacent winner at 0, the only zero pair -> merge (0,4).
#  step 4, R=2: (0,3) = 5/6*36 = 30.
# One merge per step instead takes (0,1), (0,2), (4,5), (0,4), (0,3): the same partitions
# between storms, in five steps instead of four, and different level maps at R = 4.
STRIP_A = [1, 1, 1, 7, 1, 1]


@pytest.mark.parametrize("brute", [False, True])
def test_hand_strip_adjacent_storm(brute):
    got = recs(run(strip(STRIP_A), True, brute))
    assert got == [(0, 1, 0, 5, 0.0), (4, 5, 2, 4, 0.0), (0, 2, 0, 3, 0.0), (0, 4, 1, 2, 0.0),
                   (0, 3, 0, 1, float(Fraction(5, 6) * 36))]
    one = recs(run(strip(STRIP_A), False, brute))
    assert [g[:4] for g in one] == [(0, 1, 0, 5), (0, 2, 0, 4), (4, 5, 0, 3), (0, 4, 1, 2), (0, 3, 0, 1)]


@pytest.mark.parametrize("brute", [False, True])
@pytest.mark.parametrize("target,want", [
    (5, [(0, 1, 0, 5)]),                 # the stop count ends step 1 after its first merge
    (4, [(0, 1, 0, 5), (4, 5, 2, 4)]),   # ... or exactly at its end
    (3, [(0, 1, 0, 5), (4, 5, 2, 4), (0, 2, 0, 3)]),
])
def test_hand_strip_stop_count(target, want, brute):
    assert [g[:4] for g in recs(run(strip(STRIP_A), True, brute, target=target))] == want


# 1 x 7 strip x = 1 9 1 9 1 9 1, w = 0.5, spclust_max 10: every adjacent pair is 1/2*64 = 32,
# the identical regions are never adjacent.
#  step 1, R=7: N = (0,2) at 0 < w^2*32 -> winner. Ranked non-adjacent zeros: (0,2),(0,4),(0,6),
#     (1,3),(1,5),(2,4),(2,6),(3,5),(4,6); greedy takes (0,2), (1,3), (4,6).
#  step 2, R=4: {0,2} n2 mean 1, {1,3} n2 mean 9, {4,6} n2 mean 1, {5} 9. Adjacent (0,1) =
#     1*64 = 64, (1,4) = 64, (4,5) = 2/3*64; non-adjacent zeros (0,4), (1,5): both taken.
#  step 3, R=2: (0,1) = 4*3/7*64 = 768/7.
# One merge per step: (0,2), (0,4), (0,6), (1,3), (1,5), (0,1).
STRIP_B = [1, 9, 1, 9, 1, 9, 1]


@pytest.mark.parametrize("brute", [False, True])
def test_hand_strip_spectral_storm(brute):
    got = recs(run(strip(STRIP_B), True, brute))
    assert got == [(0, 2, 1, 6, 0.0), (1, 3, 3, 5, 0.0), (4, 6, 3, 4, 0.0), (0, 4, 1, 3, 0.0),
                   (1, 5, 3, 2, 0.0), (0, 1, 0, 1, float(Fraction(768, 7)))]
    one = recs(run(strip(STRIP_B), False, brute))
    assert [g[:4] for g in one] == [(0, 2, 1, 6), (0, 4, 1, 5), (0, 6, 1, 4), (1, 3, 1, 3), (1, 5, 1, 2),
                                    (0, 1, 0, 1)]


@pytest.mark.parametrize("brute", [False, True])
def test_hand_strip_without_spectral_stage(brute):
    # no spectral stage: the identical regions of STRIP_B never merge for being identical; every
    # step is a positive adjacent merge, as with one merge per step
    a = recs(run(strip(STRIP_B), True, brute, w=0.0, kmax=0))
    b = recs(run(strip(STRIP_B), False, brute, w=0.0, kmax=0))
    assert a == b and all(k == 0 for _, _, k, _, _ in a)


def test_rejected_with_two_merges_or_spectral_angle():
    with pytest.raises(ValueError):
        oracle.rhseg(strip(STRIP_A), multi_merge=True, two_merges=True)
    with pytest.raises(ValueError):
        oracle.rhseg(strip(STRIP_A), multi_merge=True, criterion="sam")


GRID = [
    dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=12, rnb_levels=2, section_regions=3),
    dict(connectivity=8, seam_connectivity=8, spclust_wght=0.21, spclust_max=30, rnb_levels=1),
    dict(connectivity=4, seam_connectivity=4, spclust_wght=1.0, spclust_max=40, rnb_levels=2, section_regions=4),
    dict(connectivity=8, seam_connectivity=4, spclust_wght=0.8, spclust_max=9, rnb_levels=3, section_regions=2),
    dict(connectivity=4, seam_connectivity=8, spclust_wght=0.0, spclust_max=0, rnb_levels=2, section_regions=3),
]


def tie_cube(H, W, B, seed):
    """Tie-heavy: values 0..2 in one or two bands, so many pixels are identical."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 3, size=(H, W, B)).astype(np.float32)


@pytest.mark.parametrize("t", range(12))
def test_matches_python_hseg(t):
    p = GRID[t % len(GRID)]
    rng = np.random.default_rng(500 + t)
    H, W = int(rng.integers(4, 8)), int(rng.integers(4, 8))
    B = int(rng.integers(1, 3))
    cube = tie_cube(H, W, B, 90 + t) if t % 4 else synth.random_cube(H, W, B, seed=90 + t, kind="continuous")
    counts = sorted({max(2, H * W // 2), max(2, H * W // 4), 2}, reverse=True)
    kw = dict(p, target_regions=2, level_counts=counts, multi_merge=True)
    res = oracle.rhseg(cube, **kw)
    brute = oracle.rhseg(cube, **kw, brute=True)
    assert np.array_equal(res.log, brute.log) and np.array_equal(res.labels, brute.labels)
    snaps, log = pybrute.rhseg(cube, **kw)
    assert recs(res) == [tuple(x) for x in log]
    for i in range(len(counts)):
        assert np.array_equal(res.labels[i], np.array(snaps[i]))
    check_partition_levels(res.labels, counts)
    if t % 4 == 0:  # tie-free: the rational decisions agree (on the tie cubes, positive values
        # that are equal in exact arithmetic may differ in FP64, which moves the tie-break)
        _, xlog = pybrute.rhseg(cube, **kw, exact=True)
        assert [g[:4] for g in recs(res)] == [tuple(x[:4]) for x in xlog]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tie_free_cube_equals_one_merge(seed):
    # without a zero-valued pair every step is one merge
    cube = synth.random_cube(10, 9, 3, seed=seed)
    p = dict(connectivity=8, seam_connectivity=8, spclust_wght=0.5, spclust_max=40, rnb_levels=2,
             section_regions=6, target_regions=2, level_counts=[30, 8, 2])
    a = oracle.rhseg(cube, **p, multi_merge=True)
    b = oracle.rhseg(cube, **p)
    assert np.array_equal(a.log, b.log) and np.array_equal(a.labels, b.labels)


def partitions_before_positive_merges(log, labels0):
    """Replay a merge log with union-find; before every merge of positive
    value record the partition (as a frozenset of frozensets of labels)."""
    parent = {l: l for l in labels0}

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    out = []
    for m in log:
        if m["d2"] > 0:
            groups = {}
            for l in labels0:
                groups.setdefault(find(l), []).append(l)
            out.append((int(m["lo"]), int(m["hi"]), float(m["d2"]),
                        frozenset(frozenset(g) for g in groups.values())))
        parent[int(m["hi"])] = int(m["lo"])
    return out


@pytest.mark.parametrize("salt,seed", [(0.15, 1), (0.3, 2), (0.0, 3)])
def test_partitions_between_storms_equal_one_merge(salt, seed):
    """HSWO to one region: a zero storm ends, in either reading, once every
    eligible pair of identical regions is merged, which fixes the partition;
    so the positive merges and the partitions before each of them agree with
    the one-merge reading, while the zero merges come in fewer steps."""
    sc = synth.mixer_scene(14, 13, 4, K=5, sigma=0.0, seed=seed, salt=salt)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.6, spclust_max=60, rnb_levels=1,
             target_regions=1, level_counts=[1])
    a = oracle.rhseg(sc.cube, **p, multi_merge=True)
    b = oracle.rhseg(sc.cube, **p)
    labels0 = list(range(14 * 13))
    pa, pb = partitions_before_positive_merges(a.log, labels0), partitions_before_positive_merges(b.log, labels0)
    assert pa == pb and len(pa) > 3
    steps_a = int((a.log["kind"] < 2).sum())
    assert steps_a < len(b.log) and len(a.log) == len(b.log)


def test_log_structure_and_sse_identity():
    """The merges of one step are disjoint and of value 0; a step of several
    merges starts with a merge of kind 0 or 1; the merged values add up to
    each level's SSE (Ward's identity holds whatever the merge order)."""
    sc = synth.mixer_scene(24, 20, 3, K=6, sigma=0.0, seed=11, salt=0.2)
    counts = [150, 60, 12, 3]  # the top pass starts at 4 x 40 = 160 regions
    res = oracle.rhseg(sc.cube, connectivity=4, seam_connectivity=8, spclust_wght=0.6, spclust_max=150,
                       rnb_levels=2, section_regions=40, target_regions=3, level_counts=counts, multi_merge=True)
    log = res.log
    multi_steps = 0
    k = 0
    while k < len(log):
        j = k + 1
        while j < len(log) and log["kind"][j] >= 2:
            j += 1
        assert log["kind"][k] in (0, 1)
        if j - k > 1:
            multi_steps += 1
            step = log[k:j]
            assert (step["d2"] == 0.0).all()
            seen = np.concatenate([step["lo"], step["hi"]])
            assert len(np.unique(seen)) == len(seen)
            assert np.array_equal(step["r_after"], log["r_after"][k] - np.arange(j - k))
        k = j
    assert multi_steps > 5
    cube = sc.cube.astype(np.float64)
    csum = np.concatenate([[0.0], np.cumsum(log["d2"])])
    H, W = sc.cube.shape[:2]
    for i, c in enumerate(counts):
        assert len(np.unique(res.labels[i])) == c
        assert abs(csum[H * W - c] - sse_of_partition(cube, res.labels[i])) <= 1e-9 * (1 + csum[H * W - c])
