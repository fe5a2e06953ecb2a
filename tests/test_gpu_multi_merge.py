"""GPU parity of several merges per step for identical regions (a step whose
winner has the value 0 merges a greedy disjoint set of zero-valued pairs:
adjacent pairs by (lo, hi), then, with the spectral stage on, non-adjacent
pairs by (lo, hi)), incremental form, persistent section driver. The GPU
finds the non-adjacent zero pairs as classes of equal FP64 mean rows (hash
sort, exact comparison); merge logs (with the step structure in the kind
field) and every label map must equal the oracle's multi-merge mode bit for
bit: tie-heavy tiny cubes, salt scenes, ragged multi-tile shapes, the batch
entry point and the full 1024 x 1024 x 220 salt workload."""
import numpy as np
import pytest

import oracle
from paper_2106_12942_amd import hswo, synth
from tests.test_gpu_parity import TINY, _say, assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MULTI = dict(multi_merge=True)


def _steps(log):
    """Number of steps of a log (a merge of kind >= 2 continues its step)."""
    return int((np.asarray(log["kind"]) < 2).sum())


@pytest.mark.parametrize("pi", range(len(TINY)))
@pytest.mark.parametrize("kind", ["integer", "continuous"])
def test_tiny_random_cubes(pi, kind):
    rng = np.random.default_rng(830 + pi)
    for trial in range(3):
        H, W = int(rng.integers(4, 14)), int(rng.integers(4, 14))
        B = int(rng.choice([1, 3, 8, 33]))
        p = dict(TINY[pi], **MULTI)
        target = int(rng.integers(1, 4))
        p["target_regions"] = target
        p["level_counts"] = sorted({target, max(target, H * W // 2), max(target, H * W // 5)}, reverse=True)
        cube = synth.random_cube(H, W, B, seed=2100 * pi + trial, kind=kind)
        assert_parity(cube, p, incremental=True, tag=f"multi tiny pi={pi} {kind} trial={trial}")


@pytest.mark.parametrize("w,kmax", [(0.5, 2000), (1.0, 300), (0.3, 120), (0.0, 0)])
def test_salt_scenes(w, kmax):
    """Salt pixels of one spectrum: storms of adjacent and non-adjacent
    zero-valued pairs, at the spectral stage's start and inside it."""
    sc = synth.mixer_scene(44, 40, 12, K=8, sigma=25.0, seed=17, salt=0.2)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=w, spclust_max=kmax, rnb_levels=2,
             section_regions=100, target_regions=5, level_counts=[300, 40, 5], **MULTI)
    stats = assert_parity(sc.cube, p, incremental=True, tag=f"multi salt w={w} kmax={kmax}")
    ref = oracle.rhseg(sc.cube, **p)
    assert stats["iterations"] == _steps(ref.log)
    if w > 0:
        assert _steps(ref.log) < len(ref.log) - 50


@pytest.mark.parametrize("B", [1, 37, 300])
def test_band_counts_and_ragged_shapes(B):
    # integer-valued cube: many regions share a mean row; 300 bands span several hash lanes
    cube = synth.random_cube(37, 29, B, seed=B + 5, kind="integer")
    p = dict(connectivity=8, seam_connectivity=8, spclust_wght=0.7, spclust_max=600, rnb_levels=2,
             section_regions=40, target_regions=3, level_counts=[400, 60, 3], **MULTI)
    assert_parity(cube, p, incremental=True, tag=f"multi integer B={B}")


@pytest.mark.parametrize("H,W", [(1, 1), (1, 9), (7, 1), (2, 2)])
def test_degenerate_shapes(H, W):
    cube = synth.random_cube(H, W, 2, seed=H * 10 + W + 3, kind="integer")
    p = dict(connectivity=8, seam_connectivity=8, spclust_wght=0.9, spclust_max=16, rnb_levels=1,
             target_regions=1, level_counts=[1], **MULTI)
    assert_parity(cube, p, incremental=True, tag=f"multi degenerate {H}x{W}")


def test_constant_cube():
    # every pair has the value 0: the first step takes a maximal matching of the adjacent pairs,
    # then the regions pair off by label
    cube = np.full((16, 12, 3), 5.0, dtype=np.float32)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=200, rnb_levels=2,
             section_regions=10, target_regions=1, level_counts=[40, 1], **MULTI)
    stats = assert_parity(cube, p, incremental=True, tag="multi constant")
    assert stats["iterations"] < 30


def test_batch_matches_oracle_per_section():
    from tests.test_gpu_forms import BATCH_P
    p = dict(BATCH_P, **MULTI)
    cubes = [synth.mixer_scene(int(s), int(s) + 3, 16, K=6, sigma=20.0, seed=s, salt=0.1).cube
             for s in (24, 31, 40, 52)]
    _say(f"[gpu] multi-merge batch of {len(cubes)} shapes={[c.shape for c in cubes]}")
    res = hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c in cubes], merge_log=True, incremental=True, **p)
    torch.cuda.synchronize()
    for i, c in enumerate(cubes):
        ref = oracle.rhseg(c, **p)
        assert np.array_equal(res.logs[i][: len(ref.log)], ref.log), f"section {i}: merge log differs"
        assert np.array_equal(res.labels[i].cpu().numpy(), ref.labels), f"section {i}: labels differ"


def test_rejected_outside_the_incremental_equation_1_form():
    sc = synth.voronoi_scene(8, 8, 3, K=3, sigma=5.0, seed=1)
    t = torch.from_numpy(sc.cube).cuda()
    for kw in (dict(incremental=False), dict(incremental=True, criterion="sam"),
               dict(incremental=True, two_merges=True)):
        with pytest.raises(RuntimeError):
            hswo.rhseg_segment(t, rnb_levels=1, target_regions=2, multi_merge=True, **kw)


def test_workload_rhseg1024_salt_full_parity():
    """The 1024 x 1024 x 220 salt workload (5% identical pixels): the whole
    merge log, with its step structure, and all label maps."""
    from tests.test_gpu_workloads import host_threads
    sc, p = synth.workload("rhseg1024_salt")
    p = dict(p, **MULTI)
    _say("[gpu] rhseg1024_salt multi-merge oracle (CPU)")
    ref = oracle.rhseg(sc.cube, **p, n_threads=host_threads(), progress="rhseg1024_salt multi")
    L = p.pop("rnb_levels")
    _say("[gpu] rhseg1024_salt multi-merge, GPU")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=L, merge_log=True, stats=True,
                             incremental=True, **p)
    torch.cuda.synchronize()
    n = len(ref.log)
    _say(f"[gpu] rhseg1024_salt multi-merge: {n} merges in {_steps(ref.log)} steps, "
         f"{res.stats['ms_total']:.0f} ms")
    assert res.stats["merges"] == n and res.stats["iterations"] == _steps(ref.log)
    got = res.log[:n]
    if not np.array_equal(got, ref.log):
        bad = int(np.nonzero(got != ref.log)[0][0])
        pytest.fail(f"merge log diverges at record {bad}: gpu {got[bad]} oracle {ref.log[bad]}")
    assert np.array_equal(res.labels.cpu().numpy(), ref.labels)
