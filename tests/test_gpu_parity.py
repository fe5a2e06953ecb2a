"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Labels must be identical at every requested level and the merge logs equal
record by record, with the FP64 criterion bit-equal (both sides evaluate the
same canonical operation order). Inputs are seeded synthetic cubes.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2106_12942_amd import hswo, synth
from tests.invariants import check_partition_levels

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_run(cube, params, entry="rhseg", precision="fp32", incremental=False):
    t = torch.from_numpy(np.ascontiguousarray(cube)).cuda()
    p = dict(params)
    L = p.pop("rnb_levels", 1)
    if entry == "hswo":
        res = hswo.hswo_run(t, **p, precision=precision, merge_log=True, stats=True, incremental=incremental)
    else:
        res = hswo.rhseg_segment(t, rnb_levels=L, **p, precision=precision, merge_log=True, stats=True,
                                 incremental=incremental)
    torch.cuda.synchronize()
    return res.labels.cpu().numpy(), res.log, res.stats


def assert_parity(cube, params, entry="rhseg", precision="fp32", tag="", incremental=False):
    _say(f"[gpu] {tag} shape={cube.shape} dtype={cube.dtype} entry={entry} prec={precision} inc={incremental} "
         f"params={params}")
    lab, log, stats = gpu_run(cube, params, entry, precision, incremental)
    ref = oracle.rhseg(cube, **params)
    n = len(ref.log)
    assert stats["merges"] == n
    got = log[:n]
    if not np.array_equal(got, ref.log):
        bad = int(np.nonzero(got != ref.log)[0][0])
        pytest.fail(f"{tag}: merge log diverges at record {bad}: gpu {got[bad]} oracle {ref.log[bad]}")
    for li in range(lab.shape[0]):
        assert np.array_equal(lab[li], ref.labels[li]), f"{tag}: level {li} labels differ"
    check_partition_levels(lab, params["level_counts"])
    return stats


TINY = [
    dict(connectivity=4, seam_connectivity=8, spclust_wght=0.0, spclust_max=0, rnb_levels=1),
    dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=40, rnb_levels=1),
    dict(connectivity=8, seam_connectivity=8, spclust_wght=1.0, spclust_max=1000, rnb_levels=1),
    dict(connectivity=4, seam_connectivity=8, spclust_wght=0.15, spclust_max=30, rnb_levels=2, section_regions=6),
    dict(connectivity=8, seam_connectivity=4, spclust_wght=0.5, spclust_max=24, rnb_levels=3, section_regions=3),
    dict(connectivity=4, seam_connectivity=4, spclust_wght=0.21, spclust_max=60, rnb_levels=2, section_regions=10),
]


PRECS = ["fp32", "bf16", "fp16"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("pi", range(len(TINY)))
@pytest.mark.parametrize("kind", ["continuous", "integer"])
def test_tiny_random_cubes(pi, kind, prec):
    rng = np.random.default_rng(10 + pi)
    for trial in range(4):
        H, W = int(rng.integers(4, 14)), int(rng.integers(4, 14))
        B = int(rng.choice([1, 3, 8, 33]))
        p = dict(TINY[pi])
        target = int(rng.integers(1, 4))
        p["target_regions"] = target
        p["level_counts"] = sorted({target, max(target, H * W // 2), max(target, H * W // 5)}, reverse=True)
        cube = synth.random_cube(H, W, B, seed=100 * pi + trial, kind=kind)
        assert_parity(cube, p, precision=prec, tag=f"tiny pi={pi} kind={kind} trial={trial}")


def test_hswo_entry_point_matches():
    cube = synth.random_cube(9, 11, 5, seed=3)
    p = dict(TINY[1], target_regions=2, level_counts=[50, 10, 2])
    assert_parity(cube, p, entry="hswo", tag="hswo entry")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("H,W,B,kmax", [(40, 37, 7, 600), (33, 65, 3, 1500), (70, 70, 16, 300)])
def test_multi_tile_ragged(H, W, B, kmax, prec):
    """Spectral stage over several 64-wide tiles with a ragged tail."""
    sc = synth.voronoi_scene(H, W, B, K=12, sigma=25.0, seed=H * W + B)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=kmax, rnb_levels=1,
             target_regions=3, level_counts=[kmax, 64, 3])
    assert_parity(sc.cube, p, precision=prec, tag=f"multi-tile {H}x{W}x{B} kmax={kmax}")


@pytest.mark.parametrize("prec", PRECS)
def test_float16_cube(prec):
    sc = synth.mixer_scene(48, 40, 24, K=10, sigma=25.0, seed=5, dtype="f16")
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=200, rnb_levels=2,
             section_regions=64, target_regions=4, level_counts=[200, 50, 4])
    assert_parity(sc.cube, p, precision=prec, tag="f16 mixer")


@pytest.mark.parametrize("prec", PRECS)
def test_salt_ties(prec):
    """Identical salt spectra: exact zero-D2 ties decided by (lo, hi)."""
    sc = synth.mixer_scene(40, 40, 12, K=8, sigma=25.0, seed=7, salt=0.05)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=400, rnb_levels=2,
             section_regions=100, target_regions=5, level_counts=[300, 40, 5])
    assert_parity(sc.cube, p, precision=prec, tag="salt ties")


@pytest.mark.parametrize("H,W", [(1, 1), (1, 9), (7, 1), (2, 2)])
def test_degenerate_shapes(H, W):
    cube = synth.random_cube(H, W, 3, seed=H * 10 + W)
    p = dict(connectivity=8, seam_connectivity=8, spclust_wght=0.5, spclust_max=16, rnb_levels=1,
             target_regions=1, level_counts=[1])
    assert_parity(cube, p, tag=f"degenerate {H}x{W}")


def test_no_merges_when_target_is_pixel_count():
    cube = synth.random_cube(5, 6, 2, seed=9)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=16, rnb_levels=1,
             target_regions=30, level_counts=[30])
    assert_parity(cube, p, tag="no merges")


def test_deterministic_repeat():
    sc, p = synth.workload("hswo64")
    _say("[gpu] determinism hswo64 x2")
    a = gpu_run(sc.cube, p)
    b = gpu_run(sc.cube, p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("prec", PRECS)
def test_workload_hswo64_full_parity(prec):
    sc, p = synth.workload("hswo64")
    stats = assert_parity(sc.cube, p, entry="hswo", precision=prec, tag="hswo64 full")
    assert stats["merges"] == 64 * 64 - 2
    if prec != "fp32":
        assert stats["mfma_tiles"] > 0


@pytest.mark.parametrize("prec", PRECS)
def test_workload_rhseg512_full_parity(prec):
    sc, p = synth.workload("rhseg512")
    stats = assert_parity(sc.cube, p, precision=prec, tag="rhseg512 full")
    assert stats["merges"] == 512 * 512 - 8
    _say(f"[gpu] rhseg512 {prec}: {stats}")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("B", [1000, 4096])
def test_wide_band_counts(B, prec):
    """The screened and plain forms at band counts up to the maximum (4096)."""
    sc = synth.voronoi_scene(10, 9, B, K=4, sigma=25.0, seed=B + 3)
    p = dict(connectivity=8, seam_connectivity=8, spclust_wght=0.5, spclust_max=90, rnb_levels=2,
             section_regions=12, target_regions=2, level_counts=[30, 2])
    assert_parity(sc.cube, p, precision=prec, tag=f"wide bands B={B} {prec}")
