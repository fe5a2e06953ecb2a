"""GPU parity of the two-merge reading of the HSEG step list (each iteration
merges the least adjacent pair, then the least non-adjacent pair of the
resulting partition if it is below w^2 times the first merge's value),
incremental form: the spectral step takes a masked minimum (adjacency bitmap
of the live slots, rebuilt after every merge of the spectral stage). Merge
logs and labels must equal the oracle's two-merge mode bit for bit, in both
level modes, across the persistent-to-wide hand-over and in the batched
entry point."""
import numpy as np
import pytest

import oracle
from paper_2106_12942_amd import hswo, synth
from tests.test_gpu_parity import TINY, _say, assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MODES = ["persistent", "wide"]
TWO = dict(two_merges=True)


def _mode(monkeypatch, mode):
    monkeypatch.setattr(hswo, "DEFAULT_TUNING", {"wide_max_sections": 0 if mode == "persistent" else 100000})


def _spectral_merges(cube, p):
    return int(oracle.rhseg(cube, **p).log["kind"].sum())


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("pi", range(len(TINY)))
def test_tiny_random_cubes(pi, mode, monkeypatch):
    _mode(monkeypatch, mode)
    rng = np.random.default_rng(270 + pi)
    for trial in range(3):
        H, W = int(rng.integers(4, 14)), int(rng.integers(4, 14))
        B = int(rng.choice([1, 3, 8, 33]))
        p = dict(TINY[pi], **TWO)
        target = int(rng.integers(1, 4))
        p["target_regions"] = target
        p["level_counts"] = sorted({target, max(target, H * W // 2), max(target, H * W // 5)}, reverse=True)
        cube = synth.random_cube(H, W, B, seed=1100 * pi + trial, kind="integer" if trial == 1 else "continuous")
        assert_parity(cube, p, incremental=True, tag=f"two tiny pi={pi} {mode} trial={trial}")


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("B", [1, 37, 300])
def test_band_counts(B, mode, monkeypatch):
    _mode(monkeypatch, mode)
    sc = synth.voronoi_scene(36, 30, B, K=9, sigma=25.0, seed=B + 1)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=500, rnb_levels=2,
             section_regions=60, target_regions=3, level_counts=[240, 30, 3], **TWO)
    assert_parity(sc.cube, p, incremental=True, tag=f"two B={B} {mode}")


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("kmax", [150, 400])
def test_spectral_stage_entry(kmax, mode, monkeypatch):
    """Step 3 starting mid-pass, at the hand-over from the persistent driver
    (which runs the iterations before the spectral stage) to the wide
    kernels, and at parent passes that start inside the stage."""
    _mode(monkeypatch, mode)
    sc = synth.voronoi_scene(64, 56, 24, K=14, sigma=25.0, seed=kmax + 1)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=kmax, rnb_levels=3,
             section_regions=80, target_regions=5, level_counts=[300, 64, 5], **TWO)
    assert _spectral_merges(sc.cube, p) > 0
    assert_parity(sc.cube, p, incremental=True, tag=f"two entry kmax={kmax} {mode}")


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("w", [1.0, 0.3])
def test_salt_ties(w, mode, monkeypatch):
    _mode(monkeypatch, mode)
    sc = synth.mixer_scene(40, 40, 12, K=8, sigma=25.0, seed=7, salt=0.2)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=w, spclust_max=1600, rnb_levels=2,
             section_regions=100, target_regions=5, level_counts=[300, 40, 5], **TWO)
    assert_parity(sc.cube, p, incremental=True, tag=f"two salt w={w} {mode}")


@pytest.mark.parametrize("mode", MODES)
def test_spectral_angle(mode, monkeypatch):
    _mode(monkeypatch, mode)
    sc = synth.voronoi_scene(48, 40, 16, K=10, sigma=25.0, seed=12)
    p = dict(connectivity=8, seam_connectivity=8, spclust_wght=0.6, spclust_max=300, rnb_levels=2,
             section_regions=60, target_regions=4, level_counts=[150, 20, 4], criterion="sam", **TWO)
    assert_parity(sc.cube, p, incremental=True, tag=f"two sam {mode}")


def test_hybrid_levels_off(monkeypatch):
    monkeypatch.setattr(hswo, "DEFAULT_TUNING", {"hybrid": 0})
    sc = synth.voronoi_scene(48, 40, 16, K=10, sigma=25.0, seed=3)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=120, rnb_levels=2,
             section_regions=50, target_regions=4, level_counts=[200, 4], **TWO)
    assert_parity(sc.cube, p, incremental=True, tag="two hybrid off")


@pytest.mark.parametrize("H,W", [(1, 1), (1, 9), (7, 1), (2, 2)])
def test_degenerate_shapes(H, W):
    cube = synth.random_cube(H, W, 3, seed=H * 10 + W + 1)
    p = dict(connectivity=8, seam_connectivity=8, spclust_wght=0.9, spclust_max=16, rnb_levels=1,
             target_regions=1, level_counts=[1], **TWO)
    assert_parity(cube, p, incremental=True, tag=f"two degenerate {H}x{W}")


def test_sequential_sections():
    sc = synth.voronoi_scene(40, 40, 8, K=8, sigma=25.0, seed=21)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=200, rnb_levels=2,
             section_regions=50, target_regions=4, level_counts=[100, 4], **TWO)
    _say("[gpu] two-merge sequential sections")
    t = torch.from_numpy(sc.cube).cuda()
    kw = {k: v for k, v in p.items() if k != "rnb_levels"}
    a = hswo.rhseg_segment(t, rnb_levels=2, incremental=True, sequential=True, merge_log=True, **kw)
    b = hswo.rhseg_segment(t, rnb_levels=2, incremental=True, merge_log=True, **kw)
    torch.cuda.synchronize()
    assert torch.equal(a.labels, b.labels)
    assert np.array_equal(a.log, b.log)


def test_batch_matches_oracle_per_section():
    from tests.test_gpu_forms import BATCH_P, uneven_sections
    p = dict(BATCH_P, **TWO)
    cubes = uneven_sections(8, seed0=6161)
    _say(f"[gpu] two-merge batch of {len(cubes)} shapes={[c.shape for c in cubes]}")
    res = hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c in cubes], merge_log=True, incremental=True, **p)
    torch.cuda.synchronize()
    for i, c in enumerate(cubes):
        ref = oracle.rhseg(c, **p)
        assert np.array_equal(res.logs[i][: len(ref.log)], ref.log), f"section {i}: merge log differs"
        assert np.array_equal(res.labels[i].cpu().numpy(), ref.labels), f"section {i}: labels differ"


def test_workload_rhseg512_full_parity():
    sc, p = synth.workload("rhseg512")
    p = dict(p, **TWO)
    stats = assert_parity(sc.cube, p, incremental=True, tag="two rhseg512 full")
    assert stats["merges"] == 512 * 512 - 8
