"""GPU parity of the spectral angle criterion (Section 4.1 lists the
spectral angle mapper among the dissimilarities HSEG can use), incremental
form: per-edge cache of the exact value for the adjacent stage and the
spectral row cache over band-sum rows and their squared norms. Merge logs
(with the FP64 criterion value) and labels must equal the oracle's bit for
bit, in both level modes and in the batched entry point."""
import numpy as np
import pytest

import oracle
from paper_2106_12942_amd import hswo, synth
from tests.test_gpu_parity import TINY, _say, assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MODES = ["persistent", "wide"]
SAM = dict(criterion="sam")


def _mode(monkeypatch, mode):
    monkeypatch.setattr(hswo, "DEFAULT_TUNING", {"wide_max_sections": 0 if mode == "persistent" else 100000})


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("pi", range(len(TINY)))
def test_tiny_random_cubes(pi, mode, monkeypatch):
    _mode(monkeypatch, mode)
    rng = np.random.default_rng(170 + pi)
    for trial in range(3):
        H, W = int(rng.integers(4, 14)), int(rng.integers(4, 14))
        B = int(rng.choice([1, 2, 3, 8, 33]))
        p = dict(TINY[pi], **SAM)
        target = int(rng.integers(1, 4))
        p["target_regions"] = target
        p["level_counts"] = sorted({target, max(target, H * W // 2), max(target, H * W // 5)}, reverse=True)
        cube = synth.random_cube(H, W, B, seed=900 * pi + trial, kind="integer" if trial == 1 else "continuous")
        assert_parity(cube, p, incremental=True, tag=f"sam tiny pi={pi} {mode} trial={trial}")


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("B", [1, 37, 257, 300])
def test_band_counts(B, mode, monkeypatch):
    """Band counts around the 8-band groups and the 256-band chunks of the
    common summation tree, for the dot product and the squared norms."""
    _mode(monkeypatch, mode)
    sc = synth.voronoi_scene(36, 30, B, K=9, sigma=25.0, seed=B)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=500, rnb_levels=2,
             section_regions=60, target_regions=3, level_counts=[240, 30, 3], **SAM)
    assert_parity(sc.cube, p, incremental=True, tag=f"sam B={B} {mode}")


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("kmax", [150, 400])
def test_spectral_stage_entry(kmax, mode, monkeypatch):
    _mode(monkeypatch, mode)
    sc = synth.voronoi_scene(64, 56, 24, K=14, sigma=25.0, seed=kmax)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=kmax, rnb_levels=3,
             section_regions=80, target_regions=5, level_counts=[300, 64, 5], **SAM)
    assert_parity(sc.cube, p, incremental=True, tag=f"sam entry kmax={kmax} {mode}")


@pytest.mark.parametrize("mode", MODES)
def test_salt_ties(mode, monkeypatch):
    """Identical salt spectra: exact zero values and their label tie-break."""
    _mode(monkeypatch, mode)
    sc = synth.mixer_scene(40, 40, 12, K=8, sigma=25.0, seed=7, salt=0.2)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=1.0, spclust_max=1600, rnb_levels=2,
             section_regions=100, target_regions=5, level_counts=[300, 40, 5], **SAM)
    assert_parity(sc.cube, p, incremental=True, tag=f"sam salt {mode}")


def test_signed_and_zero_spectra():
    """Mixed-sign data (obtuse angles, the 1 + t branch) with some all-zero
    pixels (the zero-spectrum value 1)."""
    cube = synth.random_cube(20, 18, 5, seed=5)
    cube[::4, ::3, :] = 0.0
    p = dict(connectivity=8, seam_connectivity=8, spclust_wght=0.3, spclust_max=200, rnb_levels=2,
             section_regions=40, target_regions=2, level_counts=[100, 10, 2], **SAM)
    assert_parity(cube, p, incremental=True, tag="sam signed/zero")


def test_hybrid_levels_off(monkeypatch):
    monkeypatch.setattr(hswo, "DEFAULT_TUNING", {"hybrid": 0})
    sc = synth.voronoi_scene(48, 40, 16, K=10, sigma=25.0, seed=3)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=120, rnb_levels=2,
             section_regions=50, target_regions=4, level_counts=[200, 4], **SAM)
    assert_parity(sc.cube, p, incremental=True, tag="sam hybrid off")


@pytest.mark.parametrize("H,W", [(1, 1), (1, 9), (7, 1), (2, 2)])
def test_degenerate_shapes(H, W):
    cube = synth.random_cube(H, W, 3, seed=H * 10 + W)
    p = dict(connectivity=8, seam_connectivity=8, spclust_wght=0.5, spclust_max=16, rnb_levels=1,
             target_regions=1, level_counts=[1], **SAM)
    assert_parity(cube, p, incremental=True, tag=f"sam degenerate {H}x{W}")


def test_batch_matches_oracle_per_section():
    from tests.test_gpu_forms import BATCH_P, uneven_sections
    p = dict(BATCH_P, **SAM)
    cubes = uneven_sections(8, seed0=5151)
    _say(f"[gpu] sam batch of {len(cubes)} shapes={[c.shape for c in cubes]}")
    res = hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c in cubes], merge_log=True, incremental=True, **p)
    torch.cuda.synchronize()
    for i, c in enumerate(cubes):
        ref = oracle.rhseg(c, **p)
        assert np.array_equal(res.logs[i][: len(ref.log)], ref.log), f"section {i}: merge log differs"
        assert np.array_equal(res.labels[i].cpu().numpy(), ref.labels), f"section {i}: labels differ"


def test_workload_rhseg512_full_parity():
    """The 512 x 512 x 128 four-level workload under the spectral angle."""
    sc, p = synth.workload("rhseg512")
    p = dict(p, **SAM)
    stats = assert_parity(sc.cube, p, incremental=True, tag="sam rhseg512 full")
    assert stats["merges"] == 512 * 512 - 8
    _say(f"[gpu] sam rhseg512: {stats['ms_total'] if 'ms_total' in stats else stats}")
