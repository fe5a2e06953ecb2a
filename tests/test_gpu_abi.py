"""GPU: what the C ABI promises beyond the merges themselves.

* A cube with a NaN or an infinity: the call merges nothing, writes no label,
  and (when it synchronises) returns HSWO_E_NONFINITE.
* Graph replays are keyed on the exact parameters (a weight and its
  neighbouring float are different calls).
* Every execution setting of hswo_tuning, and the autotuner's choice, give
  the oracle's merges and labels.
* HSWO_FLAG_DEBUG_VERIFY_BOUND: every pair a screen passes on to the FP64
  re-check lies inside the certified bounds that screen relies on, for the
  FP32 adjacent screen, the FP32 spectral tiles and the BF16 / FP16
  matrix-core Gram screen.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2106_12942_amd import hswo, synth
from tests.test_gpu_forms import BATCH_P, check_against_oracle, uneven_sections

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


SMALL_P = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=300, target_regions=5,
               section_regions=80, level_counts=[300, 64, 5])


# ---------------------------------------------------------------------------
# non-finite input
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("bad", [float("nan"), float("inf"), float("-inf")])
@pytest.mark.parametrize("incremental", [False, True])
def test_nonfinite_cube_rejected_and_outputs_untouched(dtype, bad, incremental):
    cube = synth.random_cube(24, 20, 5, seed=3)
    cube[7, 11, 2] = bad
    cube[0, 0, 4] = bad
    if dtype == "f16":
        cube = cube.astype(np.float16)
    p = dict(SMALL_P, spclust_max=100, section_regions=30, level_counts=[50, 5])
    _say(f"[gpu] non-finite cube {dtype} {bad} inc={incremental}")
    t = torch.from_numpy(cube).cuda()
    labels = torch.full((2, 24, 20), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(hswo.HswoError) as ei:
        hswo.rhseg_segment(t, rnb_levels=2, stats=True, labels_out=labels, incremental=incremental, **p)
    assert ei.value.code == hswo.HSWO_E_NONFINITE
    assert "2 NaN or infinite" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((labels == -7).all()), "labels written for a non-finite cube"
    # asynchronous call (no stats): no error code, still nothing written
    hswo.rhseg_segment(t, rnb_levels=2, labels_out=labels, incremental=incremental, **p)
    torch.cuda.synchronize()
    assert bool((labels == -7).all())
    # the next call with a finite cube on the same workspace runs normally
    good = synth.random_cube(24, 20, 5, seed=3)
    if dtype == "f16":
        good = good.astype(np.float16)
    res = hswo.rhseg_segment(torch.from_numpy(good).cuda(), rnb_levels=2, stats=True, merge_log=True,
                             incremental=incremental, **p)
    check_against_oracle(good, res.labels.cpu().numpy(), res.log, dict(p, rnb_levels=2), "after non-finite")
    assert res.stats["nonfinite_values"] == 0


def test_nonfinite_section_in_a_batch():
    cubes = uneven_sections(4, seed0=31)
    cubes[2] = cubes[2].copy()
    cubes[2][1, 1, 0] = np.nan
    _say("[gpu] non-finite section in a batch")
    outs = [torch.full((3, c.shape[0], c.shape[1]), -9, dtype=torch.int32, device="cuda") for c in cubes]
    with pytest.raises(hswo.HswoError) as ei:
        hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c in cubes], stats=True, labels_out=outs, **BATCH_P)
    assert ei.value.code == hswo.HSWO_E_NONFINITE
    torch.cuda.synchronize()
    assert all(bool((o == -9).all()) for o in outs)


# ---------------------------------------------------------------------------
# graph cache key
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pair", [(0.0, 1e-7), (0.21, float(np.nextafter(np.float32(0.21), np.float32(1))))])
def test_graph_replays_keyed_on_the_exact_weight(pair):
    """Alternate two weights that print alike with six decimals through one
    workspace and one set of output pointers, each call replayed from its own
    graph; every replay must give that weight's oracle result. (0 turns the
    spectral row cache off, 1e-7 on.)"""
    sc = synth.voronoi_scene(40, 36, 12, 9, 25.0, 77)
    cube = torch.from_numpy(sc.cube).cuda()
    stream = torch.cuda.Stream()
    ws = hswo.Workspace()
    labels = torch.empty((3, 40, 36), dtype=torch.int32, device="cuda")
    refs = {}
    for k, w in enumerate(pair * 3):
        p = dict(SMALL_P, spclust_wght=float(w), spclust_max=200, section_regions=40, level_counts=[200, 40, 5])
        _say(f"[gpu] graph replay {k} w={w!r}")
        res = hswo.rhseg_segment(cube, rnb_levels=2, graph=True, stream=stream, workspace=ws, labels_out=labels,
                                 incremental=True, merge_log=True, **p)
        stream.synchronize()
        if w not in refs:
            refs[w] = oracle.rhseg(sc.cube, **dict(p, rnb_levels=2))
        assert np.array_equal(res.log[: len(refs[w].log)], refs[w].log), f"replay {k} (w={w!r}): merge log differs"
        assert np.array_equal(labels.cpu().numpy(), refs[w].labels), f"replay {k} (w={w!r}): labels differ"


# ---------------------------------------------------------------------------
# execution settings
# ---------------------------------------------------------------------------
TUNING_CASES = [
    ("incremental", dict(wide_max_sections=0)),
    ("incremental", dict(wide_max_sections=1)),
    ("incremental", dict(wide_max_sections=100000, rows_grid=1)),
    ("incremental", dict(wide_max_sections=100000, rows_grid=7)),
    ("incremental", dict(wide_max_sections=100000, rows_grid=1024, hybrid=0)),
    ("incremental", dict(bare_bounds=0)),
    ("incremental", dict(row_matrix=0)),
    ("incremental", dict(row_matrix=1, wide_max_sections=100000, rows_grid=3)),
    ("incremental", dict(bare_bounds=2, wide_max_sections=4)),
    ("fp16", dict(wide_max_sections=100000, wide_groups=1)),
    ("fp16", dict(wide_max_sections=100000, wide_groups=3)),
    ("fp16", dict(wide_max_sections=100000, wide_groups=2048, driver_variant=2)),
    ("bf16", dict(wide_max_sections=0, driver_variant=4)),
    ("fp32", dict(wide_max_sections=4, wide_groups=512)),
]


@pytest.mark.parametrize("case", range(len(TUNING_CASES)))
def test_every_tuning_gives_the_oracle_result(case):
    form, tu = TUNING_CASES[case]
    sc = synth.voronoi_scene(96, 80, 20, 14, 25.0, 57)
    p = dict(SMALL_P)
    _say(f"[gpu] tuning {form} {tu}")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=3, merge_log=True, stats=True,
                             precision="fp16" if form == "incremental" else form, incremental=form == "incremental",
                             tuning=tu, **p)
    for k, v in tu.items():
        assert res.stats["tuning"][k] == v, (k, res.stats["tuning"])
    check_against_oracle(sc.cube, res.labels.cpu().numpy(), res.log, dict(p, rnb_levels=3), f"tuning {form} {tu}")


@pytest.mark.parametrize("form", ["incremental", "fp16"])
def test_autotuner_choice_is_reported_and_exact(form, tmp_path, monkeypatch):
    monkeypatch.setenv("HSWO_TUNE_CACHE", str(tmp_path / "tune.txt"))
    sc = synth.voronoi_scene(128, 128, 24, 20, 25.0, 58)
    p = dict(SMALL_P, level_counts=[500, 64, 5])
    stream = torch.cuda.Stream()
    _say(f"[gpu] autotune {form}")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=3, merge_log=True, stats=True,
                             autotune=True, graph=True, stream=stream,
                             precision="fp16" if form == "incremental" else form, incremental=form == "incremental",
                             **p)
    stream.synchronize()
    tu = res.stats["tuning"]
    assert all(v >= 0 for v in tu.values()), tu
    check_against_oracle(sc.cube, res.labels.cpu().numpy(), res.log, dict(p, rnb_levels=3), f"autotuned {form}")
    lines = (tmp_path / "tune.txt").read_text().split()
    assert len(lines) == 2 and lines[1].count(",") == 6


# ---------------------------------------------------------------------------
# screen error bounds
# ---------------------------------------------------------------------------
def _check_records(rec, stats, tag):
    assert stats["verify_records"] == len(rec) > 0, (stats["verify_records"], len(rec))
    lo_ok = rec["lower"] <= rec["d2"]
    hi_ok = rec["d2"] <= rec["upper"]
    bad = np.nonzero(~(lo_ok & hi_ok))[0]
    assert bad.size == 0, f"{tag}: {bad.size} pairs outside their certified bounds, first {rec[bad[0]]}"
    out = {}
    for st, name in hswo.SCREEN_STAGES.items():
        r = rec[rec["stage"] == st]
        if r.size == 0:
            continue
        pos = r["d2"] > 0
        rel = np.abs(np.sqrt(np.maximum(r["screen"][pos], 0)) - np.sqrt(r["d2"][pos])) / np.sqrt(r["d2"][pos])
        out[name] = dict(pairs=int(r.size), p50=float(np.percentile(rel, 50)) if rel.size else 0.0,
                         p99=float(np.percentile(rel, 99)) if rel.size else 0.0,
                         max=float(rel.max()) if rel.size else 0.0)
    _say(f"[gpu] {tag} screen error (sqrt domain): {out}")
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_screen_bounds_hold_on_a_salt_cube(prec):
    sc = synth.mixer_scene(128, 128, 220, 40, 25.0, 313, salt=0.05)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=1024, target_regions=8,
             section_regions=256, level_counts=[1024, 64, 8])
    _say(f"[gpu] verify bounds 128x128x220 salt prec={prec}")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=2, merge_log=True, stats=True,
                             precision=prec, verify_cap=1 << 24, **p)
    # the 16-bit forms write two records per spectral candidate (FP32 tile and Gram screen): about 8 M here
    assert res.stats["verify_records"] <= 1 << 24, res.stats["verify_records"]
    check_against_oracle(sc.cube, res.labels.cpu().numpy(), res.log, dict(p, rnb_levels=2), f"verify {prec}")
    err = _check_records(res.verify, res.stats, f"salt128 {prec}")
    assert "adjacent_fp32" in err and "spectral_fp32" in err
    if prec != "fp32":
        assert "spectral_16bit" in err
    # the FP32 screens are within 1e-5 of the canonical value for the median pair
    assert err["adjacent_fp32"]["p50"] < 1e-5 and err["spectral_fp32"]["p50"] < 1e-5


def test_screen_fallback_count():
    """A tie storm (identical salt spectra at D2 = 0) makes re-check sets
    larger than screen_topk: those iterations count as fallbacks, and a
    larger screen_topk counts fewer."""
    sc = synth.mixer_scene(64, 64, 32, 12, 25.0, 314, salt=0.2)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=512, target_regions=8,
             section_regions=128, level_counts=[8])
    n = {}
    for k in (1, 8, 100000):
        res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=2, stats=True, precision="bf16",
                                 screen_topk=k, **p)
        n[k] = (res.stats["screen_fallbacks"], res.stats["screen_iterations"])
    _say(f"[gpu] fallbacks by screen_topk {n}")
    assert n[1][1] == n[8][1] == n[100000][1] > 0
    assert n[1][0] >= n[8][0] >= n[100000][0] == 0
    assert n[1][0] > 0
