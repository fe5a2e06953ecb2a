"""GPU: the batching form (hswo_run_batch), hipGraph capture and replay,
the autotuner, and every section-driver variant -- all against the FP64
oracle, since none of them may change a single label or merge."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2106_12942_amd import hswo, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


BATCH_P = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=300, target_regions=20,
               section_regions=0, level_counts=[100, 50, 20])


def uneven_sections(n, seed0=4040):
    out = []
    for s in range(n):
        rng = np.random.default_rng(seed0 + s)
        side_h = int(rng.integers(8, 41))
        side_w = int(rng.integers(8, 41))
        B = int(rng.choice([8, 32, 64, 96]))
        K = int(rng.integers(3, 12))
        out.append(synth.voronoi_scene(side_h, side_w, B, K, 30.0, seed0 + s).cube)
    return out


def check_against_oracle(cube, lab, log, p, tag):
    ref = oracle.rhseg(cube, **p)
    assert np.array_equal(log[: len(ref.log)], ref.log), f"{tag}: merge log differs"
    assert np.array_equal(lab, ref.labels), f"{tag}: labels differ"


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_batch_matches_oracle_per_section(prec):
    cubes = uneven_sections(12)
    _say(f"[gpu] batch of {len(cubes)} uneven sections prec={prec} shapes={[c.shape for c in cubes]}")
    res = hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c in cubes], precision=prec, merge_log=True,
                              stats=True, **BATCH_P)
    torch.cuda.synchronize()
    for i, c in enumerate(cubes):
        check_against_oracle(c, res.labels[i].cpu().numpy(), res.logs[i], BATCH_P, f"section {i}")
    assert res.stats["driver_launches"] == 1


def test_batch_f16_sections():
    cubes = [synth.mixer_scene(24 + 3 * s, 20 + 2 * s, 16, 6, 25.0, 600 + s, dtype="f16").cube for s in range(5)]
    _say("[gpu] batch f16 sections")
    res = hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c in cubes], precision="fp16", merge_log=True,
                              **BATCH_P)
    torch.cuda.synchronize()
    for i, c in enumerate(cubes):
        check_against_oracle(c, res.labels[i].cpu().numpy(), res.logs[i], BATCH_P, f"f16 section {i}")


def test_batch_equals_individual_runs():
    cubes = uneven_sections(6, seed0=777)
    _say("[gpu] batch vs individual hswo_run")
    dc = [torch.from_numpy(c).cuda() for c in cubes]
    res = hswo.hswo_run_batch(dc, precision="fp16", **BATCH_P)
    for i, c in enumerate(dc):
        one = hswo.hswo_run(c, precision="fp32", **BATCH_P)
        assert torch.equal(one.labels, res.labels[i])


@pytest.mark.parametrize("variant", [2, 4, 6])
def test_driver_variants_identical(variant, monkeypatch):
    sc = synth.voronoi_scene(48, 48, 40, 15, 25.0, 31)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=400, target_regions=4,
             section_regions=100, level_counts=[300, 40, 4])
    monkeypatch.setattr(hswo, "DEFAULT_TUNING", {"driver_variant": variant})
    _say(f"[gpu] driver variant {variant}")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=2, precision="fp16", merge_log=True,
                             stats=True, **p)
    assert res.stats["driver_variant"] == variant
    check_against_oracle(sc.cube, res.labels.cpu().numpy(), res.log, dict(p, rnb_levels=2), f"variant {variant}")


def test_autotune_chooses_a_variant_and_keeps_results(tmp_path, monkeypatch):
    monkeypatch.setenv("HSWO_TUNE_CACHE", str(tmp_path / "tune.txt"))
    cubes = uneven_sections(5, seed0=999)
    _say("[gpu] autotune batch")
    dc = [torch.from_numpy(c).cuda() for c in cubes]
    res = hswo.hswo_run_batch(dc, precision="fp16", autotune=True, merge_log=True, stats=True, **BATCH_P)
    torch.cuda.synchronize()
    assert res.stats["driver_variant"] in (2, 4, 6)
    for i, c in enumerate(cubes):
        check_against_oracle(c, res.labels[i].cpu().numpy(), res.logs[i], BATCH_P, f"tuned section {i}")
    # the cache line holds the settings in hswo_tuning order; the sixth is the driver variant
    fields = (tmp_path / "tune.txt").read_text().strip().split()[-1].split(",")
    assert int(fields[5]) == res.stats["driver_variant"]


def test_graph_replays_match_eager():
    """Capture once, replay several times with other eager work in between;
    every replay must equal the eager result."""
    sc = synth.voronoi_scene(64, 64, 24, 12, 25.0, 71)
    other = synth.voronoi_scene(40, 40, 24, 8, 25.0, 72)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=256, target_regions=6,
             section_regions=64, level_counts=[200, 30, 6])
    stream = torch.cuda.Stream()
    cube = torch.from_numpy(sc.cube).cuda()
    cube2 = torch.from_numpy(other.cube).cuda()
    ref = oracle.rhseg(sc.cube, **p, rnb_levels=2)
    ws = hswo.Workspace()
    with torch.cuda.stream(stream):
        eager = hswo.rhseg_segment(cube, rnb_levels=2, precision="fp16", stream=stream, **p)
        stream.synchronize()
        assert np.array_equal(eager.labels.cpu().numpy(), ref.labels)
        out = torch.empty_like(eager.labels)
        for k in range(4):
            _say(f"[gpu] graph replay {k}")
            out.fill_(-7)
            g = hswo.rhseg_segment(cube, rnb_levels=2, precision="fp16", graph=True, stream=stream, workspace=ws,
                                   labels_out=out, **p)
            stream.synchronize()
            assert np.array_equal(g.labels.cpu().numpy(), ref.labels), f"replay {k} differs"
            # unrelated eager work on the same stream between replays
            hswo.rhseg_segment(cube2, rnb_levels=1, precision="fp32", stream=stream,
                               **dict(p, level_counts=[6], target_regions=6))
            stream.synchronize()


def test_graph_batch_replays():
    cubes = uneven_sections(8, seed0=1234)
    stream = torch.cuda.Stream()
    dc = [torch.from_numpy(c).cuda() for c in cubes]
    ws = hswo.Workspace()
    with torch.cuda.stream(stream):
        eager = hswo.hswo_run_batch(dc, precision="fp16", stream=stream, **BATCH_P)
        stream.synchronize()
        outs = [torch.empty_like(t) for t in eager.labels]
        for k in range(3):
            _say(f"[gpu] batch graph replay {k}")
            for o in outs:
                o.fill_(-7)
            hswo.hswo_run_batch(dc, precision="fp16", graph=True, stream=stream, workspace=ws, labels_out=outs,
                                **BATCH_P)
            stream.synchronize()
            for a, b in zip(eager.labels, outs):
                assert torch.equal(a, b), f"batch replay {k} differs"


@pytest.mark.parametrize("mode", ["persistent", "wide"])
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_level_modes_identical(mode, prec, monkeypatch):
    """Every level run by the persistent driver, or every level in wide mode
    (G workgroups per section, one launch sequence per iteration)."""
    monkeypatch.setattr(hswo, "DEFAULT_TUNING", {"wide_max_sections": 0 if mode == "persistent" else 100000})
    sc = synth.voronoi_scene(96, 80, 20, 14, 25.0, 55)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=300, target_regions=5,
             section_regions=80, level_counts=[300, 64, 5])
    _say(f"[gpu] level mode {mode} prec={prec}")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=3, precision=prec, merge_log=True,
                             stats=True, **p)
    check_against_oracle(sc.cube, res.labels.cpu().numpy(), res.log, dict(p, rnb_levels=3), f"{mode}/{prec}")


@pytest.mark.parametrize("mode", ["persistent", "wide"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_incremental_adjacent_identical(mode, prec, monkeypatch):
    """Cached exact per-edge D2, re-scoring only what a merge changed: the
    same merges and labels as the full sweep (and the oracle)."""
    monkeypatch.setattr(hswo, "DEFAULT_TUNING", {"wide_max_sections": 0 if mode == "persistent" else 100000})
    sc = synth.voronoi_scene(96, 80, 20, 14, 25.0, 56)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=300, target_regions=5,
             section_regions=80, level_counts=[300, 64, 5])
    _say(f"[gpu] incremental {mode} prec={prec}")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=3, precision=prec, merge_log=True,
                             incremental=True, stats=True, **p)
    check_against_oracle(sc.cube, res.labels.cpu().numpy(), res.log, dict(p, rnb_levels=3), f"inc {mode}/{prec}")


def test_incremental_batch_and_salt():
    cubes = uneven_sections(6, seed0=4321)
    _say("[gpu] incremental batch")
    res = hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c in cubes], precision="fp16", merge_log=True,
                              incremental=True, **BATCH_P)
    torch.cuda.synchronize()
    for i, c in enumerate(cubes):
        check_against_oracle(c, res.labels[i].cpu().numpy(), res.logs[i], BATCH_P, f"inc section {i}")
    sc = synth.mixer_scene(40, 40, 12, K=8, sigma=25.0, seed=7, salt=0.05)
    p = dict(connectivity=8, seam_connectivity=8, spclust_wght=0.5, spclust_max=400, rnb_levels=2,
             section_regions=100, target_regions=5, level_counts=[300, 40, 5])
    _say("[gpu] incremental salt ties")
    r = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=2, precision="fp16", merge_log=True,
                           incremental=True, **{k: v for k, v in p.items() if k != "rnb_levels"})
    check_against_oracle(sc.cube, r.labels.cpu().numpy(), r.log, p, "inc salt")


@pytest.mark.parametrize("form", ["fp32", "incremental"])
def test_sequential_sections_identical(form):
    """Sections of a level one after another, each with the whole device: the
    same merges and labels as the batched levels (and the oracle)."""
    sc = synth.voronoi_scene(64, 56, 24, 14, 25.0, 57)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=300, target_regions=5,
             section_regions=80, level_counts=[300, 64, 5])
    _say(f"[gpu] sequential sections {form}")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=3, precision="fp32", merge_log=True,
                             incremental=form == "incremental", sequential=True, stats=True, **p)
    check_against_oracle(sc.cube, res.labels.cpu().numpy(), res.log, dict(p, rnb_levels=3), f"sequential {form}")
    cubes = uneven_sections(5, seed0=5151)
    res = hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c in cubes], precision="fp32", merge_log=True,
                              incremental=form == "incremental", sequential=True, **BATCH_P)
    torch.cuda.synchronize()
    for i, c in enumerate(cubes):
        check_against_oracle(c, res.labels[i].cpu().numpy(), res.logs[i], BATCH_P, f"sequential batch {i}")


@pytest.mark.parametrize("variant", [dict(), dict(criterion="sam"), dict(two_merges=True)],
                         ids=["incremental", "sam", "two_merges"])
def test_graph_replays_incremental_variants(variant):
    """The incremental form and its variants, captured once and replayed
    three times with other eager work in between (which reuses the
    workspace-independent state of the library); every replay must equal the
    oracle. The section state that carries across launches -- cached
    minimum, row cache, the two-merge step -- starts afresh on each replay."""
    sc = synth.voronoi_scene(64, 64, 24, 12, 25.0, 73)
    other = synth.voronoi_scene(40, 40, 24, 8, 25.0, 74)
    p = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.6, spclust_max=300, target_regions=6,
             section_regions=64, level_counts=[200, 30, 6], **variant)
    ref = oracle.rhseg(sc.cube, **p, rnb_levels=2)
    stream = torch.cuda.Stream()
    cube = torch.from_numpy(sc.cube).cuda()
    cube2 = torch.from_numpy(other.cube).cuda()
    ws = hswo.Workspace()
    with torch.cuda.stream(stream):
        out = torch.empty((len(p["level_counts"]), 64, 64), dtype=torch.int32, device="cuda")
        for k in range(3):
            _say(f"[gpu] incremental graph replay {k} {variant}")
            out.fill_(-7)
            hswo.rhseg_segment(cube, rnb_levels=2, incremental=True, graph=True, stream=stream, workspace=ws,
                               labels_out=out, **p)
            stream.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref.labels), f"replay {k} differs"
            hswo.rhseg_segment(cube2, rnb_levels=2, incremental=True, stream=stream, **p)  # eager work between
            stream.synchronize()
