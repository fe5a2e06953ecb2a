"""rhseg_segment_noalloc: RHSEG with the library's static device scratch.

CPU: the symbol is exported, and what the entry point refuses (a problem
larger than its scratch, the flags that create graphs or events) is refused
on the host before any device call.
GPU: two calls in a row, the second on a smaller input, give exactly what
rhseg_segment gives with a workspace of its own (label maps at every level,
the merge log and the merge count), in the incremental and the screened
forms.
"""
import ctypes
import sys

import numpy as np
import pytest

from paper_2106_12942_amd import hswo, synth

P = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=300, target_regions=5,
         section_regions=80, level_counts=[300, 64, 5])


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _call(lib, H, W, B, params, L=1):
    p = hswo.make_params(**params, rnb_levels=L)
    # fake, aligned device addresses: the host checks reject the call before any device access
    return lib.rhseg_segment_noalloc(256, H, W, B, hswo.HSWO_F32, ctypes.byref(p), L, 512, None, None, None)


def test_noalloc_symbol_exported():
    assert hasattr(hswo.load(), "rhseg_segment_noalloc")
    assert "rhseg_segment_noalloc" in hswo.EXPORTS


def test_noalloc_rejects_a_problem_beyond_its_scratch_on_the_host():
    lib = hswo.load()
    p = dict(P, level_counts=[5])
    need = hswo.workspace_bytes(1024, 1024, 128, hswo.HSWO_F32, hswo.make_params(**p, rnb_levels=5))
    assert need > hswo.HSWO_NOALLOC_SCRATCH_BYTES
    rc = _call(lib, 1024, 1024, 128, p, L=5)
    assert rc == hswo.HSWO_E_NOMEM
    msg = hswo.last_error()
    assert "rhseg_segment_noalloc" in msg and str(hswo.HSWO_NOALLOC_SCRATCH_BYTES) in msg and str(need) in msg


@pytest.mark.parametrize("flag", ["graph", "autotune", "kernel_times"])
def test_noalloc_rejects_flags_that_create_graphs_or_events(flag):
    rc = _call(hswo.load(), 32, 32, 8, dict(P, level_counts=[5], **{flag: True}))
    assert rc == hswo.HSWO_E_INVAL
    assert "rhseg_segment_noalloc" in hswo.last_error()


def test_noalloc_validates_like_rhseg_segment():
    lib = hswo.load()
    assert _call(lib, 32, 32, 8, dict(P, level_counts=[5], spclust_wght=2.0)) == hswo.HSWO_E_INVAL
    assert _call(lib, 32, 32, 8, dict(P, level_counts=[5]), L=0) == hswo.HSWO_E_INVAL
    assert _call(lib, 0, 32, 8, dict(P, level_counts=[5])) == hswo.HSWO_E_INVAL


def _both(torch, cube_h, L, form):
    kw = dict(P, precision="fp16" if form == "incremental" else form, incremental=form == "incremental")
    cube = torch.from_numpy(cube_h).cuda()
    H, W, _ = cube_h.shape
    ref = hswo.rhseg_segment(cube, rnb_levels=L, merge_log=True, stats=True, **kw)
    labels = torch.full((len(P["level_counts"]), H, W), -1, dtype=torch.int32, device="cuda")
    log_t = torch.zeros(((H * W - P["target_regions"]) * hswo.MERGE_DTYPE.itemsize,), dtype=torch.uint8,
                        device="cuda")
    got = hswo.rhseg_segment_noalloc(cube, labels, rnb_levels=L, merge_log_out=log_t, stats=True, **kw)
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.gpu
@pytest.mark.parametrize("form", ["incremental", "fp16", "fp32"])
def test_noalloc_matches_rhseg_segment_on_two_calls(form):
    torch = pytest.importorskip("torch")
    big = synth.voronoi_scene(160, 144, 48, 24, 25.0, 71).cube
    small = synth.voronoi_scene(96, 80, 32, 12, 25.0, 72).cube
    for tag, cube_h, L in (("first", big, 3), ("second, smaller", small, 2)):
        _say(f"[gpu] noalloc {form} {tag} call {cube_h.shape} L={L}")
        ref, got = _both(torch, cube_h, L, form)
        assert got.stats["merges"] == ref.stats["merges"] == cube_h.shape[0] * cube_h.shape[1] - P["target_regions"]
        assert np.array_equal(got.log, ref.log), f"{tag} call: merge log differs from rhseg_segment's"
        assert torch.equal(got.labels, ref.labels), f"{tag} call: labels differ from rhseg_segment's"
        assert got.stats["ms_total"] == 0.0  # no events in this entry point


@pytest.mark.gpu
def test_noalloc_nonfinite_cube_reported():
    torch = pytest.importorskip("torch")
    cube_h = synth.random_cube(24, 20, 5, seed=3)
    cube_h[4, 5, 1] = np.nan
    cube = torch.from_numpy(cube_h).cuda()
    labels = torch.full((1, 24, 20), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(hswo.HswoError) as ei:
        hswo.rhseg_segment_noalloc(cube, labels, rnb_levels=2, stats=True, **dict(P, level_counts=[5]))
    assert ei.value.code == hswo.HSWO_E_NONFINITE
    torch.cuda.synchronize()
    assert bool((labels == -7).all())
