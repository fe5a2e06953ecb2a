"""GPU parity at the benchmark workloads' full sizes.

* rhseg1024_salt (1024 x 1024 x 220, 5% identical salt pixels, L = 5): the
  whole merge log and every label map against the oracle, for the
  incremental form and the BF16 matrix-core screened form.
* rhseg2048_f16 (2048 x 2048 x 224 float16, L = 5, incremental form): the GPU runs the whole
  image; the oracle, which would take minutes, checks a sample that is exact
  on its own: the top-left 1024 x 1024 quadrant. Below the top pass that
  quadrant's sections are independent of the rest, so the oracle run on the
  quadrant alone (four levels, stopping at the section count) must produce
  exactly the GPU's merges inside it, in the same order. The full label maps
  are checked for the properties every level must have.
* batch256 (256 uneven independent sections): sampled sections against the
  oracle, all sections against the partition properties.
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


_C3_REF = {}


def _c3_reference():
    if "ref" not in _C3_REF:
        sc, p = synth.workload("rhseg1024_salt")
        _say("[gpu] rhseg1024_salt oracle (CPU)")
        _C3_REF["ref"] = (sc, p, oracle.rhseg(sc.cube, **p))
    return _C3_REF["ref"]


@pytest.mark.parametrize("form", ["incremental", "bf16"])
def test_rhseg1024_salt_full_parity(form):
    sc, p, ref = _c3_reference()
    L = p["rnb_levels"]
    kw = {k: v for k, v in p.items() if k != "rnb_levels"}
    _say(f"[gpu] rhseg1024_salt full size, form {form}")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=L, merge_log=True, stats=True,
                             precision="fp16" if form == "incremental" else form, incremental=form == "incremental",
                             **kw)
    torch.cuda.synchronize()
    _say(f"[gpu] rhseg1024_salt stats {res.stats}")
    assert np.array_equal(res.log[: len(ref.log)], ref.log)
    assert np.array_equal(res.labels.cpu().numpy(), ref.labels)


def test_rhseg2048_f16_quadrant_parity():
    sc, p = synth.workload("rhseg2048_f16")
    L = p["rnb_levels"]
    kw = {k: v for k, v in p.items() if k != "rnb_levels"}
    H, W, _ = sc.cube.shape
    _say("[gpu] rhseg2048_f16 full size, incremental form")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=L, merge_log=True, stats=True,
                             incremental=True, **kw)
    torch.cuda.synchronize()
    _say(f"[gpu] rhseg2048_f16 stats {res.stats}")
    lab = res.labels.cpu().numpy()
    check_partition_levels(lab, p["level_counts"])
    assert res.stats["merges"] == H * W - p["target_regions"]
    # top-left quadrant, below the top pass
    S = p["section_regions"]
    top_merges = 4 * S - p["target_regions"]
    log = res.log[: len(res.log) - top_merges]
    r, c = log["lo"] // W, log["lo"] % W
    inq = (r < H // 2) & (c < W // 2)
    got = log[inq]
    q = np.ascontiguousarray(sc.cube[: H // 2, : W // 2])
    ref = oracle.rhseg(q, **dict(p, rnb_levels=L - 1, target_regions=S, level_counts=[S]))
    want = ref.log.copy()
    for f in ("lo", "hi"):
        want[f] = (ref.log[f] // (W // 2)) * W + ref.log[f] % (W // 2)
    assert len(got) == len(want)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("form", ["incremental", "fp16"])
def test_batch256_sampled_parity(form):
    secs = synth.batch_sections(256)
    params = {k: v for k, v in synth.BATCH_PARAMS.items() if k != "rnb_levels"}
    _say(f"[gpu] batch256 form {form}")
    res = hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c, _ in secs], merge_log=True, stats=True,
                              precision="fp16", incremental=form == "incremental", **params)
    torch.cuda.synchronize()
    _say(f"[gpu] batch256 stats {res.stats}")
    for i, (c, _) in enumerate(secs):
        check_partition_levels(res.labels[i].cpu().numpy(), params["level_counts"])
    for i in (0, 1, 17, 100, 200, 255):
        c = secs[i][0]
        ref = oracle.rhseg(c, **params)
        assert np.array_equal(res.logs[i], ref.log), f"section {i} {c.shape}"
        assert np.array_equal(res.labels[i].cpu().numpy(), ref.labels), f"section {i}"
