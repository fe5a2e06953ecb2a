"""GPU parity at the benchmark workloads' full sizes.

* rhseg1024_salt (1024 x 1024 x 220, 5% identical salt pixels, L = 5): the
  whole merge log and every label map against the oracle, for the
  incremental form (default settings, and with the leaf level in the
  persistent driver) and the BF16 matrix-core screened form.
* rhseg2048_f16 (2048 x 2048 x 224 float16, L = 5): the whole merge log
  (4,194,288 merges) and all 8 label maps against one oracle run on the whole
  image, for the same three forms.
* batch256 (256 uneven independent sections): every section's merge log and
  label map against the oracle, for the incremental and FP16 screened forms.
"""
import os
import sys
import time

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
        _C3_REF["ref"] = (sc, p, oracle.rhseg(sc.cube, **p, n_threads=host_threads(), progress="rhseg1024_salt"))
    return _C3_REF["ref"]


@pytest.mark.parametrize("form", ["incremental", "incremental_leaves_persistent", "bf16"])
def test_rhseg1024_salt_full_parity(form):
    sc, p, ref = _c3_reference()
    L = p["rnb_levels"]
    kw = {k: v for k, v in p.items() if k != "rnb_levels"}
    _say(f"[gpu] rhseg1024_salt full size, form {form}")
    inc = form.startswith("incremental")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=L, merge_log=True, stats=True,
                             precision="fp16" if inc else form, incremental=inc,
                             tuning=dict(wide_max_sections=64) if form == "incremental_leaves_persistent" else None,
                             **kw)
    torch.cuda.synchronize()
    _say(f"[gpu] rhseg1024_salt stats {res.stats}")
    assert np.array_equal(res.log[: len(ref.log)], ref.log)
    assert np.array_equal(res.labels.cpu().numpy(), ref.labels)


def host_threads():
    """Oracle threads: the CPUs this process may run on, at most 16 (the host
    share of one GPU on the test boxes)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


_C5 = {}


def _c5_reference():
    """The whole 2048 x 2048 x 224 float16 workload through the oracle, once
    per session (a few minutes on the host; progress is printed per level)."""
    if "ref" not in _C5:
        t0 = time.perf_counter()
        sc, p = synth.workload("rhseg2048_f16")
        _say(f"[gpu] rhseg2048_f16 cube generated in {time.perf_counter() - t0:.0f} s; oracle on {host_threads()} "
             "host threads")
        t0 = time.perf_counter()
        ref = oracle.rhseg(sc.cube, **p, n_threads=host_threads(), progress="rhseg2048_f16")
        _say(f"[gpu] rhseg2048_f16 oracle done in {time.perf_counter() - t0:.0f} s ({len(ref.log)} merges)")
        _C5["ref"] = (sc, p, ref)
    return _C5["ref"]


@pytest.mark.parametrize("form", ["incremental", "incremental_leaves_persistent", "bf16"])
def test_rhseg2048_f16_full_parity(form):
    """Every merge (all five recursion levels, all 256 + 64 + 16 + 4 + 1
    sections, in order, with the FP64 criterion value) and every one of the 8
    label maps equal the oracle's: the incremental form with its default
    settings (every level of at most 256 sections wide), the incremental form
    with the leaf level in the persistent driver (interval-matrix rescans on
    one workgroup per section; the autotuner's usual choice), and the BF16
    matrix-core screened form."""
    sc, p, ref = _c5_reference()
    L = p["rnb_levels"]
    kw = {k: v for k, v in p.items() if k != "rnb_levels"}
    H, W, _ = sc.cube.shape
    _say(f"[gpu] rhseg2048_f16 full size, form {form}")
    inc = form.startswith("incremental")
    res = hswo.rhseg_segment(torch.from_numpy(sc.cube).cuda(), rnb_levels=L, merge_log=True, stats=True,
                             precision="fp16" if inc else form, incremental=inc,
                             tuning=dict(wide_max_sections=64) if form == "incremental_leaves_persistent" else None,
                             **kw)
    torch.cuda.synchronize()
    _say(f"[gpu] rhseg2048_f16 {form}: {res.stats['merges']} merges, {res.stats['ms_total']:.0f} ms")
    assert res.stats["merges"] == H * W - p["target_regions"] == len(ref.log)
    got = res.log[: len(ref.log)]
    if not np.array_equal(got, ref.log):
        bad = int(np.nonzero(got != ref.log)[0][0])
        pytest.fail(f"merge log diverges at record {bad}: gpu {got[bad]} oracle {ref.log[bad]}")
    lab = res.labels.cpu().numpy()
    for li in range(lab.shape[0]):
        assert np.array_equal(lab[li], ref.labels[li]), f"level {li} ({p['level_counts'][li]} regions) differs"
    check_partition_levels(lab, p["level_counts"])


_BATCH = {}


def _batch_reference():
    """All 256 sections of the batch workload through the oracle (one oracle
    run per section, sections spread over the host threads)."""
    if "ref" not in _BATCH:
        import concurrent.futures as cf
        secs = synth.batch_sections(256)
        params = {k: v for k, v in synth.BATCH_PARAMS.items() if k != "rnb_levels"}
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(host_threads()) as ex:
            refs = list(ex.map(lambda c: oracle.rhseg(c[0], **params, n_threads=1), secs))
        _say(f"[gpu] batch256 oracle: 256 sections in {time.perf_counter() - t0:.0f} s")
        _BATCH["ref"] = (secs, params, refs)
    return _BATCH["ref"]


@pytest.mark.parametrize("form", ["incremental", "fp16"])
def test_batch256_full_parity(form):
    """Every one of the 256 uneven sections: merge log and label map equal the
    oracle's, in one batched call."""
    secs, params, refs = _batch_reference()
    _say(f"[gpu] batch256 form {form}")
    res = hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c, _ in secs], merge_log=True, stats=True,
                              precision="fp16", incremental=form == "incremental", **params)
    torch.cuda.synchronize()
    _say(f"[gpu] batch256 {form}: {res.stats['merges']} merges, {res.stats['ms_total']:.0f} ms")
    for i, (c, _) in enumerate(secs):
        ref = refs[i]
        assert np.array_equal(res.logs[i], ref.log), f"section {i} {c.shape}: merge log differs"
        assert np.array_equal(res.labels[i].cpu().numpy(), ref.labels), f"section {i}: labels differ"
