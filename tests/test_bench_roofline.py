"""The benchmark's roofline object (CPU): which kernel kind it prices and
how. The kind is the longest-running one whose work the form defines; the
event-pair overhead is taken off every launch first. Also: a request for more
than one GPU ends with a JSON line that says why."""
import os

import pytest

import bench
from paper_2106_12942_amd.hswo import KERNEL_KINDS


def stats(ms, launches, work, overhead=0.0):
    def vec(d, z):
        v = [z] * len(KERNEL_KINDS)
        for k, x in d.items():
            v[KERNEL_KINDS.index(k)] = x
        return v
    return {"ms_kernel": vec(ms, 0.0), "kernel_launches": vec(launches, 0), "kernel_work": vec(work, 0),
            "ms_event_pair_overhead": overhead, "adjacent_pairs": 10 ** 9, "spectral_pairs": 10 ** 9}


def test_incremental_form_prices_the_decision_kernel_in_bytes():
    st = stats({"section_driver": 44.0, "wide_decide": 80.0, "wide_rows": 54.0},
               {"section_driver": 1, "wide_decide": 3320, "wide_rows": 3320},
               {"section_driver": 10 ** 9, "wide_decide": 2_600_000_000, "wide_rows": 10 ** 11}, overhead=0.003)
    r = bench.kernel_roofline(st, 128, "none")
    assert r["kernel"].startswith("k_wide_decide") and r["bound"] == "hbm" and r["unit"] == "GB/s"
    avg_s = (80.0 - 3320 * 0.003) / 3320 / 1e3
    assert r["achieved"] == pytest.approx(2_600_000_000 / 3320 / avg_s / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)


def test_screened_form_skips_its_unpriced_decision_kernels():
    # the screened form's decision kernels do no sweep: the adjacent screen is priced instead
    st = stats({"wide_adj": 136.0, "wide_decide": 160.0, "wide_mfma": 72.0, "wide_fp32": 79.0, "wide_finish": 73.0},
               {"wide_adj": 6392, "wide_decide": 6392, "wide_mfma": 3320, "wide_fp32": 3320, "wide_finish": 3320},
               {"wide_adj": 3 * 10 ** 11, "wide_mfma": 2 * 10 ** 12})
    r = bench.kernel_roofline(st, 128, "none")
    assert r["kernel"].startswith("k_wide_adj") and r["bound"] == "hbm"
    assert r["longest_kind_by_time"] == "wide_decide"
    m = bench.kernel_roofline(st, 128, "none", kind="wide_mfma")
    assert m["bound"] == "mfma" and m["peak"] == 2500.0


def test_persistent_driver_with_device_bytes_is_hbm_bound_else_fp32_model():
    inc = stats({"section_driver": 570.0}, {"section_driver": 1}, {"section_driver": 5 * 10 ** 11})
    assert bench.kernel_roofline(inc, 144, "none")["bound"] == "hbm"
    plain = stats({"section_driver": 13000.0}, {"section_driver": 7}, {})
    r = bench.kernel_roofline(plain, 128, "none")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(3.0 * 128 * 2 * 10 ** 9 / 7 / (13000.0 / 7 / 1e3) / 1e12, rel=1e-3)


def test_variant_tags_name_the_criterion_and_reading():
    class A:
        criterion, two_merges = "bsmse", False
    assert bench.variant_tag(A) == ""
    A.criterion, A.two_merges = "sam", True
    assert bench.variant_tag(A) == "_sam_two"
    assert bench.variant_kwargs(A) == {"criterion": "sam", "two_merges": True}


def test_more_than_one_gpu_is_refused_with_a_message():
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU only" in line["error"]
