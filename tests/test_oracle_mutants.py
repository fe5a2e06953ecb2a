"""The oracle's pins have teeth: plant one plausible mistake at a time in a
temporary copy of the oracle source (on the CPU), rebuild it, and check that
the pins reject every mutant. The committed oracle itself is never changed."""
import os
import tempfile

import numpy as np
import pytest

import oracle
from oracle.oracle import _SRC
from paper_2106_12942_amd import synth
from tests import pybrute
from tests.invariants import check_partition_levels, sse_of_partition
from tests.test_oracle_pins import GOLDEN_CASES

MUTANTS = {
    "size_factor": ("const double fac = (dni * dnj) / (double)(ni + nj);",
                    "const double fac = (dni * dnj) / (double)(ni + nj + 1);"),
    "mean_of_j": ("const double d = Si[b] / dni - Sj[b] / dnj;",
                  "const double d = Si[b] / dni - Sj[b] / dni;"),
    "last_band_dropped": ("for (int b = 0; b < B; ++b) {\n        const double d",
                          "for (int b = 0; b < B - 1; ++b) {\n        const double d"),
    "weight_not_squared": ("w2_ = (double)p.spclust_wght * (double)p.spclust_wght;",
                           "w2_ = (double)p.spclust_wght;"),
    "ties_prefer_nonadjacent": ("N.d2 < w2_ * A.d2", "N.d2 <= w2_ * A.d2"),
    "tiebreak_on_hi": ("if (a.lo != b.lo) return a.lo < b.lo;\n    return a.hi < b.hi;",
                       "if (a.hi != b.hi) return a.hi < b.hi;\n    return a.lo < b.lo;"),
    "sum_overwritten": ("for (int b = 0; b < st_.B; ++b) Slo[b] = Slo[b] + Shi[b];",
                        "for (int b = 0; b < st_.B; ++b) Slo[b] = Shi[b];"),
    "count_not_added": ("st_.n[lo] += st_.n[hi];", "st_.n[lo] += 0;"),
    "adjacency_not_inherited": ("                st_.adj[x][lo] = 0.0;\n                st_.adj[lo][x] = 0.0;",
                                "                (void)0;"),
    "seam_ignores_diagonals": ("const int nf = forward_offsets(p->seam_connectivity, dr, dc);",
                               "const int nf = forward_offsets(4, dr, dc);"),
    "split_rounds_up": ("const int h0 = r.h / 2, w0 = r.w / 2;\n    q[0]",
                        "const int h0 = (r.h + 1) / 2, w0 = (r.w + 1) / 2;\n    q[0]"),
    "snapshot_one_late": ("if (snap_->counts[l] == R) write_level(l);",
                          "if (snap_->counts[l] == R + 1) write_level(l);"),
    "spectral_threshold_strict": ("R <= p_.spclust_max;", "R < p_.spclust_max;"),
}


SAM_MUTANTS = {
    "sam_sign_dropped": ("const double d = dot >= 0.0 ? 1.0 - t : 1.0 + t;", "const double d = 1.0 - t;"),
    "sam_cosine_not_squared": ("const double t = (dot * dot) / den;", "const double t = dot / den;"),
    "sam_norm_of_i_twice": ("pairwise_sum(qi, P) * pairwise_sum(qj, P)", "pairwise_sum(qi, P) * pairwise_sum(qi, P)"),
    "sam_zero_spectrum_parallel": ("if (den == 0.0) return 1.0;", "if (den == 0.0) return 0.0;"),
    "sam_last_band_dropped": ("for (int b = 0; b < B; ++b) {\n        dt[b]", "for (int b = 0; b < B - 1; ++b) {\n        dt[b]"),
    "sam_not_clamped": ("return d > 0.0 ? d : 0.0;", "return d;"),
    "sam_not_dispatched": ("return crit == ORACLE_CRIT_SAM ?", "return crit == -1 ?"),
}


TWO_MERGE_MUTANTS = {
    "two_step3_vs_current_adjacent": ("if (key_exists(N) && A.d2 * w2_ > N.d2)",
                                      "if (key_exists(N) && adjacent_min().d2 * w2_ > N.d2)"),
    "two_step3_not_strict": ("if (key_exists(N) && A.d2 * w2_ > N.d2)", "if (key_exists(N) && A.d2 * w2_ >= N.d2)"),
    "two_no_stop_check": ("if (R <= stop_ || !spectral_at(R)) continue;", "if (!spectral_at(R)) continue;"),
    "two_spectral_on_count_before": ("if (R <= stop_ || !spectral_at(R)) continue;",
                                     "if (R <= stop_ || !spectral_at(R + 1)) continue;"),
    "two_step3_skipped": ("record(N, 1, R, log);  // strict", "(void)N;  // strict"),
}


MULTI_MERGE_MUTANTS = {
    "multi_taken_not_marked": ("                        used.insert(k.lo);\n                        used.insert(k.hi);\n",
                               "                        used.insert(k.lo);\n"),
    "multi_nonadjacent_first": ("for (const Key& k : pass == 0 ? za : zn)", "for (const Key& k : pass == 0 ? zn : za)"),
    "multi_no_stop_check": ("t < take.size() && R > stop_; ++t", "t < take.size(); ++t"),
    "multi_no_continuation_kind": ("take[t].second + (t ? 2 : 0)", "take[t].second"),
    "multi_spectral_storms_one_at_a_time": ("            if (win.d2 != 0.0) {\n                record(win, kind, R, log);",
                                            "            if (win.d2 != 0.0 || kind == 1) {\n                record(win, kind, R, log);"),
    "multi_nonadjacent_without_spectral": ("            if (spectral)\n                for (size_t a = 0;",
                                           "            if (true)\n                for (size_t a = 0;"),
}


def _run_multi_merge_pins(lib):
    """The multi-merge pins in compact form; returns the first that fails."""
    from tests import test_oracle_multi_merge as tm
    for vals, want in ((tm.STRIP_A, [(0, 1, 0, 5), (4, 5, 2, 4), (0, 2, 0, 3), (0, 4, 1, 2), (0, 3, 0, 1)]),
                       (tm.STRIP_B, [(0, 2, 1, 6), (1, 3, 3, 5), (4, 6, 3, 4), (0, 4, 1, 3), (1, 5, 3, 2),
                                     (0, 1, 0, 1)])):
        res = oracle.rhseg(tm.strip(vals), connectivity=4, spclust_wght=0.5, spclust_max=10, target_regions=1,
                           level_counts=[1], multi_merge=True, lib=lib)
        if [g[:4] for g in tm.recs(res)] != want:
            return "hand strips"
    res = oracle.rhseg(tm.strip(tm.STRIP_A), connectivity=4, spclust_wght=0.5, spclust_max=10, target_regions=5,
                       level_counts=[5], multi_merge=True, lib=lib)
    if [g[:4] for g in tm.recs(res)] != [(0, 1, 0, 5)]:
        return "hand strip stop count"
    for t in range(10):
        p = tm.GRID[t % len(tm.GRID)]
        H, W = 4 + t % 3, 5 + t % 2
        cube = tm.tie_cube(H, W, 1 + t % 2, 90 + t)
        counts = sorted({max(2, H * W // 2), max(2, H * W // 4), 2}, reverse=True)
        kw = dict(p, target_regions=2, level_counts=counts, multi_merge=True)
        res = oracle.rhseg(cube, **kw, lib=lib)
        try:
            check_partition_levels(res.labels, counts)
        except AssertionError:
            return "partition"
        _, log = pybrute.rhseg(cube, **kw)
        if tm.recs(res) != [tuple(x) for x in log]:
            return "python hseg"
    return None


def _run_two_merge_pins(lib):
    """The two-merge pins in compact form; returns the first that fails."""
    from tests import test_oracle_two_merges as t2
    for w, want in ((1.0, [(1, 2, 0, 3), (0, 3, 1, 2), (0, 1, 0, 1)]), (0.5, [(1, 2, 0, 3), (1, 3, 0, 2), (0, 1, 0, 1)])):
        res = oracle.rhseg(t2.ROW, connectivity=4, spclust_wght=w, spclust_max=10, target_regions=1,
                           level_counts=[1], two_merges=True, lib=lib)
        if [g[:4] for g in t2.recs(res)] != want:
            return "hand case"
    for kmax, target, want in ((3, 1, [(1, 2, 0, 3), (0, 3, 1, 2), (0, 1, 0, 1)]), (10, 3, [(1, 2, 0, 3)])):
        res = oracle.rhseg(t2.ROW, connectivity=4, spclust_wght=1.0, spclust_max=kmax, target_regions=target,
                           level_counts=[target], two_merges=True, lib=lib)
        if [g[:4] for g in t2.recs(res)] != want:
            return "hand case boundaries"
    for t in range(8):
        p = t2.GRID[t % len(t2.GRID)]
        H, W = 4 + t % 3, 5 + t % 2
        cube = synth.random_cube(H, W, 1 + t % 4, seed=80 + t, kind="continuous" if t % 3 else "integer")
        counts = sorted({max(2, H * W // 2), max(2, H * W // 4), 2}, reverse=True)
        kw = dict(p, target_regions=2, level_counts=counts, two_merges=True)
        res = oracle.rhseg(cube, **kw, lib=lib)
        try:
            check_partition_levels(res.labels, counts)
        except AssertionError:
            return "partition"
        _, log = pybrute.rhseg(cube, **kw)
        if t2.recs(res) != [tuple(x) for x in log]:
            return "python hseg"
    return None


def _run_sam_pins(lib):
    """The spectral angle pins in compact form; returns the first that fails."""
    from tests.test_oracle_sam import GRID
    f = oracle.oracle._load(lib).oracle_sam if lib else oracle.oracle._load().oracle_sam

    def sam(a, b):
        a = np.ascontiguousarray(a, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        return f(a.ctypes.data, b.ctypes.data, a.size)

    for a, b, want in (([3.0, 4.0], [4.0, 3.0], 49.0 / 625.0), ([3.0, 4.0], [-4.0, -3.0], 2.0 - 49.0 / 625.0),
                       ([0.0, 0.0, 0.0], [5.0, 1.0, 2.0], 1.0), ([1.0, 2.0, 2.0], [2.0, 2.0, 1.0], 17.0 / 81.0)):
        if abs(sam(a, b) - want) > 1e-15:
            return "closed form"
    rng = np.random.default_rng(9)
    for _ in range(200):
        a = rng.uniform(-5, 5, size=int(rng.integers(1, 40)))
        if not all(0.0 <= sam(a, k * a) for k in (3.0, 5.0, 7.0)):
            return "bounds"
    for t in range(8):
        p = GRID[t % len(GRID)]
        H, W = 3 + t % 3, 4 + t % 2
        cube = synth.random_cube(H, W, 1 + t % 4, seed=60 + t, kind="continuous" if t % 3 else "integer")
        counts = [max(2, H * W // 2), 2]
        res = oracle.rhseg(cube, **p, target_regions=2, level_counts=counts, criterion="sam", lib=lib)
        _, log = pybrute.rhseg(cube, **p, target_regions=2, level_counts=counts, criterion="sam",
                               exact=bool(t % 3))
        got = [(int(m["lo"]), int(m["hi"]), int(m["kind"]), int(m["r_after"])) for m in res.log]
        if got != [tuple(x[:4]) for x in log]:
            return "python rational hseg"
    return None


def _run_pins(lib):
    """A compact pass over the pins; returns the name of the first that fails."""
    for case in GOLDEN_CASES:
        res = oracle.rhseg(case["cube"], **case["params"], lib=lib)
        got = [(int(m["lo"]), int(m["hi"]), int(m["kind"]), int(m["r_after"]), float(m["d2"])) for m in res.log]
        want = [(lo, hi, k, r, float(d)) for (lo, hi, k, r, d) in case["merges"]]
        if len(got) != len(want) or any(g[:4] != w[:4] or abs(g[4] - w[4]) > 1e-12 * max(1, w[4])
                                        for g, w in zip(got, want)):
            return "golden:" + case["name"]
    rng = np.random.default_rng(11)
    grid = [dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=12, rnb_levels=2,
                 section_regions=3),
            dict(connectivity=8, seam_connectivity=8, spclust_wght=0.21, spclust_max=20, rnb_levels=1)]
    for t in range(8):
        p = grid[t % 2]
        H, W = int(rng.integers(3, 7)), int(rng.integers(3, 7))
        cube = synth.random_cube(H, W, 3, seed=40 + t, kind="integer" if t % 3 == 0 else "continuous")
        counts = [max(2, H * W // 2), 2]
        res = oracle.rhseg(cube, **p, target_regions=2, level_counts=counts, lib=lib)
        snaps, log = pybrute.rhseg(cube, **p, target_regions=2, level_counts=counts)
        got = [(int(m["lo"]), int(m["hi"]), int(m["kind"]), int(m["r_after"]), float(m["d2"])) for m in res.log]
        if got != [tuple(x) for x in log]:
            return "python brute force"
        if not all(np.array_equal(res.labels[i], np.array(snaps[i])) for i in range(2)):
            return "python brute force labels"
        try:
            check_partition_levels(res.labels, counts)
        except AssertionError:
            return "partition"
        csum = np.concatenate([[0.0], np.cumsum(res.log["d2"])])
        for i in range(2):
            k = H * W - len(np.unique(res.labels[i]))
            if abs(csum[k] - sse_of_partition(cube.astype(np.float64), res.labels[i])) > 1e-9 * (1 + csum[k]):
                return "sse identity"
    return None


def test_unmutated_oracle_passes_the_compact_pins():
    assert _run_pins(None) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(_SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.cpp"
    path.write_text(src.replace(old, new))
    lib = oracle.build(src=str(path), out=str(tmp_path / f"liboracle_{name}.so"))
    assert _run_pins(lib) is not None, f"mutant {name} survived every pin"


def test_unmutated_oracle_passes_the_sam_pins():
    assert _run_sam_pins(None) is None


@pytest.mark.parametrize("name", sorted(SAM_MUTANTS))
def test_sam_pins_reject_mutant(name, tmp_path):
    old, new = SAM_MUTANTS[name]
    src = open(_SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.cpp"
    path.write_text(src.replace(old, new))
    lib = oracle.build(src=str(path), out=str(tmp_path / f"liboracle_{name}.so"))
    assert _run_sam_pins(lib) is not None, f"mutant {name} survived every pin"


def test_unmutated_oracle_passes_the_two_merge_pins():
    assert _run_two_merge_pins(None) is None


@pytest.mark.parametrize("name", sorted(TWO_MERGE_MUTANTS))
def test_two_merge_pins_reject_mutant(name, tmp_path):
    old, new = TWO_MERGE_MUTANTS[name]
    src = open(_SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.cpp"
    path.write_text(src.replace(old, new))
    lib = oracle.build(src=str(path), out=str(tmp_path / f"liboracle_{name}.so"))
    assert _run_two_merge_pins(lib) is not None, f"mutant {name} survived every pin"


def test_unmutated_oracle_passes_the_multi_merge_pins():
    assert _run_multi_merge_pins(None) is None


@pytest.mark.parametrize("name", sorted(MULTI_MERGE_MUTANTS))
def test_multi_merge_pins_reject_mutant(name, tmp_path):
    # some of these mutants merge a region twice, which can leave the oracle's union-find with a
    # cycle (a hang) or its tables inconsistent (a crash): the pins run in a child process with a
    # time limit, and a hang or a crash counts as a rejection
    import subprocess
    import sys
    old, new = MULTI_MERGE_MUTANTS[name]
    src = open(_SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.cpp"
    path.write_text(src.replace(old, new))
    lib = oracle.build(src=str(path), out=str(tmp_path / f"liboracle_{name}.so"))
    code = ("import sys; from tests.test_oracle_mutants import _run_multi_merge_pins as f; "
            "print('PINS', f(sys.argv[1]))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    try:
        out = subprocess.run([sys.executable, "-c", code, lib], cwd=root, capture_output=True, text=True,
                             timeout=30)
    except subprocess.TimeoutExpired:
        return  # hung: rejected
    if out.returncode != 0:
        return  # crashed: rejected
    assert "PINS None" not in out.stdout, f"mutant {name} survived every pin"
