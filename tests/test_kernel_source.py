"""Static checks of the HIP source (CPU).

Block-level functions contain __syncthreads(); every thread of the block must
call them the same number of times. A call reached by only some threads (a
branch on the thread, lane or wave index, or a counter macro that evaluates
its argument in thread 0 only) leaves the block's barriers mismatched and can
hang the GPU, so these checks keep that pattern out of the kernels.
"""
import os
import re

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2106_12942_amd", "csrc")
# the device headers in include order, then the kernel translation units
DEVICE_FILES = ["dev_common.h", "dev_exact.h", "dev_screen.h", "dev_row_cache.h", "dev_interval_matrix.h",
                "dev_merge.h", "dev_stages.h", "dev_multi_merge.h", "hswo_driver.hip", "hswo_wide.hip",
                "hswo_levels.hip", "hswo_noalloc.hip"]


def _source():
    return "\n".join(open(os.path.join(CSRC, f)).read() for f in DEVICE_FILES)


def _functions(src):
    out = {}
    for m in re.finditer(r"\n(?:template <[^>]*>\n)?(?:\[\[maybe_unused\]\] )?__device__[^\n]*?\b(\w+)\(", src):
        i = src.index("{", m.end())
        depth, j = 0, i
        while True:
            if src[j] == "{":
                depth += 1
            elif src[j] == "}":
                depth -= 1
                if depth == 0:
                    break
            j += 1
        out[m.group(1)] = src[i:j]
    return out


def _calls(body, name):
    return re.search(r"\b%s\s*(<[^>]*>)?\s*\(" % re.escape(name), body) is not None


def barrier_functions(src):
    funcs = _functions(src)
    bar = {n for n, b in funcs.items() if "__syncthreads" in b}
    changed = True
    while changed:
        changed = False
        for n, b in funcs.items():
            if n not in bar and any(_calls(b, x) for x in bar):
                bar.add(n)
                changed = True
    return bar | {"__syncthreads"}


def test_block_functions_are_found():
    bar = barrier_functions(_source())
    for f in ("mfma_screen", "merge_pair", "adj_collect", "fp32_tiles", "spectral_collect", "zero_step_list",
              "block_min_key"):
        assert f in bar


def test_no_barrier_function_behind_a_thread_dependent_branch():
    src = _source()
    bar = barrier_functions(src)
    cond = re.compile(r"if\s*\(([^{};]*\b(tid|threadIdx\.x|lane|lane_id\(\)|gl|wave_id\(\)|wi|wj)\b[^{};]*)\)\s*(\{?)")
    bad = []
    for m in cond.finditer(src):
        if m.group(3) == "{":
            i = m.end() - 1
            depth, j = 0, i
            while True:
                if src[j] == "{":
                    depth += 1
                elif src[j] == "}":
                    depth -= 1
                    if depth == 0:
                        break
                j += 1
            body = src[i:j]
        else:
            body = src[m.end(): src.index(";", m.end()) + 1]
        for x in bar:
            if _calls(body, x):
                bad.append((src[: m.start()].count("\n") + 1, x))
    assert not bad, f"barrier functions reached by part of the block: {bad}"


def test_counter_macro_arguments_are_plain_values():
    src = _source()
    bar = barrier_functions(src)
    for m in re.finditer(r"CNT_ADD\(([^;]*)\);", src):
        arg = m.group(1)
        for x in bar:
            assert not _calls(arg, x), f"CNT_ADD evaluates {x}(...) in thread 0 only: {m.group(0)}"


def test_every_device_file_is_checked():
    have = {f for f in os.listdir(CSRC) if f.endswith(".hip") or f.startswith("dev_")}
    assert have == set(DEVICE_FILES)


def test_every_translation_unit_is_built():
    from paper_2106_12942_amd import build
    have = {f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp"))}
    assert have == {os.path.basename(f) for f in build.SOURCES}
