#!/usr/bin/env python3
"""Benchmark of the RHSEG hot path on one MI355X.

One step = one call through the C ABI on device-resident synthetic input,
covering every merge of every section: the HSEG loops of the leaf sections,
the reassembly of each recursion level, the parents' loops, and the label
maps of the requested hierarchy levels (all of it in the HIP kernels).

Workloads
  rhseg2048_f16 (default, the largest): 2048 x 2048 x 224 float16 endmember
      mixture (500 classes, sigma 25, seed 505), rnb_levels 5 (128 x 128
      leaves), w 0.5, spectral stage at <= 2048 regions, sections stop at 512,
      target 16, 8 output levels.
  rhseg1024_salt: 1024 x 1024 x 220 float32 endmember mixture with 5% identical
      salt pixels, rnb_levels 5.
  rhseg512: 512 x 512 x 128 float32 Voronoi scene (200 classes, sigma 30,
      seed 202), rnb_levels 4 (64 x 64 leaves), w 0.5, spectral stage at
      <= 1024 regions, sections stop at 256, 8 output levels.
  hswo64: 64 x 64 x 32 float32 Voronoi (40 classes, sigma 20, seed 101), one
      section, spectral at <= 256, down to 2 regions, 11 levels.
  batch256: 256 independent sections, side U{32..128}, bands U{64,96,..,224},
      10..120 Voronoi classes, sigma 30 (seed 404000+s), each merged down to
      256 regions (w 0.5, spectral at <= 1024) -- one hswo_run_batch call.

Forms (--form): "incremental" (default): cached exact per-edge D2 and the
spectral row cache; "screened": every pair screened each iteration, the
spectral stage on matrix cores (--precision fp16, the default, or bf16);
"plain": every pair screened each iteration in FP32, the sections of a level
one after another (neither the precision nor the batching form);
"plain_batched": the same FP32 screens with the sections of a level batched.
Levels run batched into one launch (persistent) or one launch sequence per
iteration (wide), replayed from a hipGraph; the first warm-up call autotunes
the execution settings (--no-autotune: library defaults). The other forms run
once on the same input for the comparison and must give the same labels (the
plain forms are skipped on the two largest workloads, where they take many
minutes).

Criterion (--criterion): "bsmse" (default), the paper's Equation 1; "sam",
the spectral angle. --two-merges: the two-merge reading of the HSEG steps.
Both exist in the incremental form only, so no other form is compared.

Output: one JSON line. `value` is dissimilarity pairs evaluated per second of
wall time, counted by the kernels: the incremental form's exact FP64
evaluations (cache re-scoring and row-cache rows); for the screened and plain
forms every live adjacent pair and every unique spectral pair screened in
each iteration. `method_pairs_per_s` counts the method's pairs instead (live
adjacent pairs, plus R(R-1)/2 per iteration of the spectral stage), whether
evaluated or read from a cache. The roofline object is for the kernel with
the largest device time in one extra eager step of the timed form with every
launch bracketed by hipEvents (HSWO_FLAG_KERNEL_TIMES). `cpu_baseline` is the
FP64 oracle on the host's threads: the whole workload where that takes
seconds, else a bounded sample of leaf sections; the whole workload always
goes through the oracle once for the per-level label check.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks (published figures / unit counts)
PEAK_HBM_GBS = 8000.0
# FP32 vector arithmetic without packed-FP32 instructions (kept out of the
# generated code): 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_FP32_VALU_TFLOPS = 78.6
PEAK_MFMA_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0}
PEAK_FP64_VALU_TFLOPS = 78.6

WORKLOAD_DESC = {
    "rhseg512": "512x512x128 f32 Voronoi (200 classes, sigma 30, seed 202); rnb_levels 4 (64x64 leaves); "
                "w 0.5; spectral at <=1024 regions; sections stop at 256; target 8; 8 levels",
    "hswo64": "64x64x32 f32 Voronoi (40 classes, sigma 20, seed 101); one section; w 0.5; spectral at "
              "<=256 regions; target 2; 11 levels",
    "batch256": "256 independent f32 sections, side U{32..128}, bands U{64..224 step 32}, 10-120 Voronoi "
                "classes, sigma 30, seeds 404000+s; each merged to 256 regions; w 0.5; spectral at <=1024",
    "rhseg1024_salt": "1024x1024x220 f32 endmember mixture (300 classes, sigma 25, seed 303, 5% identical salt "
                      "pixels); rnb_levels 5; w 0.5; spectral at <=1024; sections stop at 256; target 8",
    "rhseg2048_f16": "2048x2048x224 f16 endmember mixture (500 classes, sigma 25, seed 505); rnb_levels 5; w 0.5; "
                     "spectral at <=2048; sections stop at 512; target 16",
}

# workloads whose oracle and plain-path runs take minutes: timed on the GPU only (their parity with the
# oracle is checked by the GPU tests)
LARGE = ("rhseg1024_salt", "rhseg2048_f16")


def traffic_from_profiles(tag: str):
    """HBM bytes per launch of the dominant kernel, if a counter summary for
    exactly this kernel build and workload is committed under profiles/."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("hbm_bytes_per_launch:"):
            return float(line.split(":", 1)[1])
    return None


KIND_DESC = {
    "section_driver": "k_section_driver (one workgroup runs a section's whole pass)",
    "wide_adj": "k_wide_adj (adjacent screen, edges over G workgroups)",
    "wide_decide": "k_wide_decide (decision, merge and edge/row-cache upkeep, one workgroup per section)",
    "wide_mfma": "k_wide_mfma (matrix-core tile screen)",
    "wide_fp32": "k_wide_fp32 (FP32 tile screen)",
    "wide_finish": "k_wide_finish (spectral decision and merge)",
    "wide_rows": "k_wide_rows / k_mat_rows (row cache: rows evaluated in FP64, or rescanned from the interval matrix)",
    "rowcache_prep": "k_rowcache_prep",
    "matrix_fill": "k_mat_fill (interval matrix of starting row caches: FP32 mean differences, 64 x 64 tiles)",
}


def kernel_roofline(st, B, tag, kind=None):
    """Roofline of the kernel kind with the largest device time among those
    whose work is defined for the form (from a
    HSWO_FLAG_KERNEL_TIMES step: every launch between a pair of hipEvents on
    its stream, less what an event pair adds to a launch, which the library
    measures in the same call on an empty kernel). Algorithmic work per launch = the kind's work over the step
    divided by its launches:
      wide_decide: bytes counted on the device by the kernel (16 per edge slot
        the merge reads -- every slot on a pass over the list; on the edge
        index's path the scanned ranges, the re-minimised chunks and one per
        chunk record -- 24 per band per merge; in the spectral stage 12 per
        live row and 32 per pending row per 64 live rows) -> HBM bound;
      wide_rows: bytes counted on the device: exact row tasks read each
        column's FP64 mean row once per 4 rows (3 flops per band and pair, far
        below the ridge), rescans read a row of the interval matrix and the
        FP64 rows of the pairs it cannot rule out -> HBM bound;
      section_driver, incremental form: the wide_decide bytes of the
        iterations it runs + 8 B per band per live region for each iteration
        whose row-cache stage evaluates rows, counted on the device -> HBM bound;
      wide_mfma: 2 flops per band per unique pair of each screened section,
        counted on the device -> matrix cores;
      wide_adj: FP32 mean rows read once + 8 B per edge slot + 8 B per
        region, counted on the device -> HBM bound;
      otherwise (the screened and plain forms' section driver) 3 FP32 flops
        per band per screened pair -> FP32 vector bound."""
    from paper_2106_12942_amd.hswo import KERNEL_KINDS
    ms = st["ms_kernel"]
    n = st["kernel_launches"]
    kw = st["kernel_work"]
    ov = st["ms_event_pair_overhead"]
    # each launch's time without what its event pair adds (measured in the same call)
    ms = [max(0.0, ms[i] - n[i] * ov) for i in range(len(ms))]
    by_time = KERNEL_KINDS[max(range(len(ms)), key=lambda i: ms[i])]
    if kind is None:
        # the longest-running kind whose work this run defines: device-counted work, or the
        # screened and plain forms' own sweeps (FP32 flops per screened pair); the screened
        # form's decision kernels do neither sweep, so they are not priced
        cand = [i for i in range(len(ms))
                if n[i] and (kw[i] > 0 or KERNEL_KINDS[i] in ("section_driver", "wide_fp32"))]
        k = max(cand or range(len(ms)), key=lambda i: ms[i])
    else:
        k = KERNEL_KINDS.index(kind)
    kind = KERNEL_KINDS[k]
    avg_ms = ms[k] / max(n[k], 1)
    if kind in ("wide_decide", "section_driver") and kw[k]:
        work = float(kw[k])
        bound, peak, unit, scale = "hbm", PEAK_HBM_GBS, "GB/s", 1e9
    elif kind == "wide_rows":
        work = float(kw[k])
        bound, peak, unit, scale = "hbm", PEAK_HBM_GBS, "GB/s", 1e9
    elif kind == "matrix_fill":
        work = float(kw[k])
        bound, peak, unit, scale = "alu", PEAK_FP32_VALU_TFLOPS, "TFLOP/s", 1e12
    elif kind == "wide_mfma":
        work = float(kw[k])
        bound, peak, unit, scale = "mfma", PEAK_MFMA_TFLOPS["fp16"], "TFLOP/s", 1e12
    elif kind == "wide_adj":
        work = float(kw[k])
        bound, peak, unit, scale = "hbm", PEAK_HBM_GBS, "GB/s", 1e9
    else:
        work = 3.0 * B * (st["adjacent_pairs"] + st["spectral_pairs"])
        bound, peak, unit, scale = "alu", PEAK_FP32_VALU_TFLOPS, "TFLOP/s", 1e12
    per_launch = work / max(n[k], 1)
    achieved = per_launch / (avg_ms / 1e3) / scale
    return {"bound": bound, "achieved": round(achieved, 4), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 5), "traffic": traffic_from_profiles(f"{kind}_{tag}"),
            "kernel": KIND_DESC[kind], "longest_kind_by_time": by_time,
            "launches_per_step": n[k], "avg_launch_us": round(avg_ms * 1e3, 3),
            "event_pair_overhead_us": round(ov * 1e3, 3),
            "avg_launch_us_with_event_pair": round(st["ms_kernel"][k] / max(n[k], 1) * 1e3, 3),
            "algorithmic_work_per_launch": per_launch,
            "kernel_ms_per_step": {KERNEL_KINDS[i]: round(ms[i], 3) for i in range(len(ms)) if n[i]},
            "kernel_launches_per_step": {KERNEL_KINDS[i]: n[i] for i in range(len(ms)) if n[i]},
            "kernel_work_per_step": {KERNEL_KINDS[i]: kw[i] for i in range(len(ms)) if kw[i]}}


def form_kwargs(form, precision):
    if form == "plain":
        # neither form: FP32 screens, and the sections of a level one after another
        return dict(precision="fp32", incremental=False, sequential=True)
    if form == "plain_batched":
        return dict(precision="fp32", incremental=False)
    if form == "screened":
        return dict(precision=precision, incremental=False)
    return dict(precision=precision, incremental=True)


def variant_kwargs(args):
    return dict(criterion=args.criterion, two_merges=args.two_merges)


def variant_tag(args):
    """"" for the paper's method; else a suffix naming the criterion / reading."""
    return ("" if args.criterion == "bsmse" else f"_{args.criterion}") + ("_two" if args.two_merges else "")


def timed_steps(step, stream, torch, steps, warmup, first=None):
    """Time `steps` calls after `warmup` untimed ones; the first warm-up call's
    wall time (graph capture and instantiation included) goes to first[0]."""
    with torch.cuda.stream(stream):
        for w in range(warmup):
            t0 = time.perf_counter()
            step()
            if w == 0 and first is not None:
                stream.synchronize()
                first.append((time.perf_counter() - t0) * 1e3)
        stream.synchronize()
        torch.cuda.synchronize()
        walls, res = [], None
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            res = step()  # stats=True: the call synchronises its stream before returning
            walls.append((time.perf_counter() - ts) * 1e3)
        stream.synchronize()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    return elapsed * 1e3 / steps, walls, res


def evaluated_pairs(st, form):
    """Pairs the kernels evaluated in a call, counted on the device: the
    incremental form evaluates only what its caches miss: edge re-scoring
    and row-cache rows (rescanned from the interval matrix, and in FP64
    where a bound cannot rule a pair out); the screened and plain
    forms screen every live adjacent pair and every unique pair of the
    spectral stage in each iteration (their exact re-checks are second looks
    at pairs already screened)."""
    if form == "incremental":
        return st["exact_rechecks"] + st["row_bounded_pairs"]
    return st["adjacent_pairs"] + st["spectral_pairs"]


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def leaf_grid(H, W, L):
    """Leaf rectangles of the RHSEG quadtree (split at floor(h/2), floor(w/2);
    TL, TR, BL, BR), in quadtree order."""
    def rec(r0, c0, h, w, d):
        if d == 1:
            return [(r0, c0, h, w)]
        h0, w0 = h // 2, w // 2
        out = []
        for (rr, cc, hh, ww) in ((r0, c0, h0, w0), (r0, c0 + w0, h0, w - w0), (r0 + h0, c0, h - h0, w0),
                                 (r0 + h0, c0 + w0, h - h0, w - w0)):
            out += rec(rr, cc, hh, ww, d - 1)
        return out
    return rec(0, 0, H, W, L)


def screen_error_report(np, torch, hswo, cube_h, params, precision, leaf):
    """HSWO_FLAG_DEBUG_VERIFY_BOUND on the top-left crop of four by four
    leaves (rnb_levels 3, the workload's leaf shape and parameters): every
    pair a screen passed to the FP64 re-check with its screen estimate, its
    certified bounds and its canonical D2. Error is relative, in Equation 1's
    square-root domain, over pairs with D2 > 0."""
    side_h, side_w = 4 * leaf[0], 4 * leaf[1]
    crop = np.ascontiguousarray(cube_h[:side_h, :side_w])
    kw = {k: v for k, v in params.items() if k != "rnb_levels"}
    kw["level_counts"] = [c for c in kw["level_counts"] if c < side_h * side_w] or [kw["target_regions"]]
    cap = 1 << 23
    res = hswo.rhseg_segment(torch.from_numpy(crop).cuda(), rnb_levels=3, stats=True, precision=precision,
                             incremental=False, verify_cap=cap, **kw)
    rec = res.verify
    out = {"crop": f"{side_h}x{side_w} top-left, rnb_levels 3", "precision": precision,
           "records": int(res.stats["verify_records"]), "records_kept": int(len(rec))}
    ok = (rec["lower"] <= rec["d2"]) & (rec["d2"] <= rec["upper"])
    out["pairs_within_certified_bounds"] = float(ok.mean()) if len(rec) else None
    for st, name in hswo.SCREEN_STAGES.items():
        r = rec[(rec["stage"] == st) & (rec["d2"] > 0)]
        if r.size == 0:
            continue
        rel = np.abs(np.sqrt(np.maximum(r["screen"], 0.0)) - np.sqrt(r["d2"])) / np.sqrt(r["d2"])
        out[name] = {"pairs": int(r.size), "p50": float(np.percentile(rel, 50)),
                     "p99": float(np.percentile(rel, 99)), "max": float(rel.max())}
    return out


def cpu_leaf_sample(np, oracle, hswo, torch, cube_h, params, L, seconds=15.0):
    """The oracle on whole leaf sections of the workload (in quadtree order,
    `threads` at a time, one host thread each) until about `seconds` have
    passed; the same leaves through the GPU's incremental form give the pairs
    it evaluates for them, so the rate is in the timed value's unit."""
    import concurrent.futures as cf
    H, W, _ = cube_h.shape
    leaves = leaf_grid(H, W, L)
    S = params["section_regions"] or max(params["target_regions"], params["spclust_max"] // 4)
    lp = {k: v for k, v in params.items() if k not in ("rnb_levels", "level_counts", "section_regions",
                                                      "target_regions")}
    lp.update(target_regions=S, section_regions=0, level_counts=[S])
    threads = host_threads()
    cubes, done = [], 0
    t0 = time.perf_counter()
    while done < len(leaves) and time.perf_counter() - t0 < seconds:
        batch = leaves[done:done + threads]
        cs = [np.ascontiguousarray(cube_h[r:r + h, c:c + w]) for (r, c, h, w) in batch]
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda c: oracle.rhseg(c, **lp, n_threads=1), cs))
        cubes += cs
        done += len(batch)
    cpu_s = time.perf_counter() - t0
    rs = hswo.hswo_run_batch([torch.from_numpy(c).cuda() for c in cubes], stats=True, precision="bf16",
                             incremental=True, **lp)
    pairs = evaluated_pairs(rs.stats, "incremental")
    return {"value": pairs / cpu_s, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"leaf sections 0..{done - 1} of {len(leaves)} ({leaves[0][2]}x{leaves[0][3]} px, each merged "
                      f"to {S} regions as in the workload's deepest level), FP64 oracle in cached mode, one leaf per "
                      f"host thread on {threads} threads, {cpu_s:.2f} s; rate = the pairs the GPU's incremental "
                      f"form evaluates for those leaves ({pairs}) over that time",
            "seconds": cpu_s, "leaves": done}


def host_threads():
    """CPUs this process may run on (the oracle's thread count)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def bench_rhseg(args, np, torch, hswo, synth):
    t0 = time.perf_counter()
    sc, params = synth.workload(args.workload)
    say(f"{args.workload} cube generated in {time.perf_counter() - t0:.1f} s")
    params.update(variant_kwargs(args))
    cube_h = sc.cube
    H, W, B = cube_h.shape
    dev = torch.device("cuda:0")
    cube = torch.from_numpy(cube_h).to(dev)
    L = params["rnb_levels"]
    kw = {k: v for k, v in params.items() if k != "rnb_levels"}
    stream = torch.cuda.Stream(dev)
    ws = hswo.Workspace()
    nl = len(params["level_counts"])
    labels = torch.empty((nl, H, W), dtype=torch.int32, device=dev)

    def runner(form, out, graph, kernel_times=False, autotune=False):
        fk = form_kwargs(form, args.precision)

        def step():
            return hswo.rhseg_segment(cube, rnb_levels=L, stats=True, stream=stream, workspace=ws, labels_out=out,
                                      graph=graph, autotune=autotune, kernel_times=kernel_times, **fk, **kw)
        return step

    first = []
    say(f"timed form {args.form}: {args.warmup} warm-up + {args.steps} timed steps")
    ms_per_step, walls, res = timed_steps(runner(args.form, labels, args.graph, autotune=args.autotune), stream,
                                          torch, args.steps, args.warmup, first)
    st = res.stats
    method_pairs = st["adjacent_pairs"] + st["spectral_pairs"]
    ev = evaluated_pairs(st, args.form)
    fk = form_kwargs(args.form, args.precision)
    out = {
        "value": ev / (ms_per_step / 1e3), "unit": "pairs/s", "ms_per_step": ms_per_step,
        "wall_ms_median": statistics.median(walls), "wall_ms_min": min(walls), "wall_ms_max": max(walls),
        "config": {"workload": args.workload, "desc": WORKLOAD_DESC[args.workload], "H": H, "W": W, "B": B,
                   "cube_dtype": str(cube_h.dtype), "form": args.form,
                   "precision": fk["precision"] if args.form != "incremental" else "none: every pair evaluated "
                   "exactly in FP64", "criterion": args.criterion, "two_merges": args.two_merges,
                   "graph": args.graph, "autotune": args.autotune, "tuning": st["tuning"]},
        "evaluated_pairs_per_step": ev,
        "method_pairs_per_step": method_pairs, "method_pairs_per_s": method_pairs / (ms_per_step / 1e3),
        "merges_per_step": st["merges"], "exact_evaluations_per_step": st["exact_rechecks"],
        "fp32_tiles_per_step": st["fp32_tiles"], "mfma_super_tiles_per_step": st["mfma_tiles"],
        "first_call_ms": first[0] if first else None,
    }
    tag = f"{args.workload}_{args.form}" + variant_tag(args)
    # the same step with the cube first copied from pinned host memory on the call's stream (the
    # paper's times include that transfer); value stays the device-resident rate
    pinned = torch.from_numpy(cube_h).pin_memory()
    step = runner(args.form, labels, args.graph)
    nh = min(3, args.steps)

    def step_h2d():
        cube.copy_(pinned, non_blocking=True)
        return step()
    ms_h2d, _, _ = timed_steps(step_h2d, stream, torch, nh, 1)
    with torch.cuda.stream(stream):
        t1 = time.perf_counter()
        for _ in range(nh):
            cube.copy_(pinned, non_blocking=True)
        stream.synchronize()
        h2d_ms = (time.perf_counter() - t1) * 1e3 / nh
    out["with_h2d"] = {"ms_per_step": ms_h2d, "value": ev / (ms_h2d / 1e3), "h2d_ms": h2d_ms,
                       "h2d_bytes": int(cube_h.nbytes), "steps": nh}
    # per-kernel device times: one more step of the timed form, eager, every launch bracketed by hipEvents
    same_kt = None
    if not args.no_kernel_times:
        say("kernel-times step")
        kt = torch.empty_like(labels)
        _, _, rk = timed_steps(runner(args.form, kt, False, kernel_times=True), stream, torch, 1, 0)
        out["kernel_times_step_ms"] = rk.stats["ms_total"]
        out["roofline"] = kernel_roofline(rk.stats, B, tag)
        same_kt = bool(torch.equal(kt, labels))
    lab = labels.cpu().numpy()
    comparisons = {}
    for form in ("plain", "plain_batched", "screened", "incremental"):
        if form == args.form or (form.startswith("plain") and (args.no_plain or args.workload in LARGE)) or \
                args.no_forms:
            continue
        if variant_tag(args) and form != "incremental":
            continue  # the other criterion and the two-merge reading exist in the incremental form only
        say(f"form {form}")
        o = torch.empty_like(labels)
        # the unbatched plain path is a long launch sequence: eager, one warm-up and one timed call
        ms, _, r = timed_steps(runner(form, o, args.graph and form != "plain"), stream, torch, 1, 1)
        rst = r.stats
        comparisons[form] = {"ms_per_step": ms, "speedup_of_timed_form": ms / ms_per_step,
                             "labels_identical_to_timed_form": bool(torch.equal(o, labels)),
                             "precision": form_kwargs(form, args.precision)["precision"],
                             "evaluated_pairs_per_step": evaluated_pairs(rst, form),
                             "evaluated_pairs_per_s": evaluated_pairs(rst, form) / (ms / 1e3)}
        if form != "incremental":
            comparisons[form]["screen_iterations"] = rst["screen_iterations"]
            comparisons[form]["screen_fallbacks"] = rst["screen_fallbacks"]
            comparisons[form]["fallback_rate"] = rst["screen_fallbacks"] / max(1, rst["screen_iterations"])
        if form == "screened" and not args.no_kernel_times:
            # the screened form's own sweeps: adjacent screen against HBM, matrix-core screen against MFMA peak
            say("form screened, kernel-times step")
            _, _, rs = timed_steps(runner(form, o, False, kernel_times=True), stream, torch, 1, 0)
            comparisons[form]["rooflines"] = {
                kd: kernel_roofline(rs.stats, B, f"{args.workload}_{form}", kind=kd)
                for kd in ("wide_adj", "wide_mfma", "section_driver")
                if rs.stats["kernel_launches"][hswo.KERNEL_KINDS.index(kd)]}
    if "plain" in comparisons:
        # the plain FP32 path (no precision form, no batching) against every form
        pm = comparisons["plain"]["ms_per_step"]
        out["speedup_vs_plain"] = {args.form: pm / ms_per_step,
                                   **{f: pm / v["ms_per_step"] for f, v in comparisons.items() if f != "plain"}}
    out["forms"] = comparisons
    out["labels_identical_kernel_times_step"] = same_kt
    if not args.no_forms and not variant_tag(args):
        say("screen error report (bound-verification records)")
        leaf = leaf_grid(H, W, L)[0][2:]
        out["screen_error"] = screen_error_report(np, torch, hswo, cube_h, params,
                                                  args.precision if args.precision != "fp32" else "bf16", leaf)
    if not args.no_cpu_baseline:
        import oracle
        threads = host_threads()
        if args.workload in LARGE:
            say("cpu baseline: oracle on a bounded sample of leaf sections")
            out["cpu_baseline"] = cpu_leaf_sample(np, oracle, hswo, torch, cube_h, params, L)
            out["gpu_vs_oracle_speedup_on_sample"] = out["value"] / out["cpu_baseline"]["value"]
        say(f"oracle on the whole workload ({threads} threads) for the per-level label check")
        tc = time.perf_counter()
        ref = oracle.rhseg(cube_h, **params, n_threads=threads)
        cpu_s = time.perf_counter() - tc
        per_level = [bool(np.array_equal(lab[i], ref.labels[i])) for i in range(nl)]
        out["labels_identical_to_oracle"] = all(per_level)
        out["labels_identical_to_oracle_per_level"] = dict(zip([int(c) for c in params["level_counts"]], per_level))
        out["oracle_whole_workload_s"] = cpu_s
        out["gpu_vs_oracle_speedup"] = cpu_s * 1e3 / ms_per_step
        if args.workload not in LARGE:
            out["cpu_baseline"] = {"value": ev / cpu_s, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                                   "sample": f"the whole {args.workload} workload, FP64 oracle (cached mode, sections "
                                             f"of a level on {threads} threads), {cpu_s:.2f} s; rate = the pairs "
                                             "the timed GPU form evaluates for it over that time"}
        if args.single_thread_oracle:
            # the paper's sequential baseline: the oracle on one host thread
            tc = time.perf_counter()
            oracle.rhseg(cube_h, **params, n_threads=1)
            one_s = time.perf_counter() - tc
            out["cpu_single_thread"] = {"value": ev / one_s, "unit": "pairs/s", "seconds": one_s,
                                        "gpu_speedup": one_s * 1e3 / ms_per_step}
    return out, B


def bench_batch(args, np, torch, hswo, synth):
    secs = synth.batch_sections(256)
    params = dict(synth.BATCH_PARAMS)
    params.pop("rnb_levels", None)
    params.update(variant_kwargs(args))
    other_forms = not args.no_forms and not variant_tag(args)  # the variants: incremental form only
    dev = torch.device("cuda:0")
    dc = [torch.from_numpy(c).to(dev) for c, _ in secs]
    stream = torch.cuda.Stream(dev)
    ws = hswo.Workspace()

    def new_outs():
        return [torch.empty((len(params["level_counts"]), c.shape[0], c.shape[1]), dtype=torch.int32, device=dev)
                for c in dc]

    def runner(form, outs, graph, kernel_times=False, autotune=False):
        fk = form_kwargs(form, args.precision)

        def step():
            return hswo.hswo_run_batch(dc, stats=True, stream=stream, workspace=ws, labels_out=outs, graph=graph,
                                       autotune=autotune, kernel_times=kernel_times, **fk, **params)
        return step

    outs = new_outs()
    say(f"batch256: timed form {args.form}: {args.warmup} warm-up + {args.steps} timed steps")
    # the timed form is autotuned in its warm-up; the compared forms run with the library defaults
    ms_per_step, walls, res = timed_steps(runner(args.form, outs, args.graph, autotune=args.autotune), stream, torch,
                                          args.steps, args.warmup)
    st = res.stats
    pairs = st["adjacent_pairs"] + st["spectral_pairs"]
    ev = evaluated_pairs(st, args.form)
    Bmean = float(np.mean([c.shape[2] for c, _ in secs]))
    fk = form_kwargs(args.form, args.precision)
    out = {
        "value": ev / (ms_per_step / 1e3), "unit": "pairs/s", "ms_per_step": ms_per_step,
        "wall_ms_median": statistics.median(walls), "wall_ms_min": min(walls), "wall_ms_max": max(walls),
        "config": {"workload": "batch256", "desc": WORKLOAD_DESC["batch256"], "sections": len(secs),
                   "form": args.form, "precision": fk["precision"], "criterion": args.criterion,
                   "two_merges": args.two_merges, "graph": args.graph, "autotune": args.autotune,
                   "driver_variant": st["driver_variant"]},
        "evaluated_pairs_per_step": ev, "method_pairs_per_step": pairs,
        "method_pairs_per_s": pairs / (ms_per_step / 1e3), "merges_per_step": st["merges"],
        "exact_evaluations_per_step": st["exact_rechecks"],
    }
    if not args.no_kernel_times:
        say("batch256: kernel-times step")
        ko = new_outs()
        _, _, rk = timed_steps(runner(args.form, ko, False, kernel_times=True), stream, torch, 1, 0)
        out["kernel_times_step_ms"] = rk.stats["ms_total"]
        # the band count varies by section: the roofline uses the mean
        out["roofline"] = kernel_roofline(rk.stats, Bmean, f"batch256_{args.form}" + variant_tag(args))
    comparisons = {}
    if not args.no_plain and other_forms:
        # the plain path: 256 sequential hswo_run calls, FP32 screen, every pair each iteration
        say("batch256: plain path, 256 sequential hswo_run calls")
        torch.cuda.synchronize()
        ts = time.perf_counter()
        same = True
        for i, c in enumerate(dc):
            r = hswo.hswo_run(c, precision="fp32", **params)
            same = same and bool(torch.equal(r.labels, outs[i]))
            if (i + 1) % 32 == 0:
                say(f"batch256: plain path, {i + 1} of 256 sections")
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - ts) * 1e3
        comparisons["plain_sequential"] = {"form": "256 sequential hswo_run calls, plain FP32", "ms_per_step": plain_ms,
                                           "speedup_of_timed_form": plain_ms / ms_per_step,
                                           "labels_identical_to_timed_form": same}
    if args.form != "screened" and other_forms:
        say("batch256: screened form")
        so = new_outs()
        ms, _, _ = timed_steps(runner("screened", so, args.graph), stream, torch, 1, 1)
        comparisons["screened_batched"] = {"ms_per_step": ms, "speedup_of_timed_form": ms / ms_per_step,
                                           "precision": args.precision,
                                           "labels_identical_to_timed_form":
                                               all(bool(torch.equal(a, b)) for a, b in zip(so, outs))}
    if "plain_sequential" in comparisons:
        pm = comparisons["plain_sequential"]["ms_per_step"]
        out["speedup_vs_plain"] = {args.form: pm / ms_per_step,
                                   **{f: pm / v["ms_per_step"] for f, v in comparisons.items()
                                      if f != "plain_sequential"}}
    out["forms"] = comparisons
    if not args.no_cpu_baseline:
        import concurrent.futures as cf

        say("batch256: cpu baseline, oracle on whole sections for ~15 s")
        import oracle
        threads = host_threads()
        tc = time.perf_counter()
        done, same = 0, True
        # a bounded sample of whole sections (in index order) for ~15 s
        while done < len(secs) and time.perf_counter() - tc < 15.0:
            batch = list(range(done, min(len(secs), done + threads)))
            with cf.ThreadPoolExecutor(threads) as ex:
                refs = list(ex.map(lambda i: oracle.rhseg(secs[i][0], **params, n_threads=1), batch))
            for i, ref in zip(batch, refs):
                same = same and bool(np.array_equal(outs[i].cpu().numpy(), ref.labels))
            done += len(batch)
        cpu_s = time.perf_counter() - tc
        # the pairs the timed GPU form evaluates for the sampled sections (a batch over them)
        rs = hswo.hswo_run_batch(dc[:done], stats=True, **form_kwargs(args.form, args.precision), **params)
        cpu_pairs = evaluated_pairs(rs.stats, args.form)
        out["cpu_baseline"] = {"value": cpu_pairs / cpu_s, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                               "sample": f"sections 0..{done - 1} of 256, one oracle run per section on {threads} "
                                         f"threads, {cpu_s:.2f} s; rate = the pairs the timed GPU form evaluates "
                                         "for those sections over that time"}
        out["labels_identical_to_oracle_on_sample"] = same
    return out, Bmean


SWEEPS = {
    # image side at 220 bands (the paper's image-size table): leaves of 32 x 32
    "size": [dict(side=n, B=220, K=16) for n in (64, 128, 256, 512)],
    # detail at 50 x 50 x 220 (the paper's image-detail table): 4, 8 and 16 classes
    "detail": [dict(side=50, B=220, K=k) for k in (4, 8, 16)],
    # depth at 32 x 32 (the paper's band-count table)
    "bands": [dict(side=32, B=b, K=16) for b in (3, 10, 50, 100, 150, 220)],
    # work split of the adjacent sweep at 32 x 32 x 220 (the paper's block-size table): the
    # section-driver variants (edges in flight per 16-lane group) of the screened form
    "variant": [dict(side=32, B=220, K=16, variant=v) for v in (2, 4, 6)],
}


def sweep_params(side):
    L = 1
    while (side >> L) >= 32:
        L += 1
    target = 16
    return dict(connectivity=4, seam_connectivity=8, spclust_wght=0.15, spclust_max=1024,
                target_regions=target, section_regions=max(target, 64) if L > 1 else 0, rnb_levels=L,
                level_counts=[target])


def bench_sweep(args, np, torch, hswo, synth):
    """One point per configuration: the GPU call (median of 3 after a warm-up)
    and the FP64 oracle on the host's threads, on the same synthetic cube."""
    import oracle
    threads = host_threads()
    points = []
    for cfg in SWEEPS[args.sweep]:
        sc = synth.voronoi_scene(cfg["side"], cfg["side"], cfg["B"], cfg["K"], 30.0, 900 + cfg["side"] + cfg["B"])
        p = sweep_params(cfg["side"])
        kw = {k: v for k, v in p.items() if k != "rnb_levels"}
        cube = torch.from_numpy(sc.cube).cuda()
        tuning = None
        if "variant" in cfg:
            tuning = dict(driver_variant=cfg["variant"])
            form = "screened"
        else:
            form = args.form
        fk = form_kwargs(form, args.precision)
        times, res = [], None
        for k in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = hswo.rhseg_segment(cube, rnb_levels=p["rnb_levels"], stats=True, tuning=tuning, **fk, **kw)
            torch.cuda.synchronize()
            if k:
                times.append((time.perf_counter() - t0) * 1e3)
        gpu_ms = statistics.median(times)
        tc = time.perf_counter()
        ref = oracle.rhseg(sc.cube, **p, n_threads=threads)
        cpu_ms = (time.perf_counter() - tc) * 1e3
        points.append({**cfg, "form": form, "rnb_levels": p["rnb_levels"], "gpu_ms": round(gpu_ms, 3),
                       "oracle_ms": round(cpu_ms, 1), "speedup_vs_oracle": round(cpu_ms / gpu_ms, 2),
                       "labels_identical_to_oracle": bool(np.array_equal(res.labels.cpu().numpy(), ref.labels)),
                       "merges": res.stats["merges"]})
        print(json.dumps({"sweep_point": points[-1]}), file=sys.stderr, flush=True)
    return {"sweep": args.sweep, "cores": threads, "oracle": "FP64 oracle, cached mode, sections of a level on "
            f"{threads} threads", "params": "w 0.15, spectral at <= 1024 regions, 4-connectivity, 32x32 leaves, "
            "sections stop at 64, target 16; Voronoi scenes, sigma 30", "points": points}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rhseg2048_f16", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--form", default="incremental", choices=["incremental", "screened", "plain", "plain_batched"],
                    help="form of the timed steps (the others run once for the comparison)")
    ap.add_argument("--precision", default="fp16", choices=["fp32", "bf16", "fp16"],
                    help="matrix-core screen precision of the screened form (fp16: its finer rounding lets fewer "
                         "tiles through to the FP32 pass than bf16 on these workloads)")
    ap.add_argument("--criterion", default="bsmse", choices=["bsmse", "sam"],
                    help="dissimilarity: Equation 1 (bsmse) or the spectral angle (sam, incremental form only)")
    ap.add_argument("--two-merges", action="store_true",
                    help="two-merge reading of the HSEG steps (incremental form only)")
    ap.add_argument("--no-graph", dest="graph", action="store_false", help="launch eagerly instead of a hipGraph")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="library default execution settings instead of the autotuner's (the first warm-up call "
                         "tunes the timed form's settings: workgroups per section, which levels run persistent, "
                         "the row-stage grid, the section-driver variant)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the runs of the forms not timed")
    ap.add_argument("--single-thread-oracle", action="store_true",
                    help="also time the oracle on one host thread (the paper's sequential baseline; ~45 s on "
                         "rhseg512)")
    ap.add_argument("--sweep", choices=sorted(SWEEPS),
                    help="instead of the benchmark: GPU vs oracle over one of the paper-style sweeps")
    ap.add_argument("--no-sweeps", action="store_true",
                    help="skip the paper-style sweep points (band count, image detail, adjacent-sweep variant) "
                         "appended to the benchmark line")
    ap.add_argument("--no-kernel-times", action="store_true",
                    help="skip the per-kernel timing step (no roofline object)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only copy this many bytes device to device (3 times) and exit: the known-size "
                         "reference for the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if (args.criterion != "bsmse" or args.two_merges) and args.form != "incremental":
        ap.error("--criterion sam and --two-merges are implemented in the incremental form only")

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "one GPU only: sharding the sections of a recursion level across GPUs is not "
                                   "implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_bytes:
        n = args.copy_bytes // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "copies": 3}))
        return

    from paper_2106_12942_amd import hswo, synth

    if args.sweep:
        print(json.dumps(bench_sweep(args, np, torch, hswo, synth)))
        return
    if args.workload == "batch256":
        body, _ = bench_batch(args, np, torch, hswo, synth)
    else:
        body, _ = bench_rhseg(args, np, torch, hswo, synth)
    out = {"metric": "RHSEG wall time + dissimilarity pairs/s, MFMA+batched vs plain, same labels",
           "value": body.pop("value"), "unit": body.pop("unit"), "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": body.pop("ms_per_step"), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.form == "incremental" else (f"f32+{args.precision} screens, f64 decisions"
                                                              if args.precision != "fp32" else "f32 screen, f64 decisions"),
           "data": "synthetic"}
    out.update(body)
    if not args.no_sweeps:
        # the paper-style sweeps (GPU against the oracle, labels compared), small enough to ride along
        out["sweeps"] = {}
        for name in ("bands", "detail", "variant"):
            a = argparse.Namespace(**vars(args))
            a.sweep = name
            out["sweeps"][name] = bench_sweep(a, np, torch, hswo, synth)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
