#!/usr/bin/env python3
"""Benchmark of the RHSEG hot path on one MI355X.

One step = one call through the C ABI on device-resident synthetic input,
covering every merge of every section: the HSEG loops of the leaf sections,
the reassembly of each recursion level, the parents' loops, and the label
maps of the requested hierarchy levels (all of it in the HIP kernels).

Workloads
  rhseg512 (default): 512 x 512 x 128 float32 Voronoi scene (200 classes,
      sigma 30, seed 202), rnb_levels 4 (64 x 64 leaves), w 0.5, spectral
      stage at <= 1024 regions, sections stop at 256, 8 output levels.
  hswo64: 64 x 64 x 32 float32 Voronoi (40 classes, sigma 20, seed 101), one
      section, spectral at <= 256, down to 2 regions, 11 levels.
  batch256: 256 independent sections, side U{32..128}, bands U{64,96,..,224},
      10..120 Voronoi classes, sigma 30 (seed 404000+s), each merged down to
      256 regions (w 0.5, spectral at <= 1024) -- one hswo_run_batch call.

Forms: the timed steps use the matrix-core screened form (fp16 by default)
with levels batched into one launch (persistent) or one launch sequence
(wide), replayed from a hipGraph; the plain FP32 path is run on the same
input for the comparison.

Output: one JSON line. `value` is dissimilarity pairs per second (adjacent
pairs screened + non-adjacent pairs screened, from the kernels' counters,
over the wall time of a step).
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

WORKLOAD_DESC = {
    "rhseg512": "512x512x128 f32 Voronoi (200 classes, sigma 30, seed 202); rnb_levels 4 (64x64 leaves); "
                "w 0.5; spectral at <=1024 regions; sections stop at 256; target 8; 8 levels",
    "hswo64": "64x64x32 f32 Voronoi (40 classes, sigma 20, seed 101); one section; w 0.5; spectral at "
              "<=256 regions; target 2; 11 levels",
    "batch256": "256 independent f32 sections, side U{32..128}, bands U{64..224 step 32}, 10-120 Voronoi "
                "classes, sigma 30, seeds 404000+s; each merged to 256 regions; w 0.5; spectral at <=1024",
}


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


def stage_dict(st):
    return {k: round(st[k], 2) for k in ("ms_adjacent", "ms_mfma_screen", "ms_fp32_spectral", "ms_merge")}


def roofline_of(st, B, steps_ms, launches, tag):
    """Roofline of the section-driver launches: algorithmic work = 3 flops
    per band (difference, square, accumulate) per screened pair, over the
    live-timed driver time; screened pairs are dominated by the spectral
    all-pairs stage, so the bound is FP32 vector arithmetic."""
    pairs = st["adjacent_pairs"] + st["spectral_pairs"]
    flops = 3.0 * B * pairs
    achieved = flops / (st["ms_driver"] / 1e3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 5), "traffic": traffic_from_profiles(tag),
            "kernel": "section driver launches (persistent driver + wide-mode kernels)",
            "launches_per_step": launches, "avg_launch_ms": round(st["ms_driver"] / max(launches, 1), 4),
            "algorithmic_flops_per_launch": flops / max(launches, 1)}


def bench_rhseg(args, np, torch, hswo, synth):
    sc, params = synth.workload(args.workload)
    cube_h = sc.cube
    H, W, B = cube_h.shape
    dev = torch.device("cuda:0")
    cube = torch.from_numpy(cube_h).to(dev)
    L = params["rnb_levels"]
    kw = {k: v for k, v in params.items() if k != "rnb_levels"}
    stream = torch.cuda.Stream(dev)
    ws = hswo.Workspace()
    labels = torch.empty((len(params["level_counts"]), H, W), dtype=torch.int32, device=dev)

    def step(stats=True):
        return hswo.rhseg_segment(cube, rnb_levels=L, precision=args.precision, stats=stats, stream=stream,
                                  workspace=ws, labels_out=labels, graph=args.graph, autotune=args.autotune, **kw)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
        stream.synchronize()
        torch.cuda.synchronize()
        walls, res = [], None
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            res = step()  # stats=True: the call synchronises its stream before returning
            walls.append((time.perf_counter() - ts) * 1e3)
        stream.synchronize()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    st = res.stats
    pairs = st["adjacent_pairs"] + st["spectral_pairs"]
    out = {
        "value": pairs / (ms_per_step / 1e3), "unit": "pairs/s", "ms_per_step": ms_per_step,
        "wall_ms_median": statistics.median(walls), "wall_ms_min": min(walls), "wall_ms_max": max(walls),
        "config": {"workload": args.workload, "desc": WORKLOAD_DESC[args.workload], "H": H, "W": W, "B": B,
                   "precision": args.precision, "graph": args.graph, "autotune": args.autotune,
                   "driver_variant": st["driver_variant"]},
        "pairs_per_step": pairs, "merges_per_step": st["merges"], "exact_rechecks_per_step": st["exact_rechecks"],
        "fp32_tiles_per_step": st["fp32_tiles"], "mfma_super_tiles_per_step": st["mfma_tiles"],
        "stage_ms_persistent_levels_summed_over_sections": stage_dict(st),
        "roofline": roofline_of(st, B, ms_per_step, st["driver_launches"], f"{args.workload}_{args.precision}"),
    }
    lab = labels.cpu().numpy()
    if not args.no_plain and args.precision != "fp32":
        ts = time.perf_counter()
        rp = hswo.rhseg_segment(cube, rnb_levels=L, precision="fp32", stats=True, **kw)
        plain_ms = (time.perf_counter() - ts) * 1e3
        out["plain_fp32"] = {"ms_per_step": plain_ms, "speedup_of_timed_form": plain_ms / ms_per_step,
                             "labels_identical_to_timed_form": bool(np.array_equal(rp.labels.cpu().numpy(), lab))}
    if not args.no_incremental:
        # the incremental adjacent stage (cached exact per-edge D2): same merges, fewer pairs scored
        with torch.cuda.stream(stream):
            inc_lab = torch.empty_like(labels)
            hswo.rhseg_segment(cube, rnb_levels=L, precision=args.precision, stream=stream, labels_out=inc_lab,
                               incremental=True, **kw)
            stream.synchronize()
            ts = time.perf_counter()
            ri = hswo.rhseg_segment(cube, rnb_levels=L, precision=args.precision, stats=True, stream=stream,
                                    labels_out=inc_lab, incremental=True, **kw)
            inc_ms = (time.perf_counter() - ts) * 1e3
        out["incremental_form"] = {"ms_per_step": inc_ms, "speedup_vs_timed_form": ms_per_step / inc_ms,
                                   "labels_identical_to_timed_form": bool(torch.equal(inc_lab, labels)),
                                   "exact_rechecks": ri.stats["exact_rechecks"]}
    if not args.no_cpu_baseline:
        import oracle
        threads = os.cpu_count() or 1
        tc = time.perf_counter()
        ref = oracle.rhseg(cube_h, **params, n_threads=threads)
        cpu_s = time.perf_counter() - tc
        out["cpu_baseline"] = {"value": pairs / cpu_s, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                               "sample": f"the full {args.workload} workload, FP64 oracle (cached mode, sections of "
                                         f"a level on {threads} threads), {cpu_s:.2f} s; pairs counted as the GPU "
                                         "path screens them"}
        out["labels_identical_to_oracle"] = bool(np.array_equal(lab, ref.labels))
        out["gpu_vs_oracle_speedup"] = cpu_s * 1e3 / ms_per_step
    return out, B


def bench_batch(args, np, torch, hswo, synth):
    secs = synth.batch_sections(256)
    params = dict(synth.BATCH_PARAMS)
    params.pop("rnb_levels", None)
    dev = torch.device("cuda:0")
    dc = [torch.from_numpy(c).to(dev) for c, _ in secs]
    stream = torch.cuda.Stream(dev)
    ws = hswo.Workspace()
    outs = [torch.empty((len(params["level_counts"]), c.shape[0], c.shape[1]), dtype=torch.int32, device=dev)
            for c in dc]

    def step():
        return hswo.hswo_run_batch(dc, precision=args.precision, stats=True, stream=stream, workspace=ws,
                                   labels_out=outs, graph=args.graph, autotune=args.autotune, **params)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
        stream.synchronize()
        walls, res = [], None
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            res = step()
            walls.append((time.perf_counter() - ts) * 1e3)
        stream.synchronize()
        elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    st = res.stats
    pairs = st["adjacent_pairs"] + st["spectral_pairs"]
    Bmean = float(np.mean([c.shape[2] for c, _ in secs]))
    out = {
        "value": pairs / (ms_per_step / 1e3), "unit": "pairs/s", "ms_per_step": ms_per_step,
        "wall_ms_median": statistics.median(walls), "wall_ms_min": min(walls), "wall_ms_max": max(walls),
        "config": {"workload": "batch256", "desc": WORKLOAD_DESC["batch256"], "sections": len(secs),
                   "precision": args.precision, "graph": args.graph, "autotune": args.autotune,
                   "driver_variant": st["driver_variant"]},
        "pairs_per_step": pairs, "merges_per_step": st["merges"],
        "stage_ms_persistent_levels_summed_over_sections": stage_dict(st),
    }
    # roofline with the mean band count (the pair counts mix sections)
    out["roofline"] = roofline_of(st, Bmean, ms_per_step, st["driver_launches"], f"batch256_{args.precision}")
    per_pairs = []
    if not args.no_plain:
        # the plain path: 256 sequential hswo_run calls, FP32 screen
        torch.cuda.synchronize()
        ts = time.perf_counter()
        same = True
        for i, c in enumerate(dc):
            r = hswo.hswo_run(c, precision="fp32", stats=True, **params)
            per_pairs.append(r.stats["adjacent_pairs"] + r.stats["spectral_pairs"])
            same = same and bool(torch.equal(r.labels, outs[i]))
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - ts) * 1e3
        out["plain_fp32"] = {"form": "256 sequential hswo_run calls", "ms_per_step": plain_ms,
                             "speedup_of_timed_form": plain_ms / ms_per_step, "labels_identical_to_timed_form": same}
    if not args.no_cpu_baseline:
        import oracle
        threads = os.cpu_count() or 1
        tc = time.perf_counter()
        done, same, cpu_pairs = 0, True, 0
        # a bounded sample of whole sections (in index order) for ~15 s
        while done < len(secs) and time.perf_counter() - tc < 15.0:
            batch = list(range(done, min(len(secs), done + threads)))
            import concurrent.futures as cf
            with cf.ThreadPoolExecutor(threads) as ex:
                refs = list(ex.map(lambda i: oracle.rhseg(secs[i][0], **params, n_threads=1), batch))
            for i, ref in zip(batch, refs):
                same = same and bool(np.array_equal(outs[i].cpu().numpy(), ref.labels))
                if per_pairs:
                    cpu_pairs += per_pairs[i]
            done += len(batch)
        cpu_s = time.perf_counter() - tc
        out["cpu_baseline"] = {"value": (cpu_pairs / cpu_s) if cpu_pairs else None, "unit": "pairs/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"sections 0..{done - 1} of 256, one oracle run per section on {threads} "
                                         f"threads, {cpu_s:.2f} s"}
        out["labels_identical_to_oracle_on_sample"] = same
    return out, Bmean


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rhseg512", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--precision", default="fp16", choices=["fp32", "bf16", "fp16"],
                    help="screen of the spectral stage for the timed steps (fp32 = plain path)")
    ap.add_argument("--no-graph", dest="graph", action="store_false", help="launch eagerly instead of a hipGraph")
    ap.add_argument("--autotune", action="store_true", help="autotune the section-driver variant first")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 comparison run")
    ap.add_argument("--no-incremental", action="store_true", help="skip the incremental-adjacent run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the sections of a recursion level would be "
                                   "sharded across GPUs (see DESIGN.md), which is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2106_12942_amd import hswo, synth

    if args.workload == "batch256":
        body, _ = bench_batch(args, np, torch, hswo, synth)
    else:
        body, _ = bench_rhseg(args, np, torch, hswo, synth)
    out = {"metric": "RHSEG wall time + dissimilarity pairs/s, MFMA+batched vs plain, same labels",
           "value": body.pop("value"), "unit": body.pop("unit"), "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": body.pop("ms_per_step"), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f16 screens, f64 decisions",
           "data": "synthetic"}
    out.update(body)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
