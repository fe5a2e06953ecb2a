#!/usr/bin/env python3
"""Benchmark of the RHSEG hot path on one MI355X.

One step = one rhseg_segment() call through the C ABI on a device-resident
synthetic cube: every leaf section's HSEG loop, the reassembly of each
recursion level and the parents' HSEG loops, up to the label maps of the
requested hierarchy levels (all of the merge loop runs in the HIP kernels).

Default workload (rhseg512): 512 x 512 x 128 float32 Voronoi scene (200
classes, sigma 30, seed 202), rnb_levels 4 (64 x 64 leaves), w = 0.5,
spectral stage at <= 1024 regions, sections stop at 256, 8 output levels.

Output: one JSON line. `value` is dissimilarity pairs per second (adjacent
pairs screened + non-adjacent pairs screened, per the kernels' own counters,
divided by the wall time of a step). The line also carries the wall time per
step, the roofline fraction of the section-driver kernel (live hipEvent
timing of its launches), and the CPU oracle timed on the same workload.
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

# MI355X peaks (per the chip's published figures / unit counts)
PEAK_HBM_GBS = 8000.0
# FP32 vector arithmetic without packed-FP32 instructions (which this build
# keeps out of generated code): 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_VALU_TFLOPS = 78.6
PEAK_BF16_MFMA_TFLOPS = 2500.0

WORKLOAD_DESC = {
    "rhseg512": "512x512x128 f32 Voronoi (200 classes, sigma 30, seed 202); rnb_levels 4 (64x64 leaves); "
                "w 0.5; spectral at <=1024 regions; sections stop at 256; target 8; 8 levels",
    "hswo64": "64x64x32 f32 Voronoi (40 classes, sigma 20, seed 101); one section; w 0.5; spectral at "
              "<=256 regions; target 2; 11 levels",
}


def traffic_from_profiles(workload: str, precision: str):
    """HBM bytes per section-driver launch, if a counter summary for exactly
    this kernel build and workload is committed under profiles/."""
    path = os.path.join(ROOT, "profiles", f"traffic_section_driver_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("hbm_bytes_per_launch:"):
            return float(line.split(":", 1)[1])
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rhseg512", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--precision", default="fp16", choices=["fp32", "bf16", "fp16"],
                    help="screen of the spectral stage for the timed steps (fp32 = plain path)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the leaf sections of a level would be "
                                   "sharded across GPUs (see DESIGN.md), which is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2106_12942_amd import hswo, synth

    sc, params = synth.workload(args.workload)
    cube_h = sc.cube
    H, W, B = cube_h.shape
    dev = torch.device("cuda:0")
    cube = torch.from_numpy(cube_h).to(dev)
    L = params["rnb_levels"]
    kw = {k: v for k, v in params.items() if k != "rnb_levels"}

    def step():
        return hswo.rhseg_segment(cube, rnb_levels=L, precision=args.precision, stats=True, **kw)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    walls, drv_ms, drv_n, res = [], 0.0, 0, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        res = step()  # stats=True: the call synchronises its stream before returning
        walls.append((time.perf_counter() - ts) * 1e3)
        drv_ms += res.stats["ms_driver"]
        drv_n += res.stats["driver_launches"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    st = res.stats
    pairs = st["adjacent_pairs"] + st["spectral_pairs"]
    value = pairs / (ms_per_step / 1e3)

    # dominant kernel: the section driver. Algorithmic work = 3 flops per band
    # (difference, square, accumulate) per screened pair; spectral pairs
    # dominate, so the bound is FP32 vector arithmetic.
    flops_per_step = 3.0 * B * pairs
    launches_per_step = drv_n / args.steps
    avg_launch_ms = drv_ms / drv_n
    flops_per_launch = flops_per_step / launches_per_step
    achieved = flops_per_launch / (avg_launch_ms / 1e3) / 1e12
    peak = PEAK_FP32_VALU_TFLOPS
    traffic = traffic_from_profiles(args.workload, args.precision)
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 5), "traffic": traffic,
                "kernel": "k_section_driver", "launches_per_step": launches_per_step,
                "avg_launch_ms": round(avg_launch_ms, 4),
                "algorithmic_flops_per_launch": flops_per_launch}

    stage_ms = {k: round(st[k], 2) for k in ("ms_adjacent", "ms_mfma_screen", "ms_fp32_spectral", "ms_merge")}
    labels = res.labels.cpu().numpy()
    plain = None
    if args.precision != "fp32" and not args.no_plain:
        # the plain FP32 path on the same input, for the precision form's speed-up
        ts = time.perf_counter()
        rp = hswo.rhseg_segment(cube, rnb_levels=L, precision="fp32", stats=True, **kw)
        plain_ms = (time.perf_counter() - ts) * 1e3
        plain = {"ms_per_step": plain_ms, "speedup_of_timed_form": plain_ms / ms_per_step,
                 "labels_identical_to_timed_form": bool(np.array_equal(rp.labels.cpu().numpy(), labels)),
                 "stage_ms": {k: round(rp.stats[k], 2) for k in stage_ms}}
    out = {
        "metric": "RHSEG wall time + dissimilarity pairs/s, MFMA+batched vs plain, same labels",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "wall_ms_median": statistics.median(walls),
        "wall_ms_min": min(walls),
        "wall_ms_max": max(walls),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 screen + f64 decisions",
        "data": "synthetic",
        "config": {"workload": args.workload, "desc": WORKLOAD_DESC[args.workload], "H": H, "W": W, "B": B,
                   "precision": args.precision,
                   "form": "per-level section driver, " + ("plain FP32 screen" if args.precision == "fp32" else
                                                           f"{args.precision} matrix-core spectral screen")},
        "pairs_per_step": pairs,
        "merges_per_step": st["merges"],
        "exact_rechecks_per_step": st["exact_rechecks"],
        "roofline": roofline,
        "stage_ms_summed_over_sections": stage_ms,
        "fp32_tiles_per_step": st["fp32_tiles"],
        "mfma_super_tiles_per_step": st["mfma_tiles"],
        "plain_fp32": plain,
    }

    if not args.no_cpu_baseline:
        import oracle
        threads = os.cpu_count() or 1
        tc = time.perf_counter()
        ref = oracle.rhseg(cube_h, **params, n_threads=threads)
        cpu_s = time.perf_counter() - tc
        out["cpu_baseline"] = {"value": pairs / cpu_s, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                               "sample": f"the full {args.workload} workload, FP64 oracle (cached mode, "
                                         f"sections of a level on {threads} threads), {cpu_s:.2f} s; "
                                         "pairs counted as the GPU path screens them"}
        out["labels_identical_to_oracle"] = bool(np.array_equal(labels, ref.labels))
        out["gpu_vs_oracle_speedup"] = cpu_s * 1e3 / ms_per_step
    print(json.dumps(out))


if __name__ == "__main__":
    main()
