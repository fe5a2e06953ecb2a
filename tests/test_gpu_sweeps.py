"""GPU parity at the points of the paper-style sweeps (Section 5: the band
count at 32 x 32 pixels, the image detail at 50 x 50 x 220, the block shape
of the adjacent sweep at 32 x 32 x 220), the same synthetic scenes and
parameters as the benchmark's --sweep runs. Every point's merge log and
label maps must equal the oracle's, in the incremental form and in the BF16
matrix-core screened form; the GPU and oracle times are printed per point."""
import time

import numpy as np
import pytest

import bench
import oracle
from paper_2106_12942_amd import hswo, synth
from tests.test_gpu_parity import _say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

POINTS = [(name, i) for name in ("bands", "detail", "variant") for i in range(len(bench.SWEEPS[name]))]


@pytest.mark.parametrize("name,i", POINTS)
def test_sweep_point_matches_oracle(name, i):
    cfg = bench.SWEEPS[name][i]
    sc = synth.voronoi_scene(cfg["side"], cfg["side"], cfg["B"], cfg["K"], 30.0, 900 + cfg["side"] + cfg["B"])
    p = bench.sweep_params(cfg["side"])
    t0 = time.perf_counter()
    ref = oracle.rhseg(sc.cube, **p, n_threads=1)
    cpu_ms = (time.perf_counter() - t0) * 1e3
    kw = {k: v for k, v in p.items() if k != "rnb_levels"}
    cube = torch.from_numpy(sc.cube).cuda()
    forms = ["screened"] if "variant" in cfg else ["incremental", "screened"]
    for form in forms:
        tuning = dict(driver_variant=cfg["variant"]) if "variant" in cfg else None
        fk = bench.form_kwargs(form, "bf16")
        res = None
        for _ in range(2):  # the second call is timed (the first builds the workspace)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = hswo.rhseg_segment(cube, rnb_levels=p["rnb_levels"], merge_log=True, stats=True, tuning=tuning,
                                     **fk, **kw)
            torch.cuda.synchronize()
            gpu_ms = (time.perf_counter() - t0) * 1e3
        _say(f"[gpu] sweep {name} {cfg} form {form}: {res.stats['merges']} merges, GPU {gpu_ms:.2f} ms, "
             f"oracle (1 thread) {cpu_ms:.1f} ms")
        n = len(ref.log)
        assert res.stats["merges"] == n
        assert np.array_equal(res.log[:n], ref.log), f"{name} {cfg} {form}: merge log differs"
        assert np.array_equal(res.labels.cpu().numpy(), ref.labels), f"{name} {cfg} {form}: labels differ"
