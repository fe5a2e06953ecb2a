"""ctypes wrapper around the C++ oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hswo_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

MERGE_DTYPE = np.dtype([("lo", "<i4"), ("hi", "<i4"), ("kind", "<i4"), ("r_after", "<i4"), ("d2", "<f8")])


class _Params(ctypes.Structure):
    _fields_ = [
        ("connectivity", ctypes.c_int32),
        ("seam_connectivity", ctypes.c_int32),
        ("spclust_wght", ctypes.c_float),
        ("spclust_max", ctypes.c_int32),
        ("target_regions", ctypes.c_int32),
        ("section_regions", ctypes.c_int32),
        ("rnb_levels", ctypes.c_int32),
        ("n_levels", ctypes.c_int32),
        ("level_counts", ctypes.POINTER(ctypes.c_int32)),
        ("brute", ctypes.c_int32),
        ("n_threads", ctypes.c_int32),
        ("criterion", ctypes.c_int32),
        ("two_merges", ctypes.c_int32),
        ("multi_merge", ctypes.c_int32),
        ("progress", ctypes.c_void_p),
    ]


_PROGRESS = ctypes.CFUNCTYPE(None, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32)


def _progress_printer(tag: str):
    """Print a line when a recursion level finishes and about every tenth of
    its sections in between (called from the oracle's worker threads, one at a
    time)."""
    import sys
    import time
    t0 = time.perf_counter()

    def cb(depth, done, total):
        if done == total or done % max(1, total // 10) == 0:
            print(f"[oracle] {tag} depth {depth}: {done}/{total} sections ({time.perf_counter() - t0:.0f} s)",
                  flush=True)
            sys.stdout.flush()
    return _PROGRESS(cb)


CRITERIA = {"bsmse": 0, "sam": 1}


def lib_path() -> str:
    return _LIB


def build(sanitize: bool = False, src: Optional[str] = None, out: Optional[str] = None) -> str:
    """Compile the oracle with g++ (no fast-math, no FMA contraction)."""
    if out is None:
        out = _LIB if not sanitize else os.path.join(_HERE, "liboracle_asan.so")
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-I", _HERE, "-o", out, src or _SRC, "-lpthread"]
    if sanitize:
        cmd[3:3] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    subprocess.check_call(cmd)
    return out


_lib = None


def _load(path: Optional[str] = None):
    """Load the built oracle (building it first if needed). ``path`` loads
    another build of the same source instead (used by the mutation tests)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    lib.oracle_d2.restype = ctypes.c_double
    lib.oracle_d2.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
    lib.oracle_sam.restype = ctypes.c_double
    lib.oracle_sam.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    lib.oracle_rhseg.restype = ctypes.c_int
    lib.oracle_rhseg.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p]
    return lib


def criterion_d2(Si: np.ndarray, Sj: np.ndarray, ni: int, nj: int) -> float:
    """Canonical squared criterion of Equation 1 from band sums and counts."""
    Si = np.ascontiguousarray(Si, dtype=np.float64)
    Sj = np.ascontiguousarray(Sj, dtype=np.float64)
    return _load().oracle_d2(Si.ctypes.data, Sj.ctypes.data, int(ni), int(nj), int(Si.size))


def criterion_sam(Si: np.ndarray, Sj: np.ndarray) -> float:
    """Spectral angle criterion 1 - sign(c) c^2 (c = cosine) from band sums."""
    Si = np.ascontiguousarray(Si, dtype=np.float64)
    Sj = np.ascontiguousarray(Sj, dtype=np.float64)
    return _load().oracle_sam(Si.ctypes.data, Sj.ctypes.data, int(Si.size))


@dataclasses.dataclass
class OracleResult:
    labels: np.ndarray        # [n_levels, H, W] int32
    log: np.ndarray           # structured MERGE_DTYPE
    region_label: np.ndarray  # final regions of the top pass
    region_n: np.ndarray
    region_S: np.ndarray      # [R, B] float64


def rhseg(cube: np.ndarray, *, connectivity: int = 4, seam_connectivity: int = 8,
          spclust_wght: float = 0.0, spclust_max: int = 0, target_regions: int = 1,
          section_regions: int = 0, rnb_levels: int = 1,
          level_counts: Optional[Sequence[int]] = None, brute: bool = False,
          n_threads: Optional[int] = None, lib: Optional[str] = None, criterion: str = "bsmse",
          two_merges: bool = False, multi_merge: bool = False, progress: Optional[str] = None,
          **_ignored) -> OracleResult:
    """Run the oracle on a host H x W x B cube (float32, or float16 widened exactly).
    progress: a tag; when given, a line is printed as the sections of each
    recursion level finish."""
    cube = np.asarray(cube)
    if cube.dtype == np.float16:
        cube = cube.astype(np.float32)  # every float16 value is a float32 value
    cube = np.ascontiguousarray(cube, dtype=np.float32)
    H, W, B = cube.shape
    if level_counts is None:
        level_counts = [target_regions]
    lc = np.ascontiguousarray(level_counts, dtype=np.int32)
    p = _Params()
    p.connectivity = connectivity
    p.seam_connectivity = seam_connectivity
    p.spclust_wght = spclust_wght
    p.spclust_max = spclust_max
    p.target_regions = target_regions
    p.section_regions = section_regions
    p.rnb_levels = rnb_levels
    p.n_levels = len(lc)
    p.level_counts = lc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    p.brute = 1 if brute else 0
    p.n_threads = n_threads if n_threads is not None else (os.cpu_count() or 1)
    p.criterion = CRITERIA[criterion]
    p.two_merges = 1 if two_merges else 0
    p.multi_merge = 1 if multi_merge else 0
    cb = _progress_printer(progress) if progress else None
    p.progress = ctypes.cast(cb, ctypes.c_void_p) if cb is not None else None
    labels = np.full((len(lc), H, W), -1, dtype=np.int32)
    log = np.zeros(H * W, dtype=MERGE_DTYPE)
    n_log = ctypes.c_int64(0)
    out_R = ctypes.c_int32(0)
    out_label = np.zeros(H * W, dtype=np.int32)
    out_n = np.zeros(H * W, dtype=np.int64)
    # final band sums are returned only for small cubes (one row per pixel of capacity)
    out_S = np.zeros((H * W, B), dtype=np.float64) if H * W * B <= (1 << 24) else None
    rc = _load(lib).oracle_rhseg(cube.ctypes.data, H, W, B, ctypes.byref(p), labels.ctypes.data,
                              log.ctypes.data, ctypes.byref(n_log), ctypes.byref(out_R),
                              out_label.ctypes.data, out_n.ctypes.data,
                              out_S.ctypes.data if out_S is not None else None)
    if rc != 0:
        raise ValueError(f"oracle_rhseg rejected its parameters (rc={rc})")
    R = out_R.value
    return OracleResult(labels=labels, log=log[: n_log.value].copy(), region_label=out_label[:R].copy(),
                        region_n=out_n[:R].copy(),
                        region_S=out_S[:R].copy() if out_S is not None else np.zeros((0, B)))
