"""Thin ctypes binding over libhswo (include/hswo.h).

Argument marshalling only: every step of HSWO / HSEG / RHSEG runs in the HIP
kernels of libhswo. PyTorch provides device memory and the stream. There is
no fallback: if the library is missing, loading it raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhswo.so")

HSWO_OK = 0
HSWO_E_INVAL = -1
HSWO_E_NOMEM = -2
HSWO_E_DEVICE = -3
HSWO_E_NONFINITE = -4
HSWO_E_UNSUPPORTED = -5

HSWO_F32 = 0
HSWO_F16 = 1

PREC = {"fp32": 0, "bf16": 1, "fp16": 2}
HSWO_FLAG_MERGE_LOG = 1
HSWO_FLAG_GRAPH = 2
HSWO_FLAG_AUTOTUNE = 4
HSWO_FLAG_INCREMENTAL = 8
HSWO_FLAG_KERNEL_TIMES = 16
HSWO_FLAG_SEQUENTIAL_SECTIONS = 32
HSWO_FLAG_TWO_MERGES = 64
HSWO_FLAG_DEBUG_VERIFY_BOUND = 128
HSWO_FLAG_MULTI_MERGE = 256

HSWO_CRIT_BSMSE = 0
HSWO_CRIT_SAM = 1
CRIT = {"bsmse": HSWO_CRIT_BSMSE, "sam": HSWO_CRIT_SAM}
KERNEL_KINDS = ["section_driver", "wide_adj", "wide_decide", "wide_mfma", "wide_fp32", "wide_finish", "wide_rows",
                "rowcache_prep", "matrix_fill"]

MERGE_DTYPE = np.dtype([("lo", "<i4"), ("hi", "<i4"), ("kind", "<i4"), ("r_after", "<i4"), ("d2", "<f8")])
VERIFY_DTYPE = np.dtype([("lo", "<i4"), ("hi", "<i4"), ("stage", "<i4"), ("r", "<i4"), ("screen", "<f8"),
                         ("lower", "<f8"), ("upper", "<f8"), ("d2", "<f8")])
SCREEN_STAGES = {0: "adjacent_fp32", 1: "spectral_fp32", 2: "spectral_16bit"}
TUNING_FIELDS = ["wide_max_sections", "wide_groups", "rows_grid", "hybrid", "bare_bounds", "driver_variant",
                 "row_matrix"]

EXPORTS = ["hswo_version", "hswo_last_error", "hswo_workspace_bytes", "hswo_run", "rhseg_segment",
           "hswo_batch_workspace_bytes", "hswo_run_batch", "rhseg_segment_noalloc"]
# device scratch of rhseg_segment_noalloc (the library's static array, per GPU)
HSWO_NOALLOC_SCRATCH_BYTES = 256 << 20


class Tuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in TUNING_FIELDS]

    def as_dict(self):
        return {f: getattr(self, f) for f in TUNING_FIELDS}


class Params(ctypes.Structure):
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
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("criterion", ctypes.c_int32),
        ("screen_topk", ctypes.c_int32),
        ("verify", ctypes.c_void_p),
        ("verify_cap", ctypes.c_int64),
        ("tuning", ctypes.POINTER(Tuning)),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("merges", ctypes.c_int64),
        ("iterations", ctypes.c_int64),
        ("adjacent_pairs", ctypes.c_int64),
        ("spectral_pairs", ctypes.c_int64),
        ("exact_rechecks", ctypes.c_int64),
        ("tile_rescans", ctypes.c_int64),
        ("fp32_tiles", ctypes.c_int64),
        ("mfma_tiles", ctypes.c_int64),
        ("driver_launches", ctypes.c_int64),
        ("driver_variant", ctypes.c_int64),
        ("ms_total", ctypes.c_double),
        ("ms_driver", ctypes.c_double),
        ("ms_adjacent", ctypes.c_double),
        ("ms_mfma_screen", ctypes.c_double),
        ("ms_fp32_spectral", ctypes.c_double),
        ("ms_merge", ctypes.c_double),
        ("ms_kernel", ctypes.c_double * 9),
        ("kernel_launches", ctypes.c_int64 * 9),
        ("kernel_work", ctypes.c_int64 * 9),
        ("ms_event_pair_overhead", ctypes.c_double),
        ("nonfinite_values", ctypes.c_int64),
        ("screen_iterations", ctypes.c_int64),
        ("screen_fallbacks", ctypes.c_int64),
        ("verify_records", ctypes.c_int64),
        ("row_bounded_pairs", ctypes.c_int64),
        ("tuning", Tuning),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            if k in ("ms_kernel", "kernel_launches", "kernel_work"):
                v = list(v)
            elif k == "tuning":
                v = v.as_dict()
            d[k] = v
        return d


class Section(ctypes.Structure):
    _fields_ = [
        ("cube", ctypes.c_void_p),
        ("H", ctypes.c_int32),
        ("W", ctypes.c_int32),
        ("B", ctypes.c_int32),
        ("labels", ctypes.c_void_p),
        ("merge_log", ctypes.c_void_p),
    ]


class HswoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libhswo error {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libhswo.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # libhswo links the system HIP runtime, torch its own copy; the device
        # must be opened by torch's first (the other order leaves torch with no
        # GPU), so a process that has a GPU initialises torch's before loading
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2106_12942_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        lib.hswo_version.restype = ctypes.c_int
        lib.hswo_last_error.restype = ctypes.c_char_p
        lib.hswo_workspace_bytes.restype = sz
        lib.hswo_workspace_bytes.argtypes = [i32, i32, i32, i32, ctypes.POINTER(Params)]
        lib.hswo_run.restype = ctypes.c_int
        lib.hswo_run.argtypes = [vp, i32, i32, i32, i32, ctypes.POINTER(Params), vp, vp,
                                 ctypes.POINTER(Stats), vp, sz, vp]
        lib.rhseg_segment.restype = ctypes.c_int
        lib.rhseg_segment.argtypes = [vp, i32, i32, i32, i32, ctypes.POINTER(Params), i32, vp, vp,
                                      ctypes.POINTER(Stats), vp, sz, vp]
        lib.hswo_batch_workspace_bytes.restype = sz
        lib.hswo_batch_workspace_bytes.argtypes = [i32, ctypes.POINTER(Section), i32, ctypes.POINTER(Params)]
        lib.hswo_run_batch.restype = ctypes.c_int
        lib.hswo_run_batch.argtypes = [i32, ctypes.POINTER(Section), i32, ctypes.POINTER(Params),
                                       ctypes.POINTER(Stats), vp, sz, vp]
        lib.rhseg_segment_noalloc.restype = ctypes.c_int
        lib.rhseg_segment_noalloc.argtypes = [vp, i32, i32, i32, i32, ctypes.POINTER(Params), i32, vp, vp,
                                              ctypes.POINTER(Stats), vp]
        _lib = lib
    return _lib


def last_error() -> str:
    return load().hswo_last_error().decode()


# hswo_tuning fields applied to calls that pass no tuning of their own (None:
# the library's defaults). The library itself reads no environment.
DEFAULT_TUNING: Optional[dict] = None


def make_tuning(tuning: Optional[dict]) -> Optional[Tuning]:
    """hswo_tuning from a dict of its fields (missing ones -1: library default or autotuned)."""
    if tuning is None:
        return None
    unknown = set(tuning) - set(TUNING_FIELDS)
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    return Tuning(*[int(tuning.get(f, -1)) for f in TUNING_FIELDS])


def make_params(*, connectivity=4, seam_connectivity=8, spclust_wght=0.0, spclust_max=0, target_regions=1,
                section_regions=0, rnb_levels=1, level_counts: Optional[Sequence[int]] = None,
                precision="fp32", merge_log=False, graph=False, autotune=False, incremental=False,
                kernel_times=False, sequential=False, criterion="bsmse", two_merges=False, multi_merge=False,
                screen_topk=0, verify_ptr=None, verify_cap=0, tuning: Optional[dict] = None, **_ignored):
    counts = list(level_counts) if level_counts is not None else [target_regions]
    arr = (ctypes.c_int32 * len(counts))(*counts)
    tu = make_tuning(tuning if tuning is not None else DEFAULT_TUNING)
    p = Params(connectivity, seam_connectivity, spclust_wght, spclust_max, target_regions, section_regions,
               rnb_levels, len(counts), ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32)),
               PREC[precision] if isinstance(precision, str) else int(precision),
               (HSWO_FLAG_MERGE_LOG if merge_log else 0) | (HSWO_FLAG_GRAPH if graph else 0) |
               (HSWO_FLAG_AUTOTUNE if autotune else 0) | (HSWO_FLAG_INCREMENTAL if incremental else 0) |
               (HSWO_FLAG_KERNEL_TIMES if kernel_times else 0) | (HSWO_FLAG_SEQUENTIAL_SECTIONS if sequential else 0) |
               (HSWO_FLAG_TWO_MERGES if two_merges else 0) | (HSWO_FLAG_DEBUG_VERIFY_BOUND if verify_ptr else 0) |
               (HSWO_FLAG_MULTI_MERGE if multi_merge else 0),
               CRIT[criterion] if isinstance(criterion, str) else int(criterion),
               int(screen_topk), verify_ptr, int(verify_cap),
               ctypes.pointer(tu) if tu is not None else None)
    p._counts_keepalive = arr  # the struct holds raw pointers into arr and tu
    p._tuning_keepalive = tu
    return p


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return HSWO_F32
    if t.dtype == torch.float16:
        return HSWO_F16
    raise TypeError(f"cube dtype must be float32 or float16, got {t.dtype}")


def _check(rc: int):
    if rc != HSWO_OK:
        raise HswoError(rc, last_error())


@dataclasses.dataclass
class Result:
    labels: "object"           # torch int32 [n_levels, H, W] on the device
    log: Optional[np.ndarray]  # MERGE_DTYPE records (host copy) or None
    stats: Optional[dict]
    verify: Optional[np.ndarray] = None  # VERIFY_DTYPE records (verify_cap > 0) or None


def _verify_buffer(params: dict, device):
    """Device buffer for HSWO_FLAG_DEBUG_VERIFY_BOUND records when params asks
    for one (verify_cap > 0); sets the pointer in params."""
    import torch
    cap = int(params.pop("verify_cap", 0))
    if cap <= 0:
        return None, 0
    t = torch.empty((cap * VERIFY_DTYPE.itemsize,), dtype=torch.uint8, device=device)
    params["verify_ptr"] = t.data_ptr()
    params["verify_cap"] = cap
    return t, cap


def _verify_records(t, cap, st, s):
    if t is None:
        return None
    s.synchronize()
    n = min(cap, int(st.verify_records)) if st is not None else cap
    return np.frombuffer(t.cpu().numpy().tobytes(), dtype=VERIFY_DTYPE)[:n].copy()


def workspace_bytes(H, W, B, dtype_code, params: Params) -> int:
    return int(load().hswo_workspace_bytes(H, W, B, dtype_code, ctypes.byref(params)))


def _order_streams(s, device):
    """The call runs on stream s; the inputs and outputs were made (copied,
    allocated) on the current stream, so s first waits for that stream."""
    import torch
    cur = torch.cuda.current_stream(device)
    if s != cur:
        s.wait_stream(cur)


def _keep_alive(s, *tensors):
    """Tell the caching allocator that stream s uses these tensors, so their
    memory is not handed out again before s has finished with them."""
    for t in tensors:
        if t is not None:
            t.record_stream(s)


def _aligned_workspace(nbytes: int, device):
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


def _segment(entry: str, cube, rnb_levels: int, merge_log: bool, stats: bool, stream, params,
             workspace=None, labels_out=None) -> Result:
    import torch
    if not cube.is_cuda:
        raise ValueError("cube must be a device tensor")
    cube = cube.contiguous()
    H, W, B = cube.shape
    code = _dtype_code(cube)
    params = dict(params)
    params["rnb_levels"] = rnb_levels
    vt, vcap = _verify_buffer(params, cube.device)
    if vt is not None and not stats:
        raise ValueError("verify_cap needs stats=True (the record count comes from the stats)")
    p = make_params(**params, merge_log=merge_log)
    lib = load()
    s = stream if stream is not None else torch.cuda.current_stream(cube.device)

    def call(labels_ptr, log_ptr, st_ref, ws_ptr, nb):
        if entry == "hswo_run":
            return lib.hswo_run(cube.data_ptr(), H, W, B, code, ctypes.byref(p), labels_ptr, log_ptr, st_ref,
                                ws_ptr, nb, s.cuda_stream)
        return lib.rhseg_segment(cube.data_ptr(), H, W, B, code, ctypes.byref(p), rnb_levels, labels_ptr,
                                 log_ptr, st_ref, ws_ptr, nb, s.cuda_stream)

    nb = int(lib.hswo_workspace_bytes(H, W, B, code, ctypes.byref(p)))
    if nb == 0:
        _check(call(None, None, None, None, 0))  # the entry point reports why
        raise HswoError(HSWO_E_INVAL, "workspace query failed")
    if workspace is not None:
        # caller-kept workspace (graph replays need the same pointers every call)
        ws, ws_ptr = workspace.get(nb, cube.device)
    else:
        ws, ws_ptr = _aligned_workspace(nb, cube.device)
    labels = labels_out if labels_out is not None else \
        torch.empty((p.n_levels, H, W), dtype=torch.int32, device=cube.device)
    if tuple(labels.shape) != (p.n_levels, H, W) or labels.dtype != torch.int32 or not labels.is_contiguous():
        raise ValueError("labels_out must be a contiguous int32 [n_levels, H, W] device tensor")
    n_merges = H * W - params.get("target_regions", 1)
    log_t = torch.empty((max(n_merges, 1) * MERGE_DTYPE.itemsize,), dtype=torch.uint8, device=cube.device) \
        if merge_log else None
    st = Stats() if stats else None
    _order_streams(s, cube.device)
    _check(call(labels.data_ptr(), log_t.data_ptr() if log_t is not None else None,
                ctypes.byref(st) if st is not None else None, ws_ptr, nb))
    # keep every buffer the call reads or writes alive until its stream has consumed it
    _keep_alive(s, ws, cube, labels, log_t, vt)
    log = None
    if log_t is not None:
        s.synchronize()
        log = np.frombuffer(log_t.cpu().numpy().tobytes(), dtype=MERGE_DTYPE)[:max(n_merges, 0)]
    return Result(labels=labels, log=log, stats=st.as_dict() if st is not None else None,
                  verify=_verify_records(vt, vcap, st, s))


class Workspace:
    """A device scratch buffer kept across calls (grows when needed)."""

    def __init__(self):
        self.buf = None
        self.ptr = 0
        self.nbytes = 0

    def get(self, nbytes, device):
        if self.buf is None or self.nbytes < nbytes:
            self.buf, self.ptr = _aligned_workspace(nbytes, device)
            self.nbytes = nbytes
        return self.buf, self.ptr


def rhseg_segment(cube, *, rnb_levels: int = 1, merge_log: bool = False, stats: bool = False, stream=None,
                  workspace: Optional[Workspace] = None, labels_out=None, **params) -> Result:
    """RHSEG of a device cube H x W x B (C entry point rhseg_segment)."""
    return _segment("rhseg_segment", cube, rnb_levels, merge_log, stats, stream, params, workspace, labels_out)


def rhseg_segment_noalloc(cube, labels_out, *, rnb_levels: int = 1, merge_log_out=None, stats: bool = False,
                          stream=None, **params) -> Result:
    """RHSEG of a device cube H x W x B with the library's static device
    scratch (C entry point rhseg_segment_noalloc): nothing is allocated by this
    call, so the caller passes the outputs -- labels_out, a contiguous int32
    [n_levels, H, W] device tensor, and optionally merge_log_out, a uint8
    device tensor of at least (H*W - target) * 24 bytes. Returns the labels
    tensor, the merge records (a host copy, after a stream sync) when
    merge_log_out is given, and the stats when asked for."""
    import torch
    if not cube.is_cuda or not cube.is_contiguous():
        raise ValueError("cube must be a contiguous device tensor (this entry point makes no copy)")
    H, W, B = cube.shape
    code = _dtype_code(cube)
    params = dict(params)
    params["rnb_levels"] = rnb_levels
    p = make_params(**params, merge_log=merge_log_out is not None)
    if tuple(labels_out.shape) != (p.n_levels, H, W) or labels_out.dtype != torch.int32 or \
            not labels_out.is_contiguous():
        raise ValueError("labels_out must be a contiguous int32 [n_levels, H, W] device tensor")
    n_merges = H * W - params.get("target_regions", 1)
    if merge_log_out is not None and merge_log_out.numel() * merge_log_out.element_size() < \
            max(n_merges, 0) * MERGE_DTYPE.itemsize:
        raise ValueError("merge_log_out is too small")
    s = stream if stream is not None else torch.cuda.current_stream(cube.device)
    st = Stats() if stats else None
    _order_streams(s, cube.device)
    _check(load().rhseg_segment_noalloc(cube.data_ptr(), H, W, B, code, ctypes.byref(p), rnb_levels,
                                        labels_out.data_ptr(),
                                        merge_log_out.data_ptr() if merge_log_out is not None else None,
                                        ctypes.byref(st) if st is not None else None, s.cuda_stream))
    _keep_alive(s, cube, labels_out, merge_log_out)
    log = None
    if merge_log_out is not None:
        s.synchronize()
        log = np.frombuffer(merge_log_out.cpu().numpy().tobytes(), dtype=MERGE_DTYPE)[:max(n_merges, 0)]
    return Result(labels=labels_out, log=log, stats=st.as_dict() if st is not None else None)


def hswo_run(cube, *, merge_log: bool = False, stats: bool = False, stream=None,
             workspace: Optional[Workspace] = None, **params) -> Result:
    """HSEG on the whole image as one section (C entry point hswo_run)."""
    params.pop("rnb_levels", None)
    return _segment("hswo_run", cube, 1, merge_log, stats, stream, params, workspace)


@dataclasses.dataclass
class BatchResult:
    labels: list               # per section: torch int32 [n_levels, H, W]
    logs: Optional[list]       # per section: MERGE_DTYPE records, or None
    stats: Optional[dict]


def hswo_run_batch(cubes, *, merge_log: bool = False, stats: bool = False, stream=None,
                   workspace: Optional[Workspace] = None, labels_out: Optional[list] = None,
                   **params) -> BatchResult:
    """Independent sections (device cubes H_s x W_s x B_s of one dtype), each
    segmented as its own top pass, all in one persistent launch."""
    import torch
    if len(cubes) == 0:
        raise ValueError("no sections")
    cubes = [c.contiguous() for c in cubes]
    code = _dtype_code(cubes[0])
    for c in cubes:
        if not c.is_cuda or _dtype_code(c) != code:
            raise ValueError("all sections must be device tensors of one dtype")
    params = dict(params)
    params["rnb_levels"] = 1
    p = make_params(**params, merge_log=merge_log)
    dev = cubes[0].device
    n = len(cubes)
    target = params.get("target_regions", 1)
    labs = labels_out if labels_out is not None else \
        [torch.empty((p.n_levels, c.shape[0], c.shape[1]), dtype=torch.int32, device=dev) for c in cubes]
    logs_t = [torch.empty((max(c.shape[0] * c.shape[1] - target, 1) * MERGE_DTYPE.itemsize,), dtype=torch.uint8,
                          device=dev) for c in cubes] if merge_log else None
    secs = (Section * n)()
    for i, c in enumerate(cubes):
        H, W, B = c.shape
        secs[i] = Section(c.data_ptr(), H, W, B, labs[i].data_ptr(), logs_t[i].data_ptr() if logs_t else None)
    lib = load()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    nb = int(lib.hswo_batch_workspace_bytes(n, secs, code, ctypes.byref(p)))
    if nb == 0:
        _check(lib.hswo_run_batch(n, secs, code, ctypes.byref(p), None, None, 0, s.cuda_stream))
        raise HswoError(HSWO_E_INVAL, "workspace query failed")
    if workspace is not None:
        ws, ws_ptr = workspace.get(nb, dev)
    else:
        ws, ws_ptr = _aligned_workspace(nb, dev)
    st = Stats() if stats else None
    _order_streams(s, dev)
    _check(lib.hswo_run_batch(n, secs, code, ctypes.byref(p), ctypes.byref(st) if st is not None else None, ws_ptr,
                              nb, s.cuda_stream))
    _keep_alive(s, ws, *cubes, *labs, *(logs_t or []))
    logs = None
    if logs_t is not None:
        s.synchronize()
        logs = []
        for c, t in zip(cubes, logs_t):
            m = c.shape[0] * c.shape[1] - target
            logs.append(np.frombuffer(t.cpu().numpy().tobytes(), dtype=MERGE_DTYPE)[:max(m, 0)])
    return BatchResult(labels=labs, logs=logs, stats=st.as_dict() if st is not None else None)
