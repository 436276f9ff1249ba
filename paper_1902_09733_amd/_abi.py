"""ctypes view of libbpstereo's C ABI (include/bp.h): argument marshalling only."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbpstereo.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bp.h")

BP_OK = 0
BP_ERR_INVALID_ARGUMENT = -1
BP_ERR_UNSUPPORTED = -2
BP_ERR_WORKSPACE_TOO_SMALL = -3
BP_ERR_HIP = -4

BP_MSG_F32, BP_MSG_F16, BP_MSG_BF16 = 0, 1, 2

# Size of bp_run_noalloc's fixed per-GPU scratch array (BP_NOALLOC_SCRATCH_BYTES).
BP_NOALLOC_SCRATCH_BYTES = 640 << 20


class BpPair(ctypes.Structure):
    _fields_ = [
        ("left", ctypes.c_void_p),
        ("right", ctypes.c_void_p),
        ("channels", ctypes.c_int32),
        ("downsample", ctypes.c_int32),
        ("row_stride_bytes", ctypes.c_int64),
        ("data_trunc", ctypes.c_float),
        ("rgb_mode", ctypes.c_int32),
    ]


class BpProblem(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("num_labels", ctypes.c_int32),
        ("cost", ctypes.c_void_p),
        ("disparity", ctypes.c_void_p),
        ("soft_disparity", ctypes.c_void_p),
        ("messages_out", ctypes.c_void_p),
        ("pair", ctypes.POINTER(BpPair)),
    ]


class BpCorner(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int32), ("y", ctypes.c_int32), ("response", ctypes.c_int64)]


class BpMatch(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int32), ("y", ctypes.c_int32), ("cost", ctypes.c_int64)]


class BpIntrinsics(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("fx", "fy", "cx", "cy", "k1", "k2", "k3")]


class BpCamera(ctypes.Structure):
    _fields_ = [
        ("baseline", ctypes.c_float),
        ("focal", ctypes.c_float),
        ("du", ctypes.c_float),
        ("dv", ctypes.c_float),
        ("u0", ctypes.c_float),
        ("v0", ctypes.c_float),
    ]


class BpParams(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("iters_per_level", ctypes.c_int32),
        ("lambda_", ctypes.c_float),
        ("tau", ctypes.c_float),
        ("msg_dtype", ctypes.c_int32),
        ("temperature", ctypes.c_float),
        ("checkpoint_every", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("pm_from", ctypes.c_int32),
    ]


class BpLaunchRecord(ctypes.Structure):
    _fields_ = [
        ("level", ctypes.c_int32),
        ("half_sweep", ctypes.c_int32),
        ("launches", ctypes.c_int32),
        ("readout_fused", ctypes.c_int32),
        ("msg_bytes", ctypes.c_int32),
        ("units", ctypes.c_double),
        ("ms", ctypes.c_float),
        ("bytes", ctypes.c_double),
    ]


class BPError(RuntimeError):
    def __init__(self, fn: str, status: int, text: str):
        super().__init__(f"{fn} failed: {text} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load libbpstereo.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
    P = ctypes.POINTER
    L.bp_status_string.argtypes = [ctypes.c_int]
    L.bp_status_string.restype = ctypes.c_char_p
    L.bp_cost_volume.argtypes = [vp, vp, i32, i32, i32, i64, i32, i32, f32, i32, vp, vp]
    L.bp_cost_volume.restype = ctypes.c_int
    L.bp_downsample.argtypes = [vp, i32, i32, i32, i64, i32, vp, vp]
    L.bp_downsample.restype = ctypes.c_int
    L.bp_workspace_size.argtypes = [P(BpProblem), i32, P(BpParams)]
    L.bp_workspace_size.restype = sz
    L.bp_checkpoint_size.argtypes = [P(BpProblem), i32, P(BpParams)]
    L.bp_checkpoint_size.restype = sz
    L.bp_run.argtypes = [P(BpProblem), i32, P(BpParams), vp, sz, vp, sz, vp]
    L.bp_run.restype = ctypes.c_int
    L.bp_run_noalloc.argtypes = [P(BpProblem), i32, P(BpParams), vp, sz, vp]
    L.bp_run_noalloc.restype = ctypes.c_int
    L.bp_run_profiled.argtypes = [P(BpProblem), i32, P(BpParams), vp, sz, vp, i32, P(BpLaunchRecord), i32, P(i32)]
    L.bp_run_profiled.restype = ctypes.c_int
    L.bp_upsample.argtypes = [vp, i32, i32, vp, i32, i32, i32, i64, f32, f32, i32, vp, vp]
    L.bp_upsample.restype = ctypes.c_int
    L.bp_harris.argtypes = [vp, i32, i32, i64, i32, i64, vp, vp, vp]
    L.bp_harris.restype = ctypes.c_int
    L.bp_zssd_match.argtypes = [vp, vp, i32, i32, i64, vp, i32, i32, i32, vp, vp]
    L.bp_zssd_match.restype = ctypes.c_int
    L.bp_icp_workspace_size.argtypes = [i32, i32]
    L.bp_icp_workspace_size.restype = sz
    L.bp_icp.argtypes = [vp, i32, vp, i32, vp, i32, f32, vp, vp, vp, vp, vp, sz, vp]
    L.bp_icp.restype = ctypes.c_int
    L.bp_undistort.argtypes = [vp, i32, i32, i32, i64, P(BpIntrinsics), vp, i64, vp]
    L.bp_undistort.restype = ctypes.c_int
    L.bp_upsample_points.argtypes = [vp, i32, i32, vp, i32, i32, i32, i64, f32, f32, i32, P(BpCamera), vp, vp, vp]
    L.bp_upsample_points.restype = ctypes.c_int
    L.bp_backward.argtypes = [P(BpProblem), i32, P(BpParams), vp, sz, vp, vp, vp, vp, vp, sz, vp]
    L.bp_backward.restype = ctypes.c_int
    L.bp_backward_workspace_size.argtypes = [P(BpProblem), i32, P(BpParams)]
    L.bp_backward_workspace_size.restype = sz
    L.bp_stream_probe.argtypes = [vp, sz, vp, sz, vp]
    L.bp_stream_probe.restype = ctypes.c_int
    L.bp_load_tune_table.argtypes = [ctypes.c_char_p]
    L.bp_load_tune_table.restype = ctypes.c_int
    L.bp_variant_count.argtypes = [i32]
    L.bp_variant_count.restype = i32
    _lib = L
    return L


def check(fn: str, status: int):
    if status != BP_OK:
        text = lib().bp_status_string(status).decode()
        if status == BP_ERR_INVALID_ARGUMENT:
            raise ValueError(f"{fn}: {text}")
        raise BPError(fn, status, text)


def header_functions():
    """Names of the functions include/bp.h declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bp_[a-z_]+)\s*\(", src)))
