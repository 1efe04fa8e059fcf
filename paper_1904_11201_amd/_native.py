"""ctypes view of libjoin.so (include/join.h).  Argument marshalling only.

The shared library is required: importing the package on a machine where it was not built raises
ImportError instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# JOIN_LIBRARY selects another build of the same library: a file name next to this file (the
# checking build libjoin_debug.so) or an absolute path (a sanitizer build of the host code); the
# default is libjoin.so next to this file.
_LIB = os.environ.get("JOIN_LIBRARY") or "libjoin.so"
LIB_PATH = _LIB if os.path.isabs(_LIB) else os.path.join(HERE, os.path.basename(_LIB))

JOIN_OK = 0
JOIN_E_INVAL = 1
JOIN_E_CAPACITY = 2
JOIN_E_WORKSPACE = 3
JOIN_E_HIP = 4
JOIN_E_UNSUPPORTED = 5
STATUS_NAMES = {0: "JOIN_OK", 1: "JOIN_E_INVAL", 2: "JOIN_E_CAPACITY", 3: "JOIN_E_WORKSPACE",
                4: "JOIN_E_HIP", 5: "JOIN_E_UNSUPPORTED"}

JOIN_KIND_HASH = 1
JOIN_KIND_THETA = 2
JOIN_KIND_THETA_REGION = 3
JOIN_KIND_HASH_PREFILTER = 4

OPS = {"none": 0, "eq": 1, "ne": 2, "lt": 3, "le": 4, "gt": 5, "ge": 6, "band": 7}

# Every symbol include/*.h declares.
EXPORTS = ("join_workspace_bytes", "join_count", "join_materialize", "join_hash", "join_theta",
           "join_hash_noalloc",
           "join_build_bytes", "join_build", "join_probe_workspace_bytes", "join_probe_count",
           "join_probe_materialize",
           "join_batch_workspace_bytes", "join_batch_prepare", "join_batch_count",
           "join_batch_materialize", "join_last_error", "join_scan_workspace_bytes",
           "join_scan_u64", "join_prof_enable", "join_prof_collect", "join_prof_count",
           "join_prof_entry", "join_prof_copy", "join_prof_stream", "join_prof_valu",
           "join_prof_wall_clock_khz",
           "join_tune_set", "join_tune_set_local", "join_tune_get")


class JoinRel(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("key2", ctypes.c_void_p), ("rid", ctypes.c_void_p),
                ("n", ctypes.c_int64)]


class JoinPred(ctypes.Structure):
    _fields_ = [("op_a", ctypes.c_int32), ("w", ctypes.c_int32), ("op_c", ctypes.c_int32)]


class JoinJob(ctypes.Structure):
    _fields_ = [("R", JoinRel), ("S", JoinRel), ("bits", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class JoinBuild(ctypes.Structure):
    _fields_ = [("opaque", ctypes.c_uint64 * 16)]


class JoinBatchPlan(ctypes.Structure):
    _fields_ = [("opaque", ctypes.c_uint64 * 64)]


def _hip_runtimes():
    """Distinct HIP runtime files mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({line.split()[-1] for line in f if "libamdhip64" in line})
    except OSError:
        return []


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1904_11201_amd.build` "
            "(hipcc, gfx950).  There is no fallback path.")
    # PyTorch ships its own HIP runtime with the same soname as the system one.  Loading torch
    # first makes libjoin bind to that same runtime, so device pointers and stream handles
    # from torch are valid inside libjoin.  Loading libjoin first would map a second runtime.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise ImportError(f"two HIP runtimes are mapped into this process ({rts}); libjoin and "
                          "torch must share one: import torch before loading libjoin")
    R = ctypes.POINTER(JoinRel)
    Pp = ctypes.POINTER(JoinPred)
    vp, sz, i64, u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_uint64
    lib.join_workspace_bytes.restype = sz
    lib.join_workspace_bytes.argtypes = [ctypes.c_int, i64, i64, Pp]
    lib.join_count.restype = ctypes.c_int
    lib.join_count.argtypes = [ctypes.c_int, R, R, Pp, vp, sz, vp, ctypes.POINTER(u64)]
    lib.join_materialize.restype = ctypes.c_int
    lib.join_materialize.argtypes = [ctypes.c_int, R, R, Pp, vp, sz, vp, u64, vp]
    lib.join_hash.restype = ctypes.c_int
    lib.join_hash.argtypes = [R, R, vp, sz, vp, u64, ctypes.POINTER(u64), vp]
    lib.join_theta.restype = ctypes.c_int
    lib.join_theta.argtypes = [R, R, Pp, vp, sz, vp, u64, ctypes.POINTER(u64), vp]
    Bd = ctypes.POINTER(JoinBuild)
    lib.join_build_bytes.restype = sz
    lib.join_build_bytes.argtypes = [i64]
    lib.join_build.restype = ctypes.c_int
    lib.join_build.argtypes = [R, vp, sz, Bd, vp]
    lib.join_probe_workspace_bytes.restype = sz
    lib.join_probe_workspace_bytes.argtypes = [Bd, i64]
    lib.join_probe_count.restype = ctypes.c_int
    lib.join_probe_count.argtypes = [Bd, vp, R, vp, sz, vp, ctypes.POINTER(u64)]
    lib.join_probe_materialize.restype = ctypes.c_int
    lib.join_probe_materialize.argtypes = [Bd, vp, R, vp, sz, vp, u64, vp]
    Jp = ctypes.POINTER(JoinJob)
    Bp = ctypes.POINTER(JoinBatchPlan)
    lib.join_batch_workspace_bytes.restype = sz
    lib.join_batch_workspace_bytes.argtypes = [ctypes.c_int, Jp]
    lib.join_batch_prepare.restype = ctypes.c_int
    lib.join_batch_prepare.argtypes = [ctypes.c_int, Jp, vp, sz, Bp, vp]
    lib.join_batch_count.restype = ctypes.c_int
    lib.join_batch_count.argtypes = [Bp, vp, sz, vp, vp]
    lib.join_batch_materialize.restype = ctypes.c_int
    lib.join_batch_materialize.argtypes = [Bp, vp, sz, vp, u64, vp]
    lib.join_hash_noalloc.restype = ctypes.c_int
    lib.join_hash_noalloc.argtypes = [ctypes.POINTER(JoinRel), ctypes.POINTER(JoinRel), vp, u64, vp, vp]
    lib.join_tune_set.restype = ctypes.c_int
    lib.join_tune_set.argtypes = [ctypes.c_char_p, i64, ctypes.c_int]
    lib.join_tune_set_local.restype = ctypes.c_int
    lib.join_tune_set_local.argtypes = [ctypes.c_char_p, i64, ctypes.c_int]
    lib.join_tune_get.restype = ctypes.c_int
    lib.join_tune_get.argtypes = [ctypes.c_char_p, i64, ctypes.POINTER(i64)]
    lib.join_last_error.restype = ctypes.c_char_p
    lib.join_last_error.argtypes = []
    lib.join_scan_workspace_bytes.restype = sz
    lib.join_scan_workspace_bytes.argtypes = [i64]
    lib.join_scan_u64.restype = ctypes.c_int
    lib.join_scan_u64.argtypes = [vp, vp, i64, vp, vp, sz, vp]
    lib.join_prof_enable.restype = ctypes.c_int
    lib.join_prof_enable.argtypes = [ctypes.c_int]
    lib.join_prof_collect.restype = ctypes.c_int
    lib.join_prof_collect.argtypes = []
    lib.join_prof_count.restype = ctypes.c_int
    lib.join_prof_count.argtypes = []
    lib.join_prof_entry.restype = ctypes.c_int
    lib.join_prof_entry.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                    ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double)]
    lib.join_prof_copy.restype = ctypes.c_int
    lib.join_prof_copy.argtypes = [vp, vp, u64, vp]
    lib.join_prof_stream.restype = ctypes.c_int
    lib.join_prof_stream.argtypes = [ctypes.c_int, vp, vp, u64, vp]
    lib.join_prof_valu.restype = ctypes.c_int
    lib.join_prof_valu.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, vp, vp, vp]
    lib.join_prof_wall_clock_khz.restype = ctypes.c_int
    lib.join_prof_wall_clock_khz.argtypes = [ctypes.POINTER(ctypes.c_int)]
    return lib


lib = _load()


def last_error() -> str:
    return (lib.join_last_error() or b"").decode(errors="replace")


def prof_enable(on: bool) -> None:
    lib.join_prof_enable(1 if on else 0)


def prof_read() -> dict:
    """{kernel name: (launches, total_ms)} of the launches recorded since prof_enable(True)."""
    if lib.join_prof_collect() != JOIN_OK:
        raise RuntimeError(last_error())
    out = {}
    for i in range(lib.join_prof_count()):
        name = ctypes.c_char_p()
        cnt = ctypes.c_uint64()
        ms = ctypes.c_double()
        if lib.join_prof_entry(i, ctypes.byref(name), ctypes.byref(cnt), ctypes.byref(ms)) == 0:
            out[name.value.decode()] = (int(cnt.value), float(ms.value))
    return out


def tune_set(name: str, value: int | None, local: bool = False) -> None:
    """Set tuning knob `name` (see include/join_tune.h); None restores environment/default.
    local=True sets it for the calling thread only (join_tune_set_local)."""
    fn = lib.join_tune_set_local if local else lib.join_tune_set
    rc = fn(name.encode(), 0 if value is None else int(value), 1 if value is None else 0)
    if rc != 0:
        raise KeyError(name)


def tune_get(name: str, default: int) -> int:
    v = ctypes.c_int64(0)
    if lib.join_tune_get(name.encode(), int(default), ctypes.byref(v)) != 0:
        raise KeyError(name)
    return int(v.value)
