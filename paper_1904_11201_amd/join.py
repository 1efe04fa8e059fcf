"""Python binding of libjoin: the same calls as include/join.h over torch device tensors.

PyTorch provides device memory and the stream; every step of the join runs in libjoin's HIP
kernels.  Typical use (the exact-size flow of count -> scan -> write):

    R = Relation(key_r)                 # int32 cuda tensors (key2 / rid optional)
    S = Relation(key_s)
    pairs = hash_join(R, S)             # [count, 2] int32: (rid_R, rid_S)

or step by step:

    ws = workspace(JOIN_KIND_HASH, R.n, S.n)
    n = join_count(JOIN_KIND_HASH, R, S, None, ws)
    out = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    join_materialize(JOIN_KIND_HASH, R, S, None, ws, out)
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _native
from ._native import (JOIN_KIND_HASH, JOIN_KIND_HASH_PREFILTER, JOIN_KIND_THETA,
                      JOIN_KIND_THETA_REGION, OPS, JoinBatchPlan, JoinBuild, JoinJob, JoinPred,
                      JoinRel)

__all__ = [
    "JoinError", "Relation", "Pred", "JOIN_KIND_HASH", "JOIN_KIND_THETA", "JOIN_KIND_THETA_REGION",
    "JOIN_KIND_HASH_PREFILTER",
    "join_workspace_bytes",
    "workspace", "join_count", "join_materialize", "join_hash", "join_theta", "join_scan_u64",
    "join_hash_noalloc",
    "hash_join", "theta_join", "Job", "Batch", "hash_join_batch", "ResidentBuild",
]


class JoinError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_native.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(rc: int):
    if rc != _native.JOIN_OK:
        raise JoinError(rc, _native.last_error())


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("join columns must be contiguous int32 cuda tensors")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else None


@dataclasses.dataclass
class Relation:
    """One relation in column layout: key (or theta column a), optional key2 (theta column c)
    and optional rid payload (absent = row position).  Device tensors."""
    key: torch.Tensor
    key2: torch.Tensor | None = None
    rid: torch.Tensor | None = None

    @property
    def n(self) -> int:
        return int(self.key.numel())

    def c(self) -> JoinRel:
        for t in (self.key2, self.rid):
            if t is not None and t.numel() != self.key.numel():
                raise ValueError("all columns of a relation need the same length")
        return JoinRel(_ptr(self.key), _ptr(self.key2), _ptr(self.rid), self.n)


@dataclasses.dataclass
class Pred:
    """Theta predicate op_a(R.key, S.key) [and op_c(R.key2, S.key2)]; op names as in OPS."""
    op_a: str = "eq"
    w: int = 0
    op_c: str = "none"

    def c(self) -> JoinPred:
        return JoinPred(OPS[self.op_a], int(self.w), OPS[self.op_c])


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _pred_ptr(pred):
    return None if pred is None else ctypes.byref(pred.c())


def join_workspace_bytes(kind: int, nR: int, nS: int, pred: Pred | None = None) -> int:
    return int(_native.lib.join_workspace_bytes(kind, nR, nS, _pred_ptr(pred)))


def workspace(kind: int, nR: int, nS: int, pred: Pred | None = None, device="cuda"):
    """A uint8 device tensor large enough for a join of this kind and these sizes."""
    return torch.empty(join_workspace_bytes(kind, nR, nS, pred), dtype=torch.uint8, device=device)


def join_count(kind: int, R: Relation, S: Relation, pred: Pred | None, ws: torch.Tensor,
               stream=None) -> int:
    """Exact number of output pairs (count pass + device scan; one 8-byte host read)."""
    cnt = ctypes.c_uint64(0)
    rr, sr = R.c(), S.c()
    _check(_native.lib.join_count(kind, ctypes.byref(rr), ctypes.byref(sr), _pred_ptr(pred),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                                  ctypes.byref(cnt)))
    return int(cnt.value)


def join_materialize(kind: int, R: Relation, S: Relation, pred: Pred | None, ws: torch.Tensor,
                     pairs: torch.Tensor, stream=None) -> None:
    """Write pass into pairs ([capacity, 2] int32) from the state join_count left in ws."""
    if pairs.dtype != torch.int32 or not pairs.is_contiguous():
        raise ValueError("pairs must be a contiguous int32 tensor")
    rr, sr = R.c(), S.c()
    cap = pairs.numel() // 2
    _check(_native.lib.join_materialize(kind, ctypes.byref(rr), ctypes.byref(sr), _pred_ptr(pred),
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                        ctypes.c_void_p(pairs.data_ptr()) if cap else None, cap,
                                        _stream(stream)))


def join_hash(R: Relation, S: Relation, ws: torch.Tensor, pairs: torch.Tensor | None,
              stream=None) -> int:
    """One-shot equi join with snprintf semantics: returns the exact count; writes only if
    pairs holds at least that many pairs (else raises JoinError with JOIN_E_CAPACITY)."""
    cnt = ctypes.c_uint64(0)
    rr, sr = R.c(), S.c()
    cap = 0 if pairs is None else pairs.numel() // 2
    rc = _native.lib.join_hash(ctypes.byref(rr), ctypes.byref(sr), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel(), ctypes.c_void_p(pairs.data_ptr()) if cap else None, cap,
                               ctypes.byref(cnt), _stream(stream))
    if rc == _native.JOIN_E_CAPACITY:
        err = JoinError(rc, _native.last_error())
        err.count = int(cnt.value)
        raise err
    _check(rc)
    return int(cnt.value)


def join_hash_noalloc(R: Relation, S: Relation, pairs: torch.Tensor | None, count: torch.Tensor,
                      stream=None) -> None:
    """join_hash with the library's static scratch array instead of a workspace: allocates
    nothing and does not synchronise.  count: a one-element int64 device tensor that receives
    the exact count; pairs ([capacity, 2] int32) is written only if the count fits."""
    if count.dtype != torch.int64 or count.numel() < 1 or count.device.type != "cuda":
        raise ValueError("count must be an int64 cuda tensor of at least one element")
    rr, sr = R.c(), S.c()
    cap = 0 if pairs is None else pairs.numel() // 2
    _check(_native.lib.join_hash_noalloc(ctypes.byref(rr), ctypes.byref(sr),
                                         ctypes.c_void_p(pairs.data_ptr()) if cap else None, cap,
                                         ctypes.c_void_p(count.data_ptr()), _stream(stream)))


def join_theta(R: Relation, S: Relation, pred: Pred, ws: torch.Tensor,
               pairs: torch.Tensor | None, stream=None) -> int:
    """One-shot theta join with snprintf semantics (see join_hash)."""
    cnt = ctypes.c_uint64(0)
    rr, sr = R.c(), S.c()
    cap = 0 if pairs is None else pairs.numel() // 2
    rc = _native.lib.join_theta(ctypes.byref(rr), ctypes.byref(sr), ctypes.byref(pred.c()),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                ctypes.c_void_p(pairs.data_ptr()) if cap else None, cap,
                                ctypes.byref(cnt), _stream(stream))
    if rc == _native.JOIN_E_CAPACITY:
        err = JoinError(rc, _native.last_error())
        err.count = int(cnt.value)
        raise err
    _check(rc)
    return int(cnt.value)


def join_scan_u64(x: torch.Tensor, stream=None):
    """Device exclusive prefix sum of a uint64 (int64-typed) cuda tensor: (out, total)."""
    if x.dtype not in (torch.int64, torch.uint64) or not x.is_contiguous():
        raise ValueError("scan input must be a contiguous 64-bit tensor")
    n = x.numel()
    out = torch.empty_like(x)
    total = torch.empty(1, dtype=x.dtype, device=x.device)
    ws = torch.empty(int(_native.lib.join_scan_workspace_bytes(n)), dtype=torch.uint8,
                     device=x.device)
    _check(_native.lib.join_scan_u64(ctypes.c_void_p(x.data_ptr()) if n else None,
                                     ctypes.c_void_p(out.data_ptr()) if n else None, n,
                                     ctypes.c_void_p(total.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    return out, total


def prof_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """Plain device copy src -> dst (same byte size, multiple of 16): the HBM ceiling."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("prof_copy: src and dst sizes differ")
    _check(_native.lib.join_prof_copy(ctypes.c_void_p(src.data_ptr()),
                                      ctypes.c_void_p(dst.data_ptr()), nb, _stream(stream)))


def prof_stream(mode: str, buf: torch.Tensor, sink: torch.Tensor | None = None, stream=None) -> None:
    """One streaming pass over buf: mode 'read' (folds into sink, an int32 tensor of at least
    4 * 1024 * compute units elements) or 'write'.  HBM traffic: buf's byte size."""
    nb = buf.numel() * buf.element_size()
    if mode == "read":
        if sink is None or sink.dtype != torch.int32:
            raise ValueError("prof_stream('read'): sink must be an int32 tensor")
        _check(_native.lib.join_prof_stream(1, ctypes.c_void_p(buf.data_ptr()),
                                            ctypes.c_void_p(sink.data_ptr()), nb, _stream(stream)))
    elif mode == "write":
        _check(_native.lib.join_prof_stream(2, None, ctypes.c_void_p(buf.data_ptr()), nb,
                                            _stream(stream)))
    else:
        raise ValueError("prof_stream: mode is 'read' or 'write'")


def prof_valu(blocks: int, iters: int, sink: torch.Tensor, clk: torch.Tensor, stream=None,
              mix: int = 0) -> int:
    """int32 VALU spin: blocks x 256 lanes x (32, or 48 for mix 2) x iters lane-operations
    (returned); mix 0 add/xor chains, mix 1 a band test's subtract, compare and mask, mix 2 the
    nested-loop join's subtract and three-input min, mix 3 subtracts from a scalar only, mix 4
    three-input minima only.  sink is an int32 tensor of blocks * 256
    elements, clk an int64 tensor of 2 (shader cycles, real-time ticks of workgroup 0)."""
    if sink.dtype != torch.int32 or sink.numel() < blocks * 256:
        raise ValueError("prof_valu: sink must be int32 with blocks * 256 elements")
    if clk.dtype != torch.int64 or clk.numel() < 2:
        raise ValueError("prof_valu: clk must be int64 with 2 elements")
    _check(_native.lib.join_prof_valu(blocks, iters, mix, ctypes.c_void_p(sink.data_ptr()),
                                      ctypes.c_void_p(clk.data_ptr()), _stream(stream)))
    return blocks * 256 * (48 if mix == 2 else 32) * iters


def prof_wall_clock_hz() -> float:
    """Rate of the device's constant real-time counter."""
    khz = ctypes.c_int()
    _check(_native.lib.join_prof_wall_clock_khz(ctypes.byref(khz)))
    return khz.value * 1e3


def _exact(kind, R, S, pred, ws, stream):
    if ws is None:
        ws = workspace(kind, R.n, S.n, pred, device=R.key.device)
    n = join_count(kind, R, S, pred, ws, stream)
    out = torch.empty((n, 2), dtype=torch.int32, device=R.key.device)
    join_materialize(kind, R, S, pred, ws, out, stream)
    return out


def hash_join(R: Relation, S: Relation, ws: torch.Tensor | None = None, stream=None,
              prefilter: bool = False):
    """Equi join R.key = S.key; returns the exact-size [count, 2] int32 tensor of (rid_R, rid_S).
    prefilter=True first drops the tuples whose key cannot occur on the other side
    (JOIN_KIND_HASH_PREFILTER); same result."""
    return _exact(JOIN_KIND_HASH_PREFILTER if prefilter else JOIN_KIND_HASH, R, S, None, ws, stream)


def theta_join(R: Relation, S: Relation, pred: Pred, ws: torch.Tensor | None = None, stream=None,
               region: bool = False, tuned: bool = False):
    """Theta join op_a(R.key, S.key) [and op_c(R.key2, S.key2)]; exact-size [count, 2] output.
    region=True uses the region-pruned algorithm (JOIN_KIND_THETA_REGION); same result.
    tuned=True applies the autotuner's S tile for these sizes (set for the calling thread only,
    for the duration of the call)."""
    kind = JOIN_KIND_THETA_REGION if region else JOIN_KIND_THETA
    if not tuned:
        return _exact(kind, R, S, pred, ws, stream)
    from . import tune
    ts = tune.theta_ts_for(R.n, S.n)
    if ts <= 0:
        return _exact(kind, R, S, pred, ws, stream)
    _native.tune_set("theta.ts", ts, local=True)
    try:
        return _exact(kind, R, S, pred, None, stream)  # the workspace size depends on the tile
    finally:
        _native.tune_set("theta.ts", None, local=True)


# ---- batched equi joins ------------------------------------------------------------------------

@dataclasses.dataclass
class Job:
    """One equi join of a batch: R.key = S.key.  bits < 0 lets the library pick the fan-out."""
    R: Relation
    S: Relation
    bits: int = -1


# join_job_t as a numpy record: R (key, key2, rid, n), S (key, key2, rid, n), bits, reserved
_JOB_DTYPE = np.dtype([("Rk", "<u8"), ("R2", "<u8"), ("Rr", "<u8"), ("Rn", "<i8"),
                       ("Sk", "<u8"), ("S2", "<u8"), ("Sr", "<u8"), ("Sn", "<i8"),
                       ("bits", "<i4"), ("reserved", "<i4")])
assert _JOB_DTYPE.itemsize == ctypes.sizeof(JoinJob)


def _col(t, n: int) -> int:
    """Device address of a join column of n rows (0 for None or an empty column)."""
    if t is None:
        return 0
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("join columns must be contiguous int32 cuda tensors")
    if t.numel() != n:
        raise ValueError("all columns of a relation need the same length")
    return t.data_ptr() if n > 0 else 0


def _jobs_array(jobs) -> np.ndarray:
    """The join_job_t array of a batch, built as one numpy record array."""
    rows = []
    for j in jobs:
        R, S = j.R, j.S
        nr, ns = R.key.numel(), S.key.numel()
        rows.append((_col(R.key, nr), _col(R.key2, nr), _col(R.rid, nr), nr,
                     _col(S.key, ns), _col(S.key2, ns), _col(S.rid, ns), ns, int(j.bits), 0))
    return np.array(rows if rows else [(0,) * 10], dtype=_JOB_DTYPE)


def _packed_array(rkeys: torch.Tensor, roffs, skeys: torch.Tensor, soffs, bits=None,
                  rrids: torch.Tensor | None = None, srids: torch.Tensor | None = None) -> np.ndarray:
    """The join_job_t array of a packed batch: join j's R keys are rkeys[roffs[j]:roffs[j+1]]
    (rids likewise, or row positions within the join when rrids is None), and the same for S."""
    roffs = np.asarray(roffs, dtype=np.int64)
    soffs = np.asarray(soffs, dtype=np.int64)
    n = len(roffs) - 1
    if n < 0 or len(soffs) != n + 1:
        raise ValueError("offsets need njobs + 1 entries on both sides")
    for offs, col in ((roffs, rkeys), (soffs, skeys)):
        if offs[0] != 0 or offs[-1] != col.numel() or np.any(np.diff(offs) < 0):
            raise ValueError("offsets must rise from 0 to the column length")
    base = {}
    for name, t, nn in (("rk", rkeys, int(roffs[-1])), ("rr", rrids, int(roffs[-1])),
                        ("sk", skeys, int(soffs[-1])), ("sr", srids, int(soffs[-1]))):
        base[name] = _col(t, nn)
    arr = np.zeros(max(n, 1), dtype=_JOB_DTYPE)
    if n == 0:
        return arr
    rn, sn = np.diff(roffs), np.diff(soffs)
    a = arr[:n]
    a["Rn"], a["Sn"] = rn, sn
    a["Rk"] = np.where(rn > 0, base["rk"] + 4 * roffs[:-1], 0)
    a["Sk"] = np.where(sn > 0, base["sk"] + 4 * soffs[:-1], 0)
    if base["rr"]:
        a["Rr"] = np.where(rn > 0, base["rr"] + 4 * roffs[:-1], 0)
    if base["sr"]:
        a["Sr"] = np.where(sn > 0, base["sr"] + 4 * soffs[:-1], 0)
    a["bits"] = -1 if bits is None else np.asarray(bits, dtype=np.int32)
    return arr


class Batch:
    """A prepared batch of independent equi joins (join_batch_prepare).  count() and
    materialize() only launch kernels, so they can run inside a captured HIP graph.  The
    relations' tensors must stay alive and unchanged while the batch is in use."""

    def __init__(self, jobs: list[Job], stream=None, device="cuda"):
        self.jobs = list(jobs)
        self._prepare(_jobs_array(self.jobs), len(self.jobs), stream, device)

    @classmethod
    def packed(cls, rkeys: torch.Tensor, roffs, skeys: torch.Tensor, soffs, bits=None,
               rrids: torch.Tensor | None = None, srids: torch.Tensor | None = None,
               stream=None, device="cuda") -> "Batch":
        """A batch whose joins are slices of packed columns: join j's R keys are
        rkeys[roffs[j]:roffs[j+1]] (rids the same slice of rrids, or row positions within the
        join when rrids is None), and likewise for S; bits: one fan-out per join or None (the
        library's default).  The job table is built with vectorised arithmetic, not per join."""
        b = cls.__new__(cls)
        b.jobs = []
        b._cols = (rkeys, skeys, rrids, srids)  # kept alive with the batch
        b._prepare(_packed_array(rkeys, roffs, skeys, soffs, bits, rrids, srids), len(roffs) - 1,
                   stream, device)
        return b

    def _prepare(self, arr: np.ndarray, n: int, stream, device):
        self._arr = arr
        self.njobs = n
        self._c = self._arr.ctypes.data_as(ctypes.POINTER(JoinJob))
        nbytes = int(_native.lib.join_batch_workspace_bytes(n, self._c))
        if nbytes == 0:
            raise JoinError(_native.JOIN_E_INVAL, _native.last_error() or "batch too large")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.plan = JoinBatchPlan()
        self.offsets = torch.zeros(n + 1, dtype=torch.int64, device=device)
        _check(_native.lib.join_batch_prepare(n, self._c, ctypes.c_void_p(self.ws.data_ptr()),
                                              self.ws.numel(), ctypes.byref(self.plan),
                                              _stream(stream)))

    def count(self, stream=None) -> torch.Tensor:
        """Count pass of every join; returns the device offsets tensor ([njobs + 1] int64:
        join j's pairs are [offsets[j], offsets[j+1]), offsets[-1] is the total)."""
        _check(_native.lib.join_batch_count(ctypes.byref(self.plan), ctypes.c_void_p(self.ws.data_ptr()),
                                            self.ws.numel(), ctypes.c_void_p(self.offsets.data_ptr()),
                                            _stream(stream)))
        return self.offsets

    def materialize(self, pairs: torch.Tensor, stream=None) -> None:
        """Write pass of every join into pairs ([capacity, 2] int32)."""
        if pairs.dtype != torch.int32 or not pairs.is_contiguous():
            raise ValueError("pairs must be a contiguous int32 tensor")
        cap = pairs.numel() // 2
        _check(_native.lib.join_batch_materialize(
            ctypes.byref(self.plan), ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
            ctypes.c_void_p(pairs.data_ptr()) if cap else None, cap, _stream(stream)))


def hash_join_batch(jobs: list[Job], stream=None, tuned: bool = False):
    """All joins of the batch: (pairs [total, 2] int32, offsets host list of njobs + 1 ints).
    tuned=True gives every job without a fan-out the autotuner's choice for its build size."""
    if tuned:
        from . import tune
        jobs = tune.apply_bits([Job(j.R, j.S, j.bits) for j in jobs])
    b = Batch(jobs, stream)
    offs = b.count(stream)
    total = int(offs[-1].item())
    out = torch.empty((total, 2), dtype=torch.int32, device=b.ws.device)
    b.materialize(out, stream)
    return out, [int(v) for v in offs.cpu().tolist()]


# ---- resident builds ---------------------------------------------------------------------------

class ResidentBuild:
    """A build relation partitioned once (join_build) and probed by many probe relations.  The
    build buffer is device memory owned by this object; R may be dropped once the build's
    work on `stream` has completed."""

    def __init__(self, R: Relation, stream=None, device="cuda"):
        self.n = R.n
        nbytes = int(_native.lib.join_build_bytes(R.n))
        if nbytes == 0:
            raise JoinError(_native.JOIN_E_INVAL, "build side too large")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.desc = JoinBuild()
        rr = R.c()
        _check(_native.lib.join_build(ctypes.byref(rr), ctypes.c_void_p(self.buf.data_ptr()),
                                      self.buf.numel(), ctypes.byref(self.desc), _stream(stream)))

    def workspace_bytes(self, nS: int) -> int:
        return int(_native.lib.join_probe_workspace_bytes(ctypes.byref(self.desc), nS))

    def workspace(self, nS: int, device="cuda") -> torch.Tensor:
        return torch.empty(self.workspace_bytes(nS), dtype=torch.uint8, device=device)

    def count(self, S: Relation, ws: torch.Tensor, stream=None) -> int:
        cnt = ctypes.c_uint64(0)
        sr = S.c()
        _check(_native.lib.join_probe_count(ctypes.byref(self.desc), ctypes.c_void_p(self.buf.data_ptr()),
                                            ctypes.byref(sr), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                            _stream(stream), ctypes.byref(cnt)))
        return int(cnt.value)

    def materialize(self, S: Relation, ws: torch.Tensor, pairs: torch.Tensor, stream=None) -> None:
        if pairs.dtype != torch.int32 or not pairs.is_contiguous():
            raise ValueError("pairs must be a contiguous int32 tensor")
        cap = pairs.numel() // 2
        sr = S.c()
        _check(_native.lib.join_probe_materialize(
            ctypes.byref(self.desc), ctypes.c_void_p(self.buf.data_ptr()), ctypes.byref(sr),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(),
            ctypes.c_void_p(pairs.data_ptr()) if cap else None, cap, _stream(stream)))

    def probe(self, S: Relation, stream=None) -> torch.Tensor:
        """R ⋈ S with R from this build: the exact-size [count, 2] int32 pairs."""
        ws = self.workspace(S.n, device=self.buf.device)
        n = self.count(S, ws, stream)
        out = torch.empty((n, 2), dtype=torch.int32, device=self.buf.device)
        self.materialize(S, ws, out, stream)
        return out
