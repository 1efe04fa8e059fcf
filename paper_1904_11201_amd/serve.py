"""Serving loop: continuous batching of join requests on one GPU.

Requests (equi joins, band theta joins) arrive over time.  A fixed number of slots, each a HIP
stream served by one host thread, take the next arrived request as soon as they are free, so the
work of several requests overlaps on the device.  Memory is admitted against an HBM budget in
two steps: a request's workspace before its count pass, and its exact output size (from the
count pass, Section 3.3.3 done exactly) before its write pass; a request whose output does not
fit yet waits, holding only its workspace, until other requests release memory.  Equi joins
whose build relation is one of the resident builds probe its partitioned form (join_probe_*)
instead of partitioning it again; band joins use region pruning (Section 4.2).

The library calls release the GIL (ctypes), so a slot thread blocked in a count pass's 8-byte
read does not stop the others.  Results are device tensors handed back per request; the budget
covers the memory of requests in flight (workspaces and outputs until completion).
"""
from __future__ import annotations

import dataclasses
import statistics
import threading
import time

import torch

from . import join as J

M = 1 << 20


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                    # "hash" or "theta"
    S: J.Relation
    R: J.Relation | None = None  # None: probe resident build `build_id`
    build_id: int = -1
    w: int = 8                   # band half-width (theta)
    arrival_s: float = 0.0       # offset from the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    pairs: torch.Tensor
    count: int
    t_arrival: float
    t_start: float
    t_done: float
    slot: int

    @property
    def latency_ms(self) -> float:
        return (self.t_done - self.t_arrival) * 1e3


class BudgetError(RuntimeError):
    pass


class _Retry(Exception):
    """Raised inside a slot whose request must give its workspace back and start over."""


class Engine:
    """slots: concurrent requests (one stream each); budget_bytes: HBM for requests in flight;
    resident: keep the large builds partitioned (False: every equi join partitions its build)."""

    def __init__(self, builds: list[J.Relation], slots: int = 4, budget_bytes: int = 64 << 30,
                 device="cuda", resident: bool = True):
        self.device = torch.device(device)
        self.slots = slots
        self.budget = int(budget_bytes)
        self.reserved = 0
        self.peak = 0
        self.waits = 0
        self.retries = 0
        self.max_request = 0  # largest workspace + output of one request served so far
        self.active = 0
        self._waiting: set = set()
        self._cv = threading.Condition()
        # Builds large enough to be partitioned are kept partitioned; small ones are joined
        # directly (the library reads a small build without partitioning it at all).
        single_max = J._native.tune_get("hash.single_max_chunks", 16) * J._native.tune_get("hash.cap", 9216)
        self.builds = builds
        self.resident = [J.ResidentBuild(R) if resident and R.n > single_max else None for R in builds]
        torch.cuda.synchronize()
        self.resident_bytes = sum(r.buf.numel() for r in self.resident if r is not None)

    # ---- memory admission ---------------------------------------------------------------
    # A request first reserves its workspace (it becomes active), then, after its count pass,
    # its exact output.  If every active request is waiting for output memory, none would ever
    # release any: the youngest of them then gives its workspace back and starts over later.
    def _reserve_ws(self, nbytes: int):
        if nbytes > self.budget:
            raise BudgetError(f"workspace of {nbytes} bytes exceeds the budget of {self.budget}")
        with self._cv:
            waited = False
            while self.reserved + nbytes > self.budget:
                waited = True
                self._cv.wait()
            self.waits += waited
            self.reserved += nbytes
            self.active += 1
            self.peak = max(self.peak, self.reserved)

    def _release_ws(self, nbytes: int):
        with self._cv:
            self.reserved -= nbytes
            self.active -= 1
            self._cv.notify_all()

    def _reserve_out(self, nbytes: int, key: float, ws_bytes: int):
        with self._cv:
            if ws_bytes + nbytes > self.budget:
                raise BudgetError(f"workspace + output of {ws_bytes + nbytes} bytes exceed the "
                                  f"budget of {self.budget}")
            self._waiting.add(key)
            try:
                while self.reserved + nbytes > self.budget:
                    if len(self._waiting) == self.active and key == max(self._waiting):
                        self.retries += 1
                        raise _Retry()
                    self._cv.wait(timeout=0.05)
                self.reserved += nbytes
                self.peak = max(self.peak, self.reserved)
            finally:
                self._waiting.discard(key)
                self._cv.notify_all()

    def _release_out(self, nbytes: int):
        with self._cv:
            self.reserved -= nbytes
            self._cv.notify_all()

    # ---- one request on one stream ----------------------------------------------------------
    def _run(self, req: Request, stream) -> tuple[torch.Tensor, int]:
        dev = self.device
        key = (req.arrival_s, req.rid)
        rb = None
        if req.kind == "hash" and req.R is None:
            rb = self.resident[req.build_id]
            R = self.builds[req.build_id]
        else:
            R = req.R
        if req.kind == "hash":
            kind, pred = J.JOIN_KIND_HASH, None
        else:
            kind, pred = J.JOIN_KIND_THETA_REGION, J.Pred("band", req.w, "none")
        wsb = rb.workspace_bytes(req.S.n) if rb is not None else J.join_workspace_bytes(kind, R.n, req.S.n, pred)
        self._reserve_ws(wsb)
        try:
            ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
            n = rb.count(req.S, ws, stream) if rb is not None else J.join_count(kind, R, req.S, pred, ws, stream)
            with self._cv:
                self.max_request = max(self.max_request, wsb + 8 * n)
            self._reserve_out(8 * n, key, wsb)
            try:
                out = torch.empty((n, 2), dtype=torch.int32, device=dev)
                if rb is not None:
                    rb.materialize(req.S, ws, out, stream)
                else:
                    J.join_materialize(kind, R, req.S, pred, ws, out, stream)
                stream.synchronize()
            finally:
                self._release_out(8 * n)
        finally:
            self._release_ws(wsb)
        return out, n

    # ---- the loop -------------------------------------------------------------------------
    def serve(self, requests: list[Request], open_loop: bool = True, keep_pairs: bool = True):
        """Serve `requests` in arrival order.  open_loop: each request becomes available at its
        arrival time; otherwise all are available at once (closed loop, capacity).  Returns
        (results in request order, wall seconds)."""
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival_s)
        results: list[Result | None] = [None] * len(requests)
        nxt = [0]
        lock = threading.Lock()
        errors = []
        t0 = time.perf_counter()

        def worker(slot: int):
            stream = torch.cuda.Stream(device=self.device)
            try:
                with torch.cuda.stream(stream):
                    while True:
                        with lock:
                            if nxt[0] >= len(order) or errors:
                                return
                            i = order[nxt[0]]
                            nxt[0] += 1
                        req = requests[i]
                        t_arr = t0 + (req.arrival_s if open_loop else 0.0)
                        delay = t_arr - time.perf_counter()
                        if delay > 0:
                            time.sleep(delay)
                        t_start = time.perf_counter()
                        while True:
                            try:
                                out, n = self._run(req, stream)
                                break
                            except _Retry:
                                with self._cv:  # wait for another request to free memory
                                    self._cv.wait(timeout=0.05)
                        t_done = time.perf_counter()
                        results[i] = Result(req.rid, out if keep_pairs else out[:0], n, t_arr,
                                            t_start, t_done, slot)
                        del out
            except BaseException as e:  # surfaced to the caller after the threads join
                errors.append(e)
                with self._cv:
                    self._cv.notify_all()

        threads = [threading.Thread(target=worker, args=(s,), daemon=True) for s in range(self.slots)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        wall = time.perf_counter() - t0
        if errors:
            raise errors[0]
        return results, wall


def summary(results: list[Result], wall_s: float) -> dict:
    lat = sorted(r.latency_ms for r in results)

    def pct(q):
        return lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]

    pairs = sum(r.count for r in results)
    return {"requests": len(results), "wall_s": round(wall_s, 3),
            "requests_per_s": round(len(results) / wall_s, 2),
            "pairs": pairs, "pairs_per_s": round(pairs / wall_s, 1),
            "p50_ms": round(pct(0.5), 3), "p99_ms": round(pct(0.99), 3),
            "mean_ms": round(statistics.mean(lat), 3)}


def requests_device(seed: int = 7, count: int = 256, lo: int = 1024, hi: int = 8 * M,
                    theta_frac: float = 0.2, reuse_frac: float = 0.3, n_resident: int = 16,
                    qps: float = 1.0, device="cuda"):
    """The serving workload generated in device memory: request kinds, sizes, build reuse and
    Poisson gaps from PCG64(seed) (the recipe of datagen.serve_requests), key columns from a
    seeded torch generator on the device.  Returns (resident builds, requests)."""
    from . import datagen
    g = datagen.rng_for(seed)
    tg = torch.Generator(device=device)
    tg.manual_seed(seed)

    def col(n, hi_):
        return torch.randint(0, max(hi_, 1), (n,), device=device, dtype=torch.int32, generator=tg)

    rsizes = datagen.log_uniform_sizes(datagen.rng_for(seed * 1000 + 1), n_resident, lo, hi)
    builds = [J.Relation(col(int(n), int(n))) for n in rsizes]
    gaps = g.exponential(1.0 / qps, size=count)
    t = gaps.cumsum() - gaps[0]
    reuse_given_hash = min(1.0, reuse_frac / max(1e-9, 1.0 - theta_frac))
    reqs = []
    for i in range(count):
        if g.random() < theta_frac:
            nr, ns = (int(x) for x in datagen.log_uniform_sizes(g, 2, lo, hi))
            R = J.Relation(col(nr, 1 << 24), col(nr, 1 << 24))
            S = J.Relation(col(ns, 1 << 24), col(ns, 1 << 24))
            reqs.append(Request(i, "theta", S, R, -1, 8, float(t[i])))
        elif g.random() < reuse_given_hash:
            b = int(g.integers(0, n_resident))
            ns = int(datagen.log_uniform_sizes(g, 1, lo, hi)[0])
            reqs.append(Request(i, "hash", J.Relation(col(ns, builds[b].n)), None, b, 8, float(t[i])))
        else:
            nr, ns = (int(x) for x in datagen.log_uniform_sizes(g, 2, lo, hi))
            reqs.append(Request(i, "hash", J.Relation(col(ns, nr)), J.Relation(col(nr, nr)), -1, 8,
                                float(t[i])))
    return builds, reqs


def at_rate(requests: list[Request], qps: float, seed: int = 7) -> list[Request]:
    """The same requests with Poisson arrival times at `qps` (seeded)."""
    from . import datagen
    g = datagen.rng_for(seed + 17)
    gaps = g.exponential(1.0 / qps, size=len(requests))
    t = gaps.cumsum() - gaps[0]
    return [dataclasses.replace(r, arrival_s=float(t[i])) for i, r in enumerate(requests)]
