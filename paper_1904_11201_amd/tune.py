"""Autotuner: measures how to cut the work for a range of sizes and caches the fastest choice.

The paper picks its cut of the work, the reducer count alpha, by measurement (Sections 5.1.4 and
5.2.4: time against alpha, best at an intermediate value).  Here the cut is the hash join's
partition fan-out (per build size; used for every join of a batch) and the theta join's S tile
(per relation size).  Only speed depends on these choices; every candidate gives the same result.

    python -m paper_1904_11201_amd.tune [--quick] [--out PATH] [--only hash|theta]

writes a JSON cache (default: tune_cache.json next to this file) that Batch / hash_join_batch and
theta_join(tuned=True) read through `load()`.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")

_loaded: dict | None = None


def load(path: str = CACHE) -> dict:
    """The cached choices ({} when nothing was tuned on this machine yet)."""
    global _loaded
    if _loaded is None or path != CACHE:
        try:
            with open(path) as f:
                c = json.load(f)
        except (OSError, ValueError):
            c = {}
        if path != CACHE:
            return c
        _loaded = c
    return _loaded


def _bucket(n: int) -> int:
    return max(0, int(math.floor(math.log2(max(n, 1)))))


def _nearest(table: dict, n: int):
    """Entry of the largest tuned bucket <= log2(n), else the smallest bucket's."""
    if not table:
        return None
    keys = sorted(int(k) for k in table)
    b = _bucket(n)
    below = [k for k in keys if k <= b]
    return table[str(below[-1] if below else keys[0])]


HASH_CAP = 4608     # entries of one LDS table of a batched join (the library's batch capacity)
HASH_MAX_BITS = 11  # the library's largest fan-out


def hash_min_bits(nR: int, cap: int = HASH_CAP) -> int:
    """Fewest bits whose mean partition holds at most 0.9 * cap build rows (the library's
    default rule): with fewer, partitions split into several R chunks and each of them probes
    the partition's S slice again."""
    if nR <= 0.9 * cap:
        return 0
    return min(HASH_MAX_BITS, int(math.ceil(math.log2(nR / (0.9 * cap)))))


def hash_bits_for(nR: int, cache: dict | None = None, cap: int = HASH_CAP) -> int:
    """Tuned fan-out (log2) for a build side of nR rows of a batched join, or -1 (library
    default).  The table is
    tuned at powers of two and looked up by the largest bucket <= log2(nR); a size up to twice its
    bucket's would overflow the partitions at the bucket's fan-out, so the result is at least
    hash_min_bits(nR)."""
    c = load() if cache is None else cache
    v = _nearest(c.get("hash_bits", {}), nR)
    return -1 if v is None else max(int(v), hash_min_bits(nR, cap))


def hash_bits_for_sizes(nR, cache: dict | None = None, cap: int = HASH_CAP):
    """hash_bits_for over an array of build sizes (numpy int array, -1 where nothing is tuned),
    by one lookup table over the log2 buckets instead of a call per size."""
    import numpy as np
    n = np.maximum(np.asarray(nR, dtype=np.int64), 1)
    b = np.floor(np.log2(n)).astype(np.int64)
    table = np.array([hash_bits_for(1 << k, cache, cap) for k in range(64)], dtype=np.int32)
    tuned = table[np.clip(b, 0, 63)]
    lo = np.where(n <= 0.9 * cap, 0,
                  np.minimum(HASH_MAX_BITS, np.ceil(np.log2(n / (0.9 * cap))))).astype(np.int32)
    return np.where(tuned < 0, tuned, np.maximum(tuned, lo)).astype(np.int32)


def theta_ts_for(nR: int, nS: int, cache: dict | None = None) -> int:
    """Tuned S rows per theta tile for an nR x nS join, or 0 (library default)."""
    c = load() if cache is None else cache
    v = _nearest(c.get("theta_ts", {}), max(nR, nS))
    return 0 if v is None else min(int(v), max(nS, 1))


def apply_bits(jobs, cache: dict | None = None):
    """Set bits = tuned fan-out on every job that leaves the choice to the library."""
    for j in jobs:
        if j.bits < 0:
            j.bits = hash_bits_for(j.R.n, cache)
    return jobs


# ---- measurement ------------------------------------------------------------------------------

def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def tune_hash(buckets, reps: int = 3, log=print) -> dict:
    """Per build-size bucket 2^b: a batch of equal-size joins (|S| = 4|R|, keys uniform over
    |R|), timed count + write for the fan-outs around the table-capacity rule."""
    import torch
    from . import _native
    from .join import Batch, Job, Relation
    cap = min(_native.tune_get("hash.cap", 9216), HASH_CAP)  # the batch kernels' table
    out = {}
    g = torch.Generator(device="cuda")
    for b in buckets:
        nR = 1 << b
        nS = 4 * nR
        count = max(1, min(64, (1 << 24) // (nR + nS)))
        g.manual_seed(1000 + b)
        jobs = []
        for _ in range(count):
            rk = torch.randint(0, nR, (nR,), device="cuda", dtype=torch.int32, generator=g)
            sk = torch.randint(0, nR, (nS,), device="cuda", dtype=torch.int32, generator=g)
            jobs.append((Relation(rk), Relation(sk)))
        lo = max(0, math.ceil(math.log2(max(1.0, nR / (0.95 * cap)))))
        cands = sorted({min(11, x) for x in range(lo, lo + 4)})
        best = None
        for bits in cands:
            batch = Batch([Job(R, S, bits) for R, S in jobs])
            def run():
                offs = batch.count()
                total = int(offs[-1].item())
                o = torch.empty((total, 2), dtype=torch.int32, device="cuda")
                batch.materialize(o)
            ms = _time(run, reps)
            log(f"hash bucket 2^{b} x{count}: bits={bits} {ms:.3f} ms")
            if best is None or ms < best[1]:
                best = (bits, ms)
            del batch
        out[str(b)] = best[0]
        del jobs
        torch.cuda.empty_cache()
    return out


def tune_theta(buckets, reps: int = 3, log=print) -> dict:
    """Per relation-size bucket 2^b (R = S = 2^b rows, band w = 8 and R.c < S.c on uniform
    [0, 2^24) columns, the band workload's shape), timed count pass for several S tile sizes."""
    import torch
    from . import _native
    from .join import JOIN_KIND_THETA, Pred, Relation, join_count, workspace
    out = {}
    g = torch.Generator(device="cuda")
    pred = Pred("band", 8, "lt")
    for b in buckets:
        n = 1 << b
        g.manual_seed(2000 + b)
        cols = [torch.randint(0, 1 << 24, (n,), device="cuda", dtype=torch.int32, generator=g)
                for _ in range(4)]
        R, S = Relation(cols[0], cols[1]), Relation(cols[2], cols[3])
        cands = [0] + [ts for ts in (512, 1024, 2048, 4096, 8192, 16384, 65536) if ts <= n]
        best = None
        for ts in cands:
            _native.tune_set("theta.ts", ts if ts > 0 else None)
            try:
                ws = workspace(JOIN_KIND_THETA, n, n, pred)
                ms = _time(lambda: join_count(JOIN_KIND_THETA, R, S, pred, ws), reps)
            finally:
                _native.tune_set("theta.ts", None)
            log(f"theta bucket 2^{b}: ts={ts or 'auto'} {ms:.3f} ms")
            if best is None or ms < best[1]:
                best = (ts, ms)
        if best[0] > 0:
            out[str(b)] = best[0]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="fewer buckets and repetitions")
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--only", choices=("hash", "theta"),
                    help="measure one table and keep the other from the existing cache")
    args = ap.parse_args(argv)
    import torch
    reps = 2 if args.quick else 3
    hb = [10, 14, 18, 22] if args.quick else [10, 12, 14, 16, 18, 20, 22]
    tb = [12, 16] if args.quick else [12, 14, 16, 18]
    t0 = time.time()
    log = lambda m: print(m, flush=True)  # noqa: E731
    old = load(args.out) if args.only else {}
    cache = {
        "device": torch.cuda.get_device_name(0),
        "hash_bits": tune_hash(hb, reps, log) if args.only != "theta" else old.get("hash_bits", {}),
        "theta_ts": tune_theta(tb, reps, log) if args.only != "hash" else old.get("theta_ts", {}),
    }
    with open(args.out, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    log(f"wrote {args.out} in {time.time() - t0:.1f}s")
    return 0


if __name__ == "__main__":
    sys.exit(main())
