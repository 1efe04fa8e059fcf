#!/usr/bin/env python3
"""Benchmark of the join hot path on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input, every input
already resident in HBM:
  * hash equi join 16M x 64M, S keys uniform over R's keys   (histogram, scan, scatter, plan,
    LDS-table count, scan, exact allocation, write)
  * the same with S keys bounded-Zipf(1.0)
  * band theta join 1M x 1M, |R.a - S.a| <= 8 and R.c < S.c    (count, scan, exact allocation,
    write)
`value` is probe tuples/s of the two hash joins (2 * 2^26 probe tuples over their summed time
inside the timed steps); the theta and latency figures ride along in their own fields.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("probe tuples/s + output pairs/s (16M⋈64M hash join, 1M×1M theta); "
          "p99 latency")
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# int32 VALU peak in lane-ops/s: 256 CUs x 2 wave64 VALU instructions per CU and clock x 64 lanes
# x 2.4 GHz.  Two per clock is the published fp32 vector rate (157.3 TFLOP/s = 128 FMA lanes per
# CU and clock); the SQ_INSTS_VALU counters of the add/xor spin show about 1.7 per CU and clock
# (profiles/valu_theta_1Mx1M.md), so one per clock (39.3 T) is not the ceiling.
VALU_ISSUE_PER_CU_CLK = 2
VALU_PEAK_TOPS = 256 * VALU_ISSUE_PER_CU_CLK * 64 * 2.4e9 / 1e12

M = 1 << 20


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-runs", type=int, default=200)
    ap.add_argument("--batch-jobs", type=int, default=4096,
                    help="joins in the batched-join comparison (0 skips it)")
    ap.add_argument("--serve-requests", type=int, default=1024,
                    help="requests in the serving comparison (0 skips it)")
    return ap.parse_args()


def src_hash(files=None) -> str:
    """Hash of the kernel sources (all of csrc/, or the named files of it)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1904_11201_amd", "csrc")
    for f in sorted(files if files else os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch from committed rocprofv3 --pmc summaries (profiles/traffic.json),
    each group valid only while the sources of its kernels are the ones it was taken on."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return {}
    with open(p) as f:
        t = json.load(f)
    kern = {}
    for grp in t.get("groups", []):
        if grp.get("src_hash") == src_hash(grp.get("files")):
            kern.update(grp.get("kernels", {}))
    return kern


def load_valu():
    """VALU instructions per launch from the committed rocprofv3 --pmc summary
    (profiles/valu.json), each group valid only while its kernel sources are unchanged."""
    p = os.path.join(ROOT, "profiles", "valu.json")
    if not os.path.exists(p):
        return {}
    with open(p) as f:
        t = json.load(f)
    kern = {}
    for grp in t.get("groups", []):
        if grp.get("src_hash") == src_hash(grp.get("files")):
            kern.update(grp.get("kernels", {}))
    return kern


def cpu_model() -> str | None:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def bench_batch(args, J, datagen, dev, stream):
    """Batched equi joins (4096 joins, per-side sizes log-uniform in [1K, 4M], keys uniform over
    the build size, 10% Zipf probe sides): one launch per join vs the batch, eager and with the
    count pass replayed from a captured graph.  Each form: count, one total read, exact
    allocation, write."""
    import numpy as np
    import torch
    from paper_1904_11201_amd import tune
    t0 = time.time()
    raw = datagen.batch_jobs_device(seed=6, jobs=args.batch_jobs, device=dev)
    # packed columns: join j's keys are a slice of one tensor per side
    rk_all = torch.cat([rk for rk, _, _ in raw])
    sk_all = torch.cat([sk for _, sk, _ in raw])
    roffs = np.concatenate([[0], np.cumsum([rk.numel() for rk, _, _ in raw])]).astype(np.int64)
    soffs = np.concatenate([[0], np.cumsum([sk.numel() for _, sk, _ in raw])]).astype(np.int64)
    del raw
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    jobs = [J.Job(J.Relation(rk_all[roffs[j]:roffs[j + 1]]), J.Relation(sk_all[soffs[j]:soffs[j + 1]]))
            for j in range(len(roffs) - 1)]
    rows_r = sum(j.R.n for j in jobs)
    rows_s = sum(j.S.n for j in jobs)
    print(f"# batch: {len(jobs)} joins, {rows_r} x {rows_s} rows generated in {gen_s:.1f}s",
          file=sys.stderr, flush=True)
    reps = 3

    def wall(fn):
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) * 1e3, r

    # one launch sequence per join (count with its 8-byte read, allocation, write)
    ws = J.workspace(J.JOIN_KIND_HASH, max(j.R.n for j in jobs), max(j.S.n for j in jobs))

    def per_join():
        tot = 0
        for j in jobs:
            n = J.join_count(J.JOIN_KIND_HASH, j.R, j.S, None, ws, stream)
            out = torch.empty((n, 2), dtype=torch.int32, device=dev)
            J.join_materialize(J.JOIN_KIND_HASH, j.R, j.S, None, ws, out, stream)
            tot += n
        return tot

    per_join()
    pj = [wall(per_join) for _ in range(reps)]
    per_ms = statistics.median(t for t, _ in pj)
    total_pj = pj[-1][1]
    del ws
    torch.cuda.empty_cache()

    cache = tune.load()
    tuned = bool(cache.get("hash_bits"))
    bits = tune.hash_bits_for_sizes(np.diff(roffs), cache) if tuned else None

    def prepare():
        return J.Batch.packed(rk_all, roffs, sk_all, soffs, bits, stream=stream)

    # preparation: host planning from the packed job table, workspace, table upload; the first
    # one also pays one-time runtime set-up, so the steady figure is the median of the others
    tp_first, b = wall(prepare)
    del b
    tps = [wall(prepare) for _ in range(reps)]
    tp = statistics.median(t for t, _ in tps)
    b = tps[-1][1]
    del tps

    def batch_once():
        offs = b.count(stream)
        total = int(offs[-1].item())
        out = torch.empty((total, 2), dtype=torch.int32, device=dev)
        b.materialize(out, stream)
        return total

    batch_once()
    bt = [wall(batch_once) for _ in range(reps)]
    batch_ms = statistics.median(t for t, _ in bt)
    total_b = bt[-1][1]
    assert total_b == total_pj, (total_b, total_pj)

    # the count pass captured once, replayed
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.count(side)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.count()

    def graph_once():
        graph.replay()
        total = int(b.offsets[-1].item())
        out = torch.empty((total, 2), dtype=torch.int32, device=dev)
        b.materialize(out)
        return total

    graph_once()
    gt = [wall(graph_once) for _ in range(reps)]
    graph_ms = statistics.median(t for t, _ in gt)
    assert gt[-1][1] == total_pj
    njobs = len(jobs)
    del graph, b, jobs, rk_all, sk_all
    torch.cuda.empty_cache()
    return {
        "workload": f"{njobs} independent equi joins, per-side sizes log-uniform in [1K, 4M], "
                    "keys uniform over the build size, 10% Zipf(1.0) probe sides",
        "jobs": njobs, "rows_R": rows_r, "rows_S": rows_s, "pairs": total_b,
        "fanout": "autotuned" if tuned else "default rule",
        "per_join_ms": round(per_ms, 2),
        "batch_ms": round(batch_ms, 2),
        "batch_prepare_ms": round(tp, 2),
        "batch_prepare_first_ms": round(tp_first, 2),
        "batch_with_prepare_ms": round(batch_ms + tp, 2),
        "graph_ms": round(graph_ms, 2),
        "per_join_probe_tuples_per_s": round(rows_s / (per_ms * 1e-3), 1),
        "batch_probe_tuples_per_s": round(rows_s / ((batch_ms + tp) * 1e-3), 1),
        "batch_probe_tuples_per_s_without_prepare": round(rows_s / (batch_ms * 1e-3), 1),
        "graph_probe_tuples_per_s": round(rows_s / (graph_ms * 1e-3), 1),
        "speedup_batch_vs_per_join": round(per_ms / (batch_ms + tp), 3),
        "speedup_graph_vs_per_join": round(per_ms / graph_ms, 3),
        "timing": "host wall clock, median of 3, count + total read + exact allocation + write; "
                  "the batched figures include prepare (job table from packed columns, host "
                  "planning, workspace, table upload; median of 3 after a first one) once; the "
                  "graph replays a prepared batch",
    }


def bench_serve(args, J):
    """Serving: Poisson stream, 80% equi / 20% band (w = 8) joins, per-side sizes log-uniform in
    [1K, 8M], 30% of requests probing one of 16 resident builds, 64 GB HBM budget.  Closed-loop
    capacity with 4 slots, then open loop at 0.5x and 0.8x that rate; the plain form (one slot,
    no resident builds) closed loop beside it."""
    import torch
    from paper_1904_11201_amd import serve
    t0 = time.time()
    builds, reqs = serve.requests_device(seed=7, count=args.serve_requests)
    torch.cuda.synchronize()
    print(f"# serve: {len(reqs)} requests generated in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    eng = serve.Engine(builds, slots=4, budget_bytes=64 << 30)
    plain = serve.Engine(builds, slots=1, budget_bytes=64 << 30, resident=False)
    eng.serve(reqs[:16], open_loop=False, keep_pairs=False)  # warm-up
    res_c, wall = eng.serve(reqs, open_loop=False, keep_pairs=False)
    closed = serve.summary(res_c, wall)
    mu = closed["requests_per_s"]
    res, wall = plain.serve(reqs, open_loop=False, keep_pairs=False)
    plain_closed = serve.summary(res, wall)
    opened = {}
    for f in (0.5, 0.8):
        res, wall = eng.serve(serve.at_rate(reqs, f * mu), open_loop=True, keep_pairs=False)
        opened[f"{f}x"] = dict(serve.summary(res, wall), qps=round(f * mu, 2))
        print(f"# serve open loop {f}x: {opened[f'{f}x']}", file=sys.stderr, flush=True)
    # the same stream under a budget that binds: 5% above the largest single request's
    # workspace + output, so that a large request in flight holds the others back
    budget = int(1.05 * eng.max_request)
    tight = serve.Engine(builds, slots=4, budget_bytes=budget)
    res_t, wall = tight.serve(reqs, open_loop=False, keep_pairs=False)
    same = all(a.count == b.count for a, b in zip(res_c, res_t))
    bound = dict(serve.summary(res_t, wall), budget_bytes=tight.budget,
                 largest_request_bytes=eng.max_request,
                 peak_reserved_bytes=tight.peak, admission_waits=tight.waits,
                 restarts=tight.retries, counts_equal_unbounded=same)
    assert same, "a request's count differs under the binding budget"
    del tight
    n_theta = sum(r.kind == "theta" for r in reqs)
    n_res = sum(r.R is None for r in reqs)
    out = {
        "workload": f"{len(reqs)} requests: {len(reqs) - n_theta} equi ({n_res} on resident "
                    f"builds), {n_theta} band w=8 (region pruned); sizes log-uniform [1K, 8M]",
        "slots": eng.slots, "budget_bytes": eng.budget, "peak_reserved_bytes": eng.peak,
        "resident_build_bytes": eng.resident_bytes, "admission_waits": eng.waits,
        "closed_loop": closed, "plain_closed_loop": plain_closed,
        "throughput_vs_plain": round(closed["pairs_per_s"] / plain_closed["pairs_per_s"], 3),
        "open_loop": opened,
        "closed_loop_binding_budget": bound,
        "latency": "arrival to completion on the host clock, count + admission + write",
    }
    del eng, plain, builds, reqs
    torch.cuda.empty_cache()
    return out


def measure_ceilings(J, _native, dev, stream, reps=5):
    """What the chip sustains: 1 GiB read-only, write-only and copy streams (HBM) and the int32
    VALU spins, whose workgroup 0 also reads the shader clock against the constant real-time
    counter (kept per spin)."""
    import torch
    props = torch.cuda.get_device_properties(dev)
    cus = props.multi_processor_count
    nb = 1 << 30
    src = torch.ones(nb // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    rsink = torch.empty(2 * 1024 * cus, dtype=torch.int32, device=dev)
    blocks, iters = cus * 8, 1 << 14
    sink = torch.empty(blocks * 256, dtype=torch.int32, device=dev)
    clk = torch.zeros(2, dtype=torch.int64, device=dev)
    J.prof_copy(src, dst, stream)
    J.prof_stream("read", src, rsink, stream)
    J.prof_stream("write", dst, None, stream)
    ops = {m: J.prof_valu(blocks, iters, sink, clk, stream, mix=m) for m in (0, 1, 2, 3, 4)}
    torch.cuda.synchronize()
    _native.prof_enable(True)
    for _ in range(reps):
        J.prof_copy(src, dst, stream)
        J.prof_stream("read", src, rsink, stream)
        J.prof_stream("write", dst, None, stream)
    ghz = {}
    hz = J.prof_wall_clock_hz()
    for mix in (0, 1, 2, 3, 4):
        for _ in range(reps):
            J.prof_valu(blocks, iters, sink, clk, stream, mix=mix)
        cyc, ticks = (int(v) for v in clk.cpu().tolist())  # the last launch of this spin
        ghz[mix] = cyc / (ticks / hz) / 1e9 if ticks > 0 else None
    torch.cuda.synchronize()
    p = _native.prof_read()
    _native.prof_enable(False)
    del src, dst, sink, clk, rsink
    torch.cuda.empty_cache()

    def avg(name):
        return p[name][1] / p[name][0]

    def tops(mix, name):
        return ops[mix] / (avg(name) * 1e-3) / 1e12

    def per_cu_clk(mix, name):
        # wave64 VALU instructions per compute unit and shader clock
        g = ghz[mix]
        return g and round(tops(mix, name) * 1e12 / 64 / cus / (g * 1e9), 3)

    out = {
        "compute_units": cus,
        "read_GBps": round(nb / (avg("ceiling.read") * 1e-3) / 1e9, 1),
        "write_GBps": round(nb / (avg("ceiling.write") * 1e-3) / 1e9, 1),
        "copy_GBps": round(2 * nb / (avg("ceiling.copy") * 1e-3) / 1e9, 1),
        "stream_workload": "1 GiB read-only, write-only and copy streams of 16-byte non-temporal "
                           "accesses, 2 workgroups of 1024 lanes per CU (the fastest shape of a "
                           f"sweep), copy traffic counted both ways, mean of {reps}",
    }
    names = {0: "ceiling.valu", 1: "ceiling.valu.band", 2: "ceiling.valu.min",
             3: "ceiling.valu.sub", 4: "ceiling.valu.min3"}
    desc = {0: "v_add_u32 + v_xor_b32 chains", 1: "v_sub_u32 from a scalar, v_cmp_le_u32 into "
            "VCC, s_or_b64: a compare-per-pair band test", 2: "two v_sub_u32 from a scalar, one "
            "v_min3_u32 into one of two running minima: the nested-loop join's group filter",
            3: "v_sub_u32 from a scalar only", 4: "v_min3_u32 only"}
    key = {0: "valu", 1: "valu_band", 2: "valu_min", 3: "valu_sub", 4: "valu_min3"}
    for m in (0, 1, 2, 3, 4):
        out[f"{key[m]}_Tops"] = round(tops(m, names[m]), 2)
        out[f"{key[m]}_shader_clock_GHz"] = ghz[m] and round(ghz[m], 3)
        out[f"{key[m]}_insts_per_cu_clk"] = per_cu_clk(m, names[m])
        out[f"{key[m]}_workload"] = (f"{blocks} workgroups x 256 lanes x "
                                     f"{(48 if m == 2 else 32) * iters} instructions: {desc[m]} "
                                     f"(mean of {reps})")
    out["valu_peak_Tops"] = round(VALU_PEAK_TOPS, 2)
    out["valu_peak_model"] = (f"{cus} CUs x {VALU_ISSUE_PER_CU_CLK} wave64 VALU instructions per "
                              "CU and clock x 64 lanes x 2.4 GHz")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is a design in DESIGN.md, not a measured path)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1904_11201_amd import _native, datagen
    from paper_1904_11201_amd import join as J

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    def d(a):
        return None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(dev)

    def rel(r):
        return J.Relation(d(r.key), d(r.key2), d(r.rid))

    t_gen = time.time()
    Ru, Su, _ = datagen.large_equi(seed=2, zipf=False)
    Rz, Sz, _ = datagen.large_equi(seed=3, zipf=True)
    Rt, St = datagen.band_theta(seed=4, n=1 * M)
    Rl, Sl = datagen.lt_theta(seed=5, n=64 * 1024)
    Rc1, Sc1 = datagen.small_equi(seed=1)
    dRu, dSu, dRz, dSz = rel(Ru), rel(Su), rel(Rz), rel(Sz)
    dRt, dSt, dRl, dSl = rel(Rt), rel(St), rel(Rl), rel(Sl)
    dRc1, dSc1 = rel(Rc1), rel(Sc1)
    print(f"# inputs generated and resident in {time.time() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    nR, nS = Ru.n, Su.n
    theta_pred = J.Pred("band", 8, "lt")
    ws_h = J.workspace(J.JOIN_KIND_HASH, nR, nS)
    ws_t = J.workspace(J.JOIN_KIND_THETA, Rt.n, St.n, theta_pred)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def run_join(kind, R, S, pred, ws):
        # The output is allocated at the exact count inside the timed region and released after
        # its write pass is queued: the caching allocator hands the same block to the next join,
        # as a serving loop reusing its memory would, instead of a fresh device allocation.
        a, b = ev(), ev()
        a.record(stream)
        n = J.join_count(kind, R, S, pred, ws, stream)
        t_a = time.perf_counter()
        out = torch.empty((n, 2), dtype=torch.int32, device=dev)
        alloc_us = (time.perf_counter() - t_a) * 1e6
        J.join_materialize(kind, R, S, pred, ws, out, stream)
        b.record(stream)
        del out
        return n, alloc_us, (a, b)

    def step():
        hu = run_join(J.JOIN_KIND_HASH, dRu, dSu, None, ws_h)
        hz = run_join(J.JOIN_KIND_HASH, dRz, dSz, None, ws_h)
        th = run_join(J.JOIN_KIND_THETA, dRt, dSt, theta_pred, ws_t)
        return hu, hz, th

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # The timed steps run without the library's per-kernel events: a pair of events around every
    # launch adds about 10 us at each boundary between dependent kernels on this GPU.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # Per-kernel launch durations: the same joins again, every launch bracketed by HIP events on
    # its own stream, one workload at a time (so that each join's kernels have their own table).
    def profiled(fn):
        _native.prof_enable(True)
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        t = _native.prof_read()
        _native.prof_enable(False)
        return t

    prof_u = profiled(lambda: run_join(J.JOIN_KIND_HASH, dRu, dSu, None, ws_h))
    prof_z = profiled(lambda: run_join(J.JOIN_KIND_HASH, dRz, dSz, None, ws_h))
    prof_t = profiled(lambda: run_join(J.JOIN_KIND_THETA, dRt, dSt, theta_pred, ws_t))
    prof = {}
    for t in (prof_u, prof_z, prof_t):
        for k, (n, ms) in t.items():
            a = prof.get(k, (0, 0.0))
            prof[k] = (a[0] + n, a[1] + ms)

    wall_ms = (t1 - t0) * 1e3 / args.steps
    ceilings = measure_ceilings(J, _native, dev, stream)
    hu_ms = [r[0][2][0].elapsed_time(r[0][2][1]) for r in recs]
    hz_ms = [r[1][2][0].elapsed_time(r[1][2][1]) for r in recs]
    th_ms = [r[2][2][0].elapsed_time(r[2][2][1]) for r in recs]
    n_hu, n_hz, n_th = recs[-1][0][0], recs[-1][1][0], recs[-1][2][0]
    # host time of the exact-size output allocation inside each hash join (caching allocator)
    alloc_us = [r[i][1] for r in recs for i in (0, 1)]
    assert n_hu == nS and n_hz == nS, "16M x 64M outputs must hold exactly |S| pairs"
    del recs

    hash_ms = statistics.mean(hu_ms) + statistics.mean(hz_ms)
    probe_tps = 2 * nS / (hash_ms * 1e-3)
    hash_pairs_ps = (n_hu + n_hz) / (hash_ms * 1e-3)
    th_mean = statistics.mean(th_ms)
    theta_pairs_eval_ps = Rt.n * St.n / (th_mean * 1e-3)

    # count-only R.a < S.a, 64K x 64K (no write pass)
    lt_pred = J.Pred("lt")
    ws_l = J.workspace(J.JOIN_KIND_THETA, Rl.n, Sl.n, lt_pred)
    lt_ms = []
    for i in range(args.warmup + 20):
        a, b = ev(), ev()
        a.record(stream)
        n_lt = J.join_count(J.JOIN_KIND_THETA, dRl, dSl, lt_pred, ws_l, stream)
        b.record(stream)
        torch.cuda.synchronize()
        if i >= args.warmup:
            lt_ms.append(a.elapsed_time(b))

    # the same count by region pruning: green tiles are counted as products, white skipped, and
    # only the diagonal (red) tiles evaluated
    ws_lr = J.workspace(J.JOIN_KIND_THETA_REGION, Rl.n, Sl.n, lt_pred)
    lt_reg_ms = []
    for i in range(args.warmup + 20):
        a, b = ev(), ev()
        a.record(stream)
        n_lt_reg = J.join_count(J.JOIN_KIND_THETA_REGION, dRl, dSl, lt_pred, ws_lr, stream)
        b.record(stream)
        torch.cuda.synchronize()
        if i >= args.warmup:
            lt_reg_ms.append(a.elapsed_time(b))
    assert n_lt_reg == n_lt, (n_lt_reg, n_lt)
    del ws_lr

    # the same band join by region pruning (shared value buckets; only red tiles evaluated)
    ws_r = J.workspace(J.JOIN_KIND_THETA_REGION, Rt.n, St.n, theta_pred)
    reg_ms = []
    for i in range(args.warmup + 10):
        a, b = ev(), ev()
        a.record(stream)
        n_reg = J.join_count(J.JOIN_KIND_THETA_REGION, dRt, dSt, theta_pred, ws_r, stream)
        out = torch.empty((n_reg, 2), dtype=torch.int32, device=dev)
        J.join_materialize(J.JOIN_KIND_THETA_REGION, dRt, dSt, theta_pred, ws_r, out, stream)
        b.record(stream)
        torch.cuda.synchronize()
        if i >= args.warmup:
            reg_ms.append(a.elapsed_time(b))
    assert n_reg == n_th, (n_reg, n_th)
    del ws_r, out

    # single-request latency of the small equi join (64K x 64K), host-observed, end to end
    ws_c1 = J.workspace(J.JOIN_KIND_HASH, Rc1.n, Sc1.n)
    lat = []
    for i in range(args.latency_runs + 10):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        n_c1 = J.join_count(J.JOIN_KIND_HASH, dRc1, dSc1, None, ws_c1, stream)
        out = torch.empty((n_c1, 2), dtype=torch.int32, device=dev)
        J.join_materialize(J.JOIN_KIND_HASH, dRc1, dSc1, None, ws_c1, out, stream)
        torch.cuda.synchronize()
        if i >= 10:
            lat.append((time.perf_counter() - s0) * 1e3)
    lat.sort()

    def pct(v, q):
        return v[min(len(v) - 1, int(round(q * (len(v) - 1))))]

    # pre-filter: a 1M-row build (keys: multiples of 100 below 100M) probed by 64M keys uniform
    # in [0, 100M), so one probe in a hundred matches
    g_pf = torch.Generator(device=dev)
    g_pf.manual_seed(8)
    R_pf = J.Relation(torch.arange(0, 100 * M, 100, device=dev, dtype=torch.int32))
    S_pf = J.Relation(torch.randint(0, 100 * M, (nS,), device=dev, dtype=torch.int32, generator=g_pf))
    pf = {}
    canon = {}
    for name, kind in (("plain_ms", J.JOIN_KIND_HASH), ("prefilter_ms", J.JOIN_KIND_HASH_PREFILTER)):
        ws_pf = J.workspace(kind, R_pf.n, nS)
        ts = []
        for i in range(args.warmup + 5):
            a, b = ev(), ev()
            a.record(stream)
            n_pf = J.join_count(kind, R_pf, S_pf, None, ws_pf, stream)
            out = torch.empty((n_pf, 2), dtype=torch.int32, device=dev)
            J.join_materialize(kind, R_pf, S_pf, None, ws_pf, out, stream)
            b.record(stream)
            torch.cuda.synchronize()
            if i >= args.warmup:
                ts.append(a.elapsed_time(b))
        pf[name] = round(statistics.median(ts), 4)
        pf["pairs"] = n_pf
        # the pairs in canonical order (R rid, then S rid), compared below: the pre-filtered join
        # must give the plain join's pairs
        canon[name] = torch.sort(out[:, 0].to(torch.int64) * (1 << 32) + out[:, 1].to(torch.int64)).values
        del ws_pf, out
    if not torch.equal(canon["plain_ms"], canon["prefilter_ms"]):
        raise SystemExit("bench: the pre-filtered 1M x 64M join's pairs differ from the plain join's")
    del canon
    pf["same_pairs_as_plain"] = True
    pf["speedup"] = round(pf["plain_ms"] / pf["prefilter_ms"], 3)
    pf["workload"] = ("hash equi-join 1M x 64M, R keys the multiples of 100 below 100M, S keys "
                      "uniform in [0, 100M): one probe in a hundred matches")
    del R_pf, S_pf
    torch.cuda.empty_cache()

    batch = bench_batch(args, J, datagen, dev, stream) if args.batch_jobs > 0 else None
    serving = bench_serve(args, J) if args.serve_requests > 0 else None

    # ---- per-kernel figures over the profiled steps (HIP events on the launch stream) -------
    traffic = load_traffic()
    valu = load_valu()
    pairs_band = Rt.n * St.n
    alg = {
        # algorithmic bytes per launch (HBM-bound kernels) or int32 ops (ALU-bound): the
        # per-unit figures of the scope table times the units of one launch
        "hash.hist": ("hbm", 4 * (nR + nS), "read"),  # both sides in one launch
        "hash.scatter": ("hbm", 16 * (nR + nS), "copy"),
        "hash.count": ("hbm", 4 * nR + 4 * nS, "read"),
        "hash.write": ("hbm", 8 * nR + 8 * nS + 8 * nS, "copy"),
        # band and R.c < S.c: one subtract and two compares per pair
        "theta.count": ("alu", 3 * pairs_band, None),
        "theta.write": ("hbm", 16 * n_th, "copy"),
    }
    spin_rate = {"theta.count": ceilings["valu_min_Tops"]}  # the spin of its own sequence

    def kernel_lines(table, steps_ms):
        rows = []
        for name, (launches, tot_ms) in sorted(table.items(), key=lambda kv: -kv[1][1]):
            avg = tot_ms / launches
            k = {"name": name, "launches": launches, "avg_ms": round(avg, 4),
                 "share_of_step": round(tot_ms / args.steps / steps_ms, 4)}
            if name in alg:
                bound, work, mix = alg[name]
                if bound == "hbm":
                    ach = work / (avg * 1e-3) / 1e9
                    meas = ceilings[f"{mix}_GBps"]
                    k.update(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=round(ach / HBM_PEAK_GBS, 4),
                             measured_ceiling=f"{mix} stream, {meas} GB/s",
                             frac_of_measured_ceiling=round(ach / meas, 4))
                    t = traffic.get(name)
                    k["traffic"] = t
                    if t:
                        k["traffic_GBps"] = round(t / (avg * 1e-3) / 1e9, 1)
                else:
                    ach = work / (avg * 1e-3) / 1e12
                    k.update(bound="alu", achieved=round(ach, 2), peak=round(VALU_PEAK_TOPS, 2),
                             unit="Tops/s", frac=round(ach / VALU_PEAK_TOPS, 4),
                             work="3 int32 ops per pair (one subtract, two compares)")
                    v = valu.get(name)
                    k["traffic"] = traffic.get(name)
                    if v:
                        lane_ops = v["SQ_INSTS_VALU"] * 64
                        rate = lane_ops / (avg * 1e-3) / 1e12
                        k.update(counter_lane_ops=lane_ops, counter_Tops=round(rate, 2),
                                 counter_frac=round(rate / VALU_PEAK_TOPS, 4),
                                 frac_of_measured_ceiling=round(rate / spin_rate[name], 4),
                                 measured_ceiling=f"spin of the same instruction sequence, "
                                                  f"{spin_rate[name]} T lane-ops/s")
            rows.append(k)
        return rows

    kernels = kernel_lines(prof, wall_ms)
    dom = max((k for k in kernels if "bound" in k), key=lambda k: k["launches"] * k["avg_ms"])
    roofline = {"kernel": dom["name"], "bound": dom["bound"], "achieved": dom["achieved"],
                "peak": dom["peak"], "unit": dom["unit"], "frac": dom["frac"],
                "traffic": dom.get("traffic")}
    for f in ("work", "counter_Tops", "counter_frac", "measured_ceiling", "frac_of_measured_ceiling"):
        if f in dom:
            roofline[f] = dom[f]

    def hash_graded(table, ms):
        """HBM bytes the counters saw over the join's kernels / their summed time / 8 TB/s."""
        names = [k for k in table if k.startswith("hash.")]
        t_ms = sum(table[k][1] / table[k][0] for k in names)
        if not names or any(traffic.get(k) is None for k in names if k in alg):
            return None
        b = sum(traffic[k] for k in names if k in alg)
        return {"kernels": sorted(names), "hbm_bytes": b, "kernel_ms": round(t_ms, 4),
                "GBps": round(b / (t_ms * 1e-3) / 1e9, 1),
                "frac": round(b / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "algorithmic_bytes": 8 * nR + 8 * nS + 8 * nS,
                "algorithmic_frac": round((8 * nR + 16 * nS) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "algorithmic_basis": "8 B per R and S tuple read once + 8 B per output pair, over "
                                     "the whole join (count, allocation, write)"}

    # ---- CPU oracle on a bounded sample of the same workload --------------------------------
    # The oracle as it stands, timed on this host: the sort-merge equi join is sequential code,
    # so "all threads" runs one instance per thread on disjoint slices of S (each sorting all of
    # R, as one call does); the nested-loop theta oracle is OpenMP code, run with 1 thread and
    # with every thread of the host.
    cpu = None
    cpu_theta = None
    if not args.no_cpu_baseline:
        import concurrent.futures
        import ctypes
        import oracle
        nthr = host_threads()
        samp = 8 * M
        c0 = time.perf_counter()
        oracle.equi_sortmerge(Ru.key, Su.key[:samp], Rrid=Ru.rid, Srid=Su.rid[:samp])
        c1 = time.perf_counter()
        one = samp / (c1 - c0)
        per = max(1, (nS - samp) // nthr)
        slices = [(samp + i * per, samp + (i + 1) * per) for i in range(nthr)]

        def leg(lo_hi):
            lo, hi = lo_hi
            oracle.equi_sortmerge(Ru.key, Su.key[lo:hi], Rrid=Ru.rid, Srid=Su.rid[lo:hi])

        c2 = time.perf_counter()
        with concurrent.futures.ThreadPoolExecutor(nthr) as ex:
            list(ex.map(leg, slices))
        c3 = time.perf_counter()
        allv = per * nthr / (c3 - c2)
        model = cpu_model()
        cpu = {"value": round(one, 1), "unit": "probe tuples/s", "cores": 1, "kind": "oracle",
               "sample": f"sort-merge oracle, all 16M R tuples x the first {samp} of the 64M "
                         f"uniform S tuples, pairs materialised and sorted ({c1 - c0:.1f}s)",
               "cpu_model": model,
               "all_threads": {"value": round(allv, 1), "cores": nthr,
                               "sample": f"{nthr} concurrent oracle calls, each all 16M R tuples x "
                                         f"{per} further S tuples ({c3 - c2:.1f}s)"}}
        rows = 8192
        gomp = None
        try:
            gomp = ctypes.CDLL("libgomp.so.1")
        except OSError:
            pass
        theta_legs = {}
        for t in (1, oracle.threads()):
            if gomp is None and t != oracle.threads():
                continue
            if gomp is not None:
                gomp.omp_set_num_threads(t)
            r = rows if t > 1 else rows // 8
            c0 = time.perf_counter()
            oracle.theta_nlj(Rt.key[:r], St.key, "band", w=8, Rc=Rt.key2[:r], Sc=St.key2,
                             op_c="lt", Rrid=Rt.rid[:r], Srid=St.rid)
            c1 = time.perf_counter()
            theta_legs[t] = (round(r * St.n / (c1 - c0), 1), r, c1 - c0)
        if gomp is not None:
            gomp.omp_set_num_threads(oracle.threads())
        tmax = max(theta_legs)
        v, r, secs = theta_legs[tmax]
        cpu_theta = {"value": v, "unit": "pair evaluations/s", "cores": tmax, "kind": "oracle",
                     "sample": f"brute-force nested-loop oracle, {r} R rows x all 1M S rows "
                               f"({secs:.1f}s)", "cpu_model": model}
        if 1 in theta_legs and tmax != 1:
            v1, r1, s1 = theta_legs[1]
            cpu_theta["one_thread"] = {"value": v1, "cores": 1,
                                       "sample": f"{r1} R rows x all 1M S rows ({s1:.1f}s)"}

    def pcts(v):
        v = sorted(v)
        return {"p50_ms": round(pct(v, 0.5), 4), "p99_ms": round(pct(v, 0.99), 4), "runs": len(v)}

    out = {
        "metric": METRIC,
        "value": round(probe_tps, 1),
        "unit": "probe tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "hash equi-join 16M x 64M (uniform and Zipf(1.0) S keys) + band theta "
                        "join 1M x 1M (|R.a-S.a|<=8 and R.c<S.c)",
            "R_rows": nR, "S_rows": nS, "theta_rows": Rt.n,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hash": {
            "ms_uniform": round(statistics.mean(hu_ms), 4),
            "ms_zipf": round(statistics.mean(hz_ms), 4),
            "probe_tuples_per_s": round(probe_tps, 1),
            "pairs_per_s": round(hash_pairs_ps, 1),
            "uniform": pcts(hu_ms),
            "zipf": pcts(hz_ms),
            "output_alloc_us_median": round(statistics.median(alloc_us), 2),
            "graded_uniform": hash_graded(prof_u, statistics.mean(hu_ms)),
            "kernels_uniform": kernel_lines(prof_u, statistics.mean(hu_ms)),
            "kernels_zipf": kernel_lines(prof_z, statistics.mean(hz_ms)),
        },
        "theta": {
            "ms": round(th_mean, 3),
            "pairs_out": n_th,
            "pairs_per_s": round(n_th / (th_mean * 1e-3), 1),
            "pair_evaluations_per_s": round(theta_pairs_eval_ps, 1),
            "lt_count_64k_ms": round(statistics.median(lt_ms), 4),
            "lt_count_64k_pair_evaluations_per_s": round(Rl.n * Sl.n / (statistics.median(lt_ms) * 1e-3), 1),
            "lt_count_64k_frac_of_valu_peak": round(
                2 * Rl.n * Sl.n / (statistics.median(lt_ms) * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4),
            "lt_count_64k_work": "2 int32 ops per pair (compare, accumulate), whole count call",
            "lt_count_64k_count": n_lt,
            "lt_count_64k_region_ms": round(statistics.median(lt_reg_ms), 4),
            "region_ms": round(statistics.median(reg_ms), 4),
            "region_pairs_per_s": round(n_th / (statistics.median(reg_ms) * 1e-3), 1),
            "region_speedup_vs_nested_loop": round(th_mean / statistics.median(reg_ms), 1),
            "cpu_baseline": cpu_theta,
        },
        "latency": {"workload": "hash equi-join 64K x 64K, keys uniform in [0,16384), "
                                "count + exact allocation + write, host-observed",
                    "runs": len(lat), "p50_ms": round(pct(lat, 0.5), 4),
                    "p99_ms": round(pct(lat, 0.99), 4), "pairs": n_c1},
        "prefilter": pf,
        "batch": batch,
        "serve": serving,
        "kernels": kernels,
        "ceilings": ceilings,
        "src_hash": src_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
