"""The benchmark's batch and serving workloads at full size against the oracle.

* Batch: the 4096 uneven equi joins (seed 6, 2.02e9 x 2.05e9 rows, autotuned fan-outs) run as
  one batch, the way the benchmark runs them.  Every join's count is checked against the
  oracle's equi-join count; the pairs of a seeded sample of 40 joins (among them the largest R,
  the largest S and Zipf probe sides) are compared element by element with the sort-merge
  oracle.
* Serving: the 1024-request stream (seed 7: equi joins, 30% of all requests on one of 16
  resident builds, band theta joins through region pruning) served by the engine with 4 slots.
  Every request's count is checked against the oracle (equi count, or the sorted-window band
  count); the pairs of a seeded sample of 24 requests (resident-build, plain equi and band
  requests, the largest band request among them) are compared element by element.

Key columns come back to the host once; oracle calls run in a pool of host threads (the
oracle's C functions release the interpreter lock)."""
from __future__ import annotations

import concurrent.futures
import os

import numpy as np
import torch

import oracle
from paper_1904_11201_amd import datagen
from tests.gpu_util import canon_gpu, gpu, log, need_gpu

_WORKERS = max(1, min(16, os.cpu_count() or 1))


def _pool_map(fn, items):
    with concurrent.futures.ThreadPoolExecutor(_WORKERS) as ex:
        return list(ex.map(fn, items))


def _host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


@gpu
def test_full_batch_4096_joins_against_the_oracle():
    need_gpu()
    from paper_1904_11201_amd import join as J
    from paper_1904_11201_amd import tune
    raw = datagen.batch_jobs_device(seed=6, jobs=4096, device="cuda")
    jobs = [J.Job(J.Relation(rk), J.Relation(sk)) for rk, sk, _ in raw]
    cache = tune.load()
    if cache.get("hash_bits"):
        jobs = tune.apply_bits(jobs, cache)
    log(f"full batch: {len(jobs)} joins, {sum(j.R.n for j in jobs)} x {sum(j.S.n for j in jobs)} rows")
    b = J.Batch(jobs)
    offs = b.count()
    total = int(offs[-1].item())
    out = torch.empty((total, 2), dtype=torch.int32, device="cuda")
    b.materialize(out)
    torch.cuda.synchronize()
    offs_h = _host(offs).astype(np.int64)
    keys = [(_host(rk), _host(sk)) for rk, sk, _ in raw]
    log(f"full batch: {total} pairs; oracle counts of every join ({_WORKERS} host threads)")
    want = np.array(_pool_map(lambda k: oracle.count_equi(k[0], k[1]), keys), dtype=np.int64)
    got = np.diff(offs_h)
    bad = np.flatnonzero(got != want)
    assert len(bad) == 0, [(int(j), int(got[j]), int(want[j])) for j in bad[:5]]
    assert offs_h[0] == 0 and offs_h[-1] == total == int(want.sum())

    # element-by-element sample: the largest R, the largest S, Zipf probe sides, seeded others
    nR = np.array([len(k[0]) for k in keys])
    nS = np.array([len(k[1]) for k in keys])
    zipf = np.flatnonzero([z for _, _, z in raw])
    g = datagen.rng_for(606)
    pick = {int(np.argmax(nR)), int(np.argmax(nS))}
    pick.update(int(j) for j in g.choice(zipf, size=min(6, len(zipf)), replace=False))
    rest = np.setdiff1d(np.arange(len(jobs)), np.array(sorted(pick)))
    pick.update(int(j) for j in g.choice(rest, size=40 - len(pick), replace=False))
    pick = sorted(pick)
    assert len(pick) == 40 and len(set(pick) & set(zipf.tolist())) >= 4
    log(f"full batch: pairs of {len(pick)} joins (largest R {nR.max()}, largest S {nS.max()})")
    refs = _pool_map(lambda j: oracle.equi_sortmerge(keys[j][0], keys[j][1]), pick)
    for j, (n, ref) in zip(pick, refs):
        part = canon_gpu(out[int(offs_h[j]):int(offs_h[j + 1])])
        assert len(part) == n and np.array_equal(part, ref), (j, int(nR[j]), int(nS[j]))


@gpu
def test_full_serving_stream_against_the_oracle():
    need_gpu()
    from paper_1904_11201_amd import serve
    builds, reqs = serve.requests_device(seed=7, count=1024)
    eng = serve.Engine(builds, slots=4, budget_bytes=64 << 30)
    n_theta = sum(r.kind == "theta" for r in reqs)
    n_res = sum(r.R is None for r in reqs)
    log(f"full serving stream: {len(reqs)} requests ({n_theta} band, {n_res} on resident builds)")
    res, _ = eng.serve(reqs, open_loop=False, keep_pairs=True)
    torch.cuda.synchronize()
    bkeys = [_host(b.key) for b in builds]

    def columns(r):
        Ra = bkeys[r.build_id] if r.R is None else _host(r.R.key)
        return Ra, _host(r.S.key)

    cols = [columns(r) for r in reqs]

    def count(i):
        r = reqs[i]
        Ra, Sa = cols[i]
        if r.kind == "hash":
            return oracle.count_equi(Ra, Sa)
        return oracle.band_window(Ra, Sa, r.w, want_pairs=False)[0]

    log(f"full serving stream: oracle counts of every request ({_WORKERS} host threads)")
    want = _pool_map(count, range(len(reqs)))
    bad = [(i, res[i].count, want[i]) for i in range(len(reqs)) if res[i].count != want[i]]
    assert not bad, bad[:5]
    assert all(res[i].pairs.shape[0] == want[i] for i in range(len(reqs)))

    # element-by-element sample: resident-build, plain equi and band requests
    g = datagen.rng_for(707)
    resident = [i for i, r in enumerate(reqs) if r.R is None]
    plain = [i for i, r in enumerate(reqs) if r.kind == "hash" and r.R is not None]
    band = [i for i, r in enumerate(reqs) if r.kind == "theta"]
    biggest_band = max(band, key=lambda i: want[i])
    pick = {biggest_band}
    for group in (resident, plain, band):
        pick.update(int(i) for i in g.choice(group, size=8, replace=False))
    pick = sorted(pick)
    assert len(pick) >= 16
    log(f"full serving stream: pairs of {len(pick)} requests (largest band output {want[biggest_band]})")

    def ref(i):
        r = reqs[i]
        Ra, Sa = cols[i]
        if r.kind == "hash":
            return oracle.equi_sortmerge(Ra, Sa)
        return oracle.band_window(Ra, Sa, r.w)

    refs = _pool_map(ref, pick)
    for i, (n, rp) in zip(pick, refs):
        got = canon_gpu(res[i].pairs)
        assert len(got) == n and np.array_equal(got, rp), (i, reqs[i].kind, reqs[i].build_id)
