"""Serving loop: every request's result is the same alone and in the mix (bit-exact after
canonical sorting, and equal to the oracle), resident builds give the same pairs as plain joins,
and memory admission stays within the budget even when it forces requests to wait."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_1904_11201_amd import datagen
from tests.gpu_util import canon_gpu, dev_rel, gpu, log, need_gpu


def _workload(seed=71, count=30):
    g = datagen.rng_for(seed)
    builds = [datagen.Rel(key=datagen.uniform_keys(g, n, 0, n)) for n in (5000, 200_000, 400_000, 1000)]
    reqs = []
    for i in range(count):
        u = g.random()
        if u < 0.25:
            nr, ns = (int(x) for x in datagen.log_uniform_sizes(g, 2, 500, 40_000))
            R = datagen.Rel(key=datagen.uniform_keys(g, nr, 0, 1 << 24), key2=datagen.uniform_keys(g, nr, 0, 1 << 24))
            S = datagen.Rel(key=datagen.uniform_keys(g, ns, 0, 1 << 24), key2=datagen.uniform_keys(g, ns, 0, 1 << 24))
            reqs.append(("theta", R, S, -1))
        elif u < 0.6:
            b = int(g.integers(0, len(builds)))
            ns = int(datagen.log_uniform_sizes(g, 1, 500, 300_000)[0])
            S = datagen.Rel(key=datagen.uniform_keys(g, ns, 0, builds[b].n), rid=g.permutation(ns).astype(np.int32))
            reqs.append(("hash", None, S, b))
        else:
            nr, ns = (int(x) for x in datagen.log_uniform_sizes(g, 2, 500, 300_000))
            R = datagen.Rel(key=datagen.uniform_keys(g, nr, 0, nr))
            S = datagen.Rel(key=datagen.uniform_keys(g, ns, 0, nr))
            reqs.append(("hash", R, S, -1))
    return builds, reqs


def _oracle(kind, R, S):
    rr = R.rid if R.rid is not None else np.arange(R.n, dtype=np.int32)
    sr = S.rid if S.rid is not None else np.arange(S.n, dtype=np.int32)
    if kind == "hash":
        return oracle.equi_sortmerge(R.key, S.key, Rrid=rr, Srid=sr)
    return oracle.band_window(R.key, S.key, 8, Rrid=rr, Srid=sr)


def _engine_requests(builds, reqs):
    from paper_1904_11201_amd.serve import Request
    out = []
    for i, (kind, R, S, b) in enumerate(reqs):
        out.append(Request(i, kind, dev_rel(S), None if R is None else dev_rel(R), b, 8, 0.0))
    return out


@gpu
def test_results_alone_equal_results_in_the_mix():
    need_gpu()
    from paper_1904_11201_amd.serve import Engine
    builds, reqs = _workload()
    dbuilds = [dev_rel(B) for B in builds]
    eng = Engine(dbuilds, slots=4)
    assert sum(r is not None for r in eng.resident) == 2  # the two builds above the single-path size
    ereqs = _engine_requests(builds, reqs)
    log(f"serving {len(ereqs)} requests alone (one slot)")
    alone, _ = Engine(dbuilds, slots=1).serve(ereqs, open_loop=False)
    log("serving the same requests in the mix (four slots)")
    mix, _ = eng.serve(ereqs, open_loop=False)
    assert len({r.slot for r in mix}) > 1
    for i, (kind, R, S, b) in enumerate(reqs):
        Rh = builds[b] if R is None else R
        n, ref = _oracle(kind, Rh, S)
        a, m = canon_gpu(alone[i].pairs), canon_gpu(mix[i].pairs)
        assert alone[i].count == mix[i].count == n, (i, kind)
        assert np.array_equal(a, m) and np.array_equal(m, ref), (i, kind)


@gpu
def test_resident_build_equals_plain_join():
    need_gpu()
    from paper_1904_11201_amd.join import ResidentBuild, hash_join, Relation
    g = datagen.rng_for(72)
    R = datagen.Rel(key=datagen.uniform_keys(g, 300_000, 0, 50_000), rid=g.permutation(300_000).astype(np.int32))
    dR = dev_rel(R)
    rb = ResidentBuild(dR)
    for ns in (0, 1, 1000, 250_000):
        S = datagen.Rel(key=datagen.uniform_keys(g, ns, 0, 60_000))
        dS = dev_rel(S)
        log(f"resident build probe ns={ns}")
        got = canon_gpu(rb.probe(dS))
        n, ref = _oracle("hash", R, S)
        assert len(got) == n and np.array_equal(got, ref)
        assert np.array_equal(got, canon_gpu(hash_join(dR, dS)))


@gpu
def test_small_budget_forces_waits_and_stays_within_it():
    need_gpu()
    from paper_1904_11201_amd.serve import BudgetError, Engine
    from paper_1904_11201_amd import join as J
    builds, reqs = _workload(seed=73, count=16)
    dbuilds = [dev_rel(B) for B in builds]
    ereqs = _engine_requests(builds, reqs)
    need = []
    for (kind, R, S, b), er in zip(reqs, ereqs):
        Rh = builds[b] if R is None else R
        n, _ = _oracle(kind, Rh, S)
        k = J.JOIN_KIND_HASH if kind == "hash" else J.JOIN_KIND_THETA_REGION
        p = None if kind == "hash" else J.Pred("band", 8, "none")
        need.append(J.join_workspace_bytes(k, Rh.n, S.n, p) + 8 * n)
    budget = int(1.2 * max(need))
    eng = Engine(dbuilds, slots=4, budget_bytes=budget)
    log(f"serving with a budget of {budget} bytes")
    res, _ = eng.serve(ereqs, open_loop=False)
    assert eng.peak <= budget and eng.reserved == 0 and eng.active == 0
    for i, (kind, R, S, b) in enumerate(reqs):
        n, ref = _oracle(kind, builds[b] if R is None else R, S)
        assert np.array_equal(canon_gpu(res[i].pairs), ref), i
    with pytest.raises(BudgetError):
        Engine(dbuilds, slots=2, budget_bytes=min(need) // 2).serve(ereqs[:2], open_loop=False)
