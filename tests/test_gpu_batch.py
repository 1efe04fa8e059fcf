"""Batched equi joins (join_batch_*): every join of a batch against the oracle, through one set of
fused launches, including a count pass captured in a HIP graph and replayed."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_1904_11201_amd import datagen
from tests.gpu_util import canon_gpu, dev_rel, gpu, log, need_gpu


def _mixed_jobs(seed: int, n: int, hi: int):
    """Uneven joins: sizes log-uniform in [1, hi] per side, some empty sides, keys uniform over a
    domain equal to |R| (so about one match per probe), a few Zipf probe sides, rid payloads or
    none, and some forced fan-outs."""
    g = datagen.rng_for(seed)
    jobs = []
    for j in range(n):
        nr, ns = (int(x) for x in datagen.log_uniform_sizes(g, 2, 1, hi))
        if j % 11 == 3:
            nr = 0
        if j % 13 == 5:
            ns = 0
        d = max(nr, 1)
        rk = datagen.uniform_keys(g, nr, 0, d)
        if j % 7 == 2:
            sk = (datagen.zipf_ranks(g, ns, d, 1.0) - 1).astype(np.int32)
        else:
            sk = datagen.uniform_keys(g, ns, 0, d)
        rid_mode = j % 3
        R = datagen.Rel(key=rk, rid=None if rid_mode == 0 else g.permutation(nr).astype(np.int32))
        S = datagen.Rel(key=sk, rid=None if rid_mode == 1 else g.integers(-2**31, 2**31 - 1, ns, dtype=np.int64).astype(np.int32))
        bits = -1 if j % 5 else int(g.integers(0, 12))
        jobs.append((R, S, bits))
    return jobs


def _to_jobs(jobs):
    from paper_1904_11201_amd.join import Job
    return [Job(dev_rel(R), dev_rel(S), bits) for R, S, bits in jobs]


def _ref(R, S):
    rr = R.rid if R.rid is not None else np.arange(R.n, dtype=np.int32)
    sr = S.rid if S.rid is not None else np.arange(S.n, dtype=np.int32)
    return oracle.equi_sortmerge(R.key, S.key, Rrid=rr, Srid=sr)


def _check_batch(jobs, pairs, offs):
    assert offs[0] == 0 and all(offs[i] <= offs[i + 1] for i in range(len(jobs)))
    assert offs[-1] == pairs.shape[0]
    for j, (R, S, _) in enumerate(jobs):
        n, ref = _ref(R, S)
        got = canon_gpu(pairs[offs[j]:offs[j + 1]])
        assert offs[j + 1] - offs[j] == n, (j, R.n, S.n)
        assert np.array_equal(got, ref), j


@gpu
def test_mixed_batch_matches_oracle_per_join():
    need_gpu()
    from paper_1904_11201_amd.join import hash_join_batch
    jobs = _mixed_jobs(61, 48, 200_000)
    log(f"batch of {len(jobs)} joins, rows R={sum(r.n for r, _, _ in jobs)} S={sum(s.n for _, s, _ in jobs)}")
    pairs, offs = hash_join_batch(_to_jobs(jobs))
    _check_batch(jobs, pairs, offs)


@gpu
def test_batch_of_one_equals_single_join_and_empty_batch():
    need_gpu()
    from paper_1904_11201_amd.join import hash_join, hash_join_batch, Job
    R, S = datagen.small_equi(seed=1)
    dR, dS = dev_rel(R), dev_rel(S)
    log("batch of one vs single join")
    pairs, offs = hash_join_batch([Job(dR, dS)])
    single = hash_join(dR, dS)
    assert offs == [0, single.shape[0]]
    assert np.array_equal(canon_gpu(pairs), canon_gpu(single))
    log("empty batch")
    pairs, offs = hash_join_batch([])
    assert offs == [0] and pairs.shape[0] == 0


@gpu
def test_small_capacity_writes_nothing():
    need_gpu()
    from paper_1904_11201_amd.join import Batch
    jobs = _mixed_jobs(62, 6, 5_000)
    b = Batch(_to_jobs(jobs))
    total = int(b.count()[-1].item())
    assert total > 1
    log(f"batch materialize into {total - 1} < {total} slots")
    out = torch.full((total - 1, 2), -7, dtype=torch.int32, device="cuda")
    b.materialize(out)
    torch.cuda.synchronize()
    assert bool((out == -7).all())


@gpu
def test_count_pass_in_a_replayed_graph():
    """The count pass (histogram, scatter, planning, count, scans) captured once and replayed;
    every replay, with eager work of another batch in between, gives the eager offsets, and the
    write pass after a replay gives the oracle's pairs."""
    need_gpu()
    from paper_1904_11201_amd.join import Batch
    jobs = _mixed_jobs(63, 24, 100_000)
    other = _mixed_jobs(64, 8, 50_000)
    b = Batch(_to_jobs(jobs))
    b2 = Batch(_to_jobs(other))
    eager = b.count().clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        b.count(s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    log("capturing the batch count pass")
    with torch.cuda.graph(g):
        b.count()
    for rep in range(3):
        b.offsets.zero_()
        b2.count()  # eager work of another batch between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        log(f"replay {rep}")
        assert torch.equal(b.offsets, eager), rep
    total = int(b.offsets[-1].item())
    out = torch.empty((total, 2), dtype=torch.int32, device="cuda")
    b.materialize(out)
    _check_batch(jobs, out, [int(v) for v in b.offsets.cpu().tolist()])


@gpu
def test_write_pass_runs_again_from_one_count():
    """One count, then three write passes from the same workspace: into a buffer one slot too
    small (writes nothing), then twice into full buffers.  The write pass takes units past a
    static head from a ticket counter that its last workgroup resets, so each run covers every
    unit; output positions depend on the plan only, so the two outputs are equal bit for bit."""
    need_gpu()
    from paper_1904_11201_amd.join import Batch
    jobs = _mixed_jobs(66, 20, 400_000)  # units well past twice the write grid
    b = Batch(_to_jobs(jobs))
    offs = b.count()
    total = int(offs[-1].item())
    log(f"batch of {len(jobs)} joins, {total} pairs, written three times")
    small = torch.full((max(total - 1, 0), 2), -7, dtype=torch.int32, device="cuda")
    b.materialize(small)
    outs = []
    for _ in range(2):
        out = torch.full((total, 2), -7, dtype=torch.int32, device="cuda")
        b.materialize(out)
        outs.append(out)
    torch.cuda.synchronize()
    assert bool((small == -7).all())
    assert torch.equal(outs[0], outs[1])
    _check_batch(jobs, outs[1], [int(v) for v in offs.cpu().tolist()])


def _side_jobs(seed: int):
    """Joins that exercise the choice of the hashed table and probes with many matches: S smaller
    than R (S hashed: pairs must still leave as (rid_R, rid_S)), with S keys from a handful of
    values (a hashed side with long runs of one key: walks and tables in canonical order) or
    uniform; R smaller with duplicate keys (3..8 matches per probe); equal sizes (R hashed);
    fan-outs 0 and 1 (claim-counter tables) and larger (marked tables).  R rids are negative and
    S rids positive, so a pair turned the wrong way round cannot match the oracle."""
    g = datagen.rng_for(seed)
    jobs = []
    specs = [  # (nR, nS, S key domain or 0 for |R|, R key domain or 0 for |R|, bits)
        (200_000, 3_000, 7, 0, -1), (150_000, 20_000, 0, 0, 0), (90_000, 40_000, 0, 0, 1),
        (60_000, 59_999, 0, 0, 3), (5_000, 120_000, 0, 1_500, -1), (20_000, 300_000, 0, 4_000, 2),
        (70_000, 70_000, 0, 0, -1), (300_000, 1_000, 3, 0, 4), (2_000, 2_000, 0, 200, 0),
        (100_000, 50_000, 0, 25_000, 1),
    ]
    for nr, ns, sdom, rdom, bits in specs:
        d = rdom or nr
        rk = datagen.uniform_keys(g, nr, 0, d)
        sk = datagen.uniform_keys(g, ns, 0, sdom) if sdom else datagen.uniform_keys(g, ns, 0, d)
        R = datagen.Rel(key=rk, rid=-1 - g.permutation(nr).astype(np.int32))
        S = datagen.Rel(key=sk, rid=g.permutation(ns).astype(np.int32))
        jobs.append((R, S, bits))
    return jobs


@gpu
@pytest.mark.parametrize("det", ["0", "1"])
def test_smaller_side_hashed_and_many_matches(monkeypatch, det):
    need_gpu()
    from paper_1904_11201_amd.join import hash_join_batch
    monkeypatch.setenv("JOIN_HASH_DETERMINISTIC", det)
    jobs = _side_jobs(67)
    log(f"batch of {len(jobs)} joins with S hashed where smaller, deterministic={det}")
    pairs, offs = hash_join_batch(_to_jobs(jobs))
    _check_batch(jobs, pairs, offs)


@gpu
def test_packed_batch_equals_the_list_form(monkeypatch):
    """Batch.packed over slices of one key tensor per side (with empty joins, rid columns and
    per-join fan-outs) gives, in a deterministic plan, exactly the output array of the list form."""
    need_gpu()
    from paper_1904_11201_amd.join import Batch, Job, Relation
    monkeypatch.setenv("JOIN_HASH_DETERMINISTIC", "1")
    jobs = _mixed_jobs(71, 24, 150_000)
    rk = np.concatenate([R.key for R, _, _ in jobs]).astype(np.int32)
    sk = np.concatenate([S.key for _, S, _ in jobs]).astype(np.int32)
    rr = np.concatenate([R.rid if R.rid is not None else np.arange(R.n, dtype=np.int32) for R, _, _ in jobs])
    sr = np.concatenate([S.rid if S.rid is not None else np.arange(S.n, dtype=np.int32) for _, S, _ in jobs])
    roffs = np.concatenate([[0], np.cumsum([R.n for R, _, _ in jobs])])
    soffs = np.concatenate([[0], np.cumsum([S.n for _, S, _ in jobs])])
    bits = [b for _, _, b in jobs]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    drk, dsk, drr, dsr = d(rk), d(sk), d(rr), d(sr)
    log(f"packed batch of {len(jobs)} joins")
    listed = [Job(Relation(drk[roffs[j]:roffs[j + 1]], rid=drr[roffs[j]:roffs[j + 1]]),
                  Relation(dsk[soffs[j]:soffs[j + 1]], rid=dsr[soffs[j]:soffs[j + 1]]), bits[j])
              for j in range(len(jobs))]

    def run(b):
        offs = b.count()
        out = torch.empty((int(offs[-1].item()), 2), dtype=torch.int32, device="cuda")
        b.materialize(out)
        return out, offs.cpu()

    a, oa = run(Batch(listed))
    p, op = run(Batch.packed(drk, roffs, dsk, soffs, bits, rrids=drr, srids=dsr))
    assert torch.equal(oa, op) and torch.equal(a, p)
    full = [(R, S if S.rid is not None else datagen.Rel(key=S.key, rid=np.arange(S.n, dtype=np.int32)), b)
            for R, S, b in jobs]
    _check_batch(full, p, [int(v) for v in op.tolist()])
