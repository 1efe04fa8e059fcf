"""The ordered scatter (plan option hash.deterministic = 1) against the oracle.

The same partitioned joins as the default (arrival-order) scatter is tested on, bit-exact after
canonical sorting: forced fan-outs up to 2^11, partial tiles and unaligned columns with and
without rid columns, heavy duplicates, a resident build probed by two relations, the pre-filter,
and a batch of uneven joins with forced fan-outs."""
import numpy as np
import pytest
import torch

import oracle
from paper_1904_11201_amd import datagen
from tests.gpu_util import canon_gpu, dev_rel, gpu, log, need_gpu


@pytest.fixture(autouse=True)
def ordered(monkeypatch):
    monkeypatch.setenv("JOIN_HASH_DETERMINISTIC", "1")


def _ref(R, S):
    return oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)


@gpu
@pytest.mark.parametrize("bits", ["1", "5", "8", "11"])
def test_fanouts(monkeypatch, bits):
    need_gpu()
    from paper_1904_11201_amd.join import hash_join
    R, S = datagen.small_random(21, 200_000, 600_000, 0, 150_000, rid_mode="random")
    n, ref = _ref(R, S)
    monkeypatch.setenv("JOIN_HASH_BITS", bits)
    log(f"ordered scatter, bits={bits}")
    got = canon_gpu(hash_join(dev_rel(R), dev_rel(S)))
    assert len(got) == n and np.array_equal(got, ref)


@gpu
@pytest.mark.parametrize("shift,with_rid", [(1, True), (3, False)])
def test_partial_tiles_and_unaligned_columns(monkeypatch, shift, with_rid):
    need_gpu()
    from paper_1904_11201_amd.join import Relation, hash_join

    def d(a):
        if a is None:
            return None
        buf = torch.zeros(len(a) + shift, dtype=torch.int32, device="cuda")
        buf[shift:] = torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
        return buf[shift:]

    monkeypatch.setenv("JOIN_HASH_BITS", "6")
    R, S = datagen.small_random(23, 300_001, 1_234_567, -50_000, 50_000, rid_mode="random")
    rr = R.rid if with_rid else None
    sr = S.rid if with_rid else None
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=rr, Srid=sr)
    log(f"ordered scatter, unaligned by {shift}, rids={with_rid}")
    got = canon_gpu(hash_join(Relation(d(R.key), None, d(rr)), Relation(d(S.key), None, d(sr))))
    assert len(got) == n and np.array_equal(got, ref)


@gpu
def test_heavy_duplicates(monkeypatch):
    need_gpu()
    from paper_1904_11201_amd.join import hash_join
    g = datagen.rng_for(41)
    keys = g.integers(-2**31, 2**31 - 1, 40, dtype=np.int64).astype(np.int32)
    R = datagen.Rel(key=keys[g.integers(0, 40, 50_000)], rid=g.permutation(50_000).astype(np.int32))
    S = datagen.Rel(key=keys[g.integers(0, 40, 10_000)], rid=np.arange(10_000, dtype=np.int32))
    n, ref = _ref(R, S)
    monkeypatch.setenv("JOIN_HASH_BITS", "3")
    log("ordered scatter, heavy duplicates")
    got = canon_gpu(hash_join(dev_rel(R), dev_rel(S)))
    assert len(got) == n and np.array_equal(got, ref)


@gpu
def test_resident_build_and_prefilter():
    need_gpu()
    from paper_1904_11201_amd.join import ResidentBuild, hash_join
    R, S = datagen.small_random(29, 500_000, 2_000_000, 0, 400_000, rid_mode="random")
    _, S2 = datagen.small_random(30, 10, 700_000, 0, 400_000, rid_mode="random")
    dR = dev_rel(R)
    b = ResidentBuild(dR)
    for X in (S, S2):
        n, ref = _ref(R, X)
        log(f"ordered scatter, resident build probed by {X.n}")
        dX = dev_rel(X)
        ws = b.workspace(X.n)
        cnt = b.count(dX, ws)
        out = torch.empty((cnt, 2), dtype=torch.int32, device="cuda")
        b.materialize(dX, ws, out)
        got = canon_gpu(out)
        assert len(got) == n and np.array_equal(got, ref)
    Rp, Sp = datagen.small_random(31, 60_000, 3_000_000, 0, 10_000_000, rid_mode="random")
    n, ref = _ref(Rp, Sp)
    log("ordered scatter, pre-filter")
    got = canon_gpu(hash_join(dev_rel(Rp), dev_rel(Sp), prefilter=True))
    assert len(got) == n and np.array_equal(got, ref)


@gpu
def test_batch_with_forced_fanouts():
    need_gpu()
    from paper_1904_11201_amd.join import Job, hash_join_batch
    g = datagen.rng_for(37)
    host, jobs = [], []
    for j in range(20):
        nr, ns = (int(x) for x in datagen.log_uniform_sizes(g, 2, 1, 300_000))
        d = max(nr, 1)
        R = datagen.Rel(key=datagen.uniform_keys(g, nr, 0, d), rid=g.permutation(nr).astype(np.int32))
        S = datagen.Rel(key=datagen.uniform_keys(g, ns, 0, d), rid=np.arange(ns, dtype=np.int32))
        host.append((R, S))
        jobs.append(Job(dev_rel(R), dev_rel(S), -1 if j % 4 else j % 12))
    log("ordered scatter, batch of 20 joins")
    pairs, offs = hash_join_batch(jobs)
    for j, (R, S) in enumerate(host):
        n, ref = _ref(R, S)
        got = canon_gpu(pairs[offs[j]:offs[j + 1]])
        assert offs[j + 1] - offs[j] == n and np.array_equal(got, ref), j
