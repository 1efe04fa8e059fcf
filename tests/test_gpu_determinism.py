"""Output order is unspecified but fixed for a given input and plan: the same join run twice
gives the same pairs in the same positions, byte for byte (the unsorted output is compared).

Joins on the unpartitioned path are deterministic in every plan.  Partitioned joins (single and
batched) are deterministic in plans with the option hash.deterministic (JOIN_HASH_DETERMINISTIC
= 1): partitioned tuples then land at positions computed from per-tile counts (runs ordered by
tile, then chunk, inside each chunk group's range of a partition; inside a tile each wave places
its tuples from its own counters); by default they land in arrival order, which is faster.  In
the write pass each wave writes from a start recorded by the count pass (no shared cursor), and
the matches of one probe leave in ascending rid order: sorted in registers when there are at
most 8, else met in that order in a table whose duplicated keys were put in canonical order."""
import numpy as np
import pytest
import torch

from paper_1904_11201_amd import datagen
from tests.gpu_util import dev_rel, gpu, log, need_gpu


def _twice(fn):
    a = fn()
    torch.cuda.synchronize()
    b = fn()
    torch.cuda.synchronize()
    return a, b


@gpu
def test_small_equi_join_is_deterministic():
    """The 64K x 64K join (keys in [0, 16384): about four build rows per key)."""
    need_gpu()
    from paper_1904_11201_amd.join import hash_join
    R, S = datagen.small_equi(seed=1)
    dR, dS = dev_rel(R), dev_rel(S)
    log("determinism hash 64K x 64K")
    a, b = _twice(lambda: hash_join(dR, dS))
    assert a.shape == b.shape and torch.equal(a, b)


@gpu
def test_duplicate_heavy_build_is_deterministic():
    """A build side with thousands of copies of a few keys (long bucket walks)."""
    need_gpu()
    from paper_1904_11201_amd.join import hash_join
    g = datagen.rng_for(43)
    keys = g.integers(-1000, 1000, 30).astype(np.int32)
    R = datagen.Rel(key=keys[g.integers(0, 30, 40_000)], rid=g.integers(0, 500, 40_000).astype(np.int32))
    S = datagen.Rel(key=keys[g.integers(0, 30, 3_000)], rid=np.arange(3_000, dtype=np.int32))
    dR, dS = dev_rel(R), dev_rel(S)
    log("determinism hash duplicate-heavy build")
    a, b = _twice(lambda: hash_join(dR, dS))
    assert a.shape == b.shape and torch.equal(a, b)


def _probe_runs_ascending(pairs: np.ndarray, col: int = 1) -> bool:
    """With unique probe rids in column `col`: inside every run of consecutive pairs of one probe
    (the matches one work unit wrote for it), the other column does not decrease."""
    if len(pairs) == 0:
        return True
    other = 1 - col
    same = pairs[1:, col] == pairs[:-1, col]
    return bool(np.all(pairs[1:, other][same] >= pairs[:-1, other][same]))


@gpu
@pytest.mark.parametrize("bits,det", [("-1", "0"), ("0", "0"), ("3", "0"), ("3", "1"), ("9", "1")])
def test_matches_of_a_probe_leave_in_rid_order(monkeypatch, bits, det):
    """Build keys with 1 to 12 entries each (random rids, some repeated), through the single
    path (bits -1) and partitioned plans: probes with up to 8 matches order them as they are
    written, probes with more meet them in a table put in canonical order.  Either way the pairs
    a work unit writes for one probe are ascending in rid_R, and the multiset equals the
    oracle's."""
    need_gpu()
    import oracle
    from tests.gpu_util import canon_gpu
    from paper_1904_11201_amd.join import hash_join
    g = datagen.rng_for(47)
    nkeys = 6000
    keys = g.permutation(1 << 20)[:nkeys].astype(np.int32) - (1 << 19)
    mult = g.integers(1, 13, nkeys)
    bk = np.repeat(keys, mult)
    perm = g.permutation(len(bk))
    R = datagen.Rel(key=bk[perm], rid=g.integers(0, 3 * len(bk), len(bk)).astype(np.int32))
    S = datagen.Rel(key=keys[g.integers(0, nkeys, 200_000)], rid=np.arange(200_000, dtype=np.int32))
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    monkeypatch.setenv("JOIN_HASH_BITS", bits)
    monkeypatch.setenv("JOIN_HASH_DETERMINISTIC", det)
    dR, dS = dev_rel(R), dev_rel(S)
    log(f"probe match order, bits={bits} deterministic={det}")
    a, b = _twice(lambda: hash_join(dR, dS))
    if det == "1" or bits in ("-1", "0"):  # the unpartitioned path is deterministic in any plan
        assert torch.equal(a, b)
    host = a.cpu().numpy()
    assert _probe_runs_ascending(host)
    got = canon_gpu(a)
    assert len(got) == n and np.array_equal(got, ref)


@gpu
@pytest.mark.parametrize("zipf", [False, True])
def test_large_partitioned_join_is_deterministic(monkeypatch, zipf):
    """The 16M x 64M join (2048 partitions), uniform and Zipf probe keys, run twice in a
    deterministic plan."""
    need_gpu()
    monkeypatch.setenv("JOIN_HASH_DETERMINISTIC", "1")
    from paper_1904_11201_amd.join import JOIN_KIND_HASH, hash_join, workspace
    R, S, _ = datagen.large_equi(seed=3 if zipf else 2, zipf=zipf)
    dR, dS = dev_rel(R), dev_rel(S)
    ws = workspace(JOIN_KIND_HASH, R.n, S.n)
    log(f"determinism hash 16M x 64M zipf={zipf}")
    a, b = _twice(lambda: hash_join(dR, dS, ws=ws))
    assert a.shape[0] == S.n and torch.equal(a, b)


@gpu
def test_batch_is_deterministic(monkeypatch):
    """A batch of uneven joins (fan-outs 0 to 11), run twice in a deterministic plan: the same
    output array."""
    need_gpu()
    monkeypatch.setenv("JOIN_HASH_DETERMINISTIC", "1")
    from paper_1904_11201_amd.join import Job, hash_join_batch
    g = datagen.rng_for(49)
    jobs = []
    for j in range(24):
        nr, ns = (int(x) for x in datagen.log_uniform_sizes(g, 2, 1, 400_000))
        rk = datagen.uniform_keys(g, nr, 0, max(nr, 1))
        sk = datagen.uniform_keys(g, ns, 0, max(nr, 1))
        jobs.append(Job(dev_rel(datagen.Rel(key=rk, rid=np.arange(nr, dtype=np.int32))),
                        dev_rel(datagen.Rel(key=sk, rid=np.arange(ns, dtype=np.int32))),
                        -1 if j % 3 else j % 12))
    log("determinism batch of 24 joins")
    (a, oa), (b, ob) = _twice(lambda: hash_join_batch(jobs))
    assert oa == ob and torch.equal(a, b)
