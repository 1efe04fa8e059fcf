"""Pre-filtered equi join (JOIN_KIND_HASH_PREFILTER): the same pairs as the plain hash join and
the oracle, from few to all keys matching, with empty survivors on one side, duplicates and rid
payloads."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1904_11201_amd import datagen
from tests.gpu_util import canon_gpu, dev_rel, gpu, log, need_gpu


def _check(R, S, label):
    from paper_1904_11201_amd.join import hash_join
    dR, dS = dev_rel(R), dev_rel(S)
    log(f"prefilter {label}: {R.n} x {S.n}")
    got = canon_gpu(hash_join(dR, dS, prefilter=True))
    rr = R.rid if R.rid is not None else np.arange(R.n, dtype=np.int32)
    sr = S.rid if S.rid is not None else np.arange(S.n, dtype=np.int32)
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=rr, Srid=sr)
    assert len(got) == n and np.array_equal(got, ref), label
    assert np.array_equal(got, canon_gpu(hash_join(dR, dS)))


@gpu
def test_few_and_all_keys_matching():
    need_gpu()
    g = datagen.rng_for(81)
    R = datagen.Rel(key=datagen.uniform_keys(g, 200_000, 0, 1_000_000),
                    rid=g.permutation(200_000).astype(np.int32))
    S = datagen.Rel(key=datagen.uniform_keys(g, 600_000, 0, 50_000_000))
    _check(R, S, "about 0.4% of probes match")
    R, S = datagen.small_equi(seed=1)
    _check(R, S, "every key shared")
    R = datagen.Rel(key=datagen.uniform_keys(g, 50_000, 0, 5_000_000))
    S = datagen.Rel(key=datagen.uniform_keys(g, 2_500_000, 0, 50_000_000))
    _check(R, S, "large probe side: the count pass records the semi-join")


@gpu
def test_no_survivors_on_one_side_and_empty_inputs():
    need_gpu()
    g = datagen.rng_for(82)
    R = datagen.Rel(key=np.arange(0, 3000, dtype=np.int32))
    S = datagen.Rel(key=datagen.uniform_keys(g, 5000, 1 << 30, (1 << 30) + 100_000))
    _check(R, S, "disjoint key ranges")
    _check(datagen.Rel(key=np.zeros(0, np.int32)), S, "empty R")
    _check(R, datagen.Rel(key=np.zeros(0, np.int32)), "empty S")


@gpu
def test_duplicates_and_extreme_keys():
    need_gpu()
    g = datagen.rng_for(83)
    ext = np.array([-2**31, 2**31 - 1, 0, -1], np.int32)
    rk = np.concatenate([g.choice(ext, 2000), datagen.uniform_keys(g, 30_000, -500, 500)])
    sk = np.concatenate([g.choice(ext, 3000), datagen.uniform_keys(g, 40_000, 0, 100_000)])
    R = datagen.Rel(key=rk.astype(np.int32), rid=g.integers(-2**31, 2**31 - 1, len(rk), dtype=np.int64).astype(np.int32))
    S = datagen.Rel(key=sk.astype(np.int32))
    _check(R, S, "duplicates and int32 extremes")


@gpu
def test_semi_join_with_longer_probe_slices():
    """A probe side past 32K rows per count workgroup (1M x 20M, 1% matching): the semi-join plan
    cuts it into longer slices; the oracle's pairs and the plain join's."""
    need_gpu()
    g = datagen.rng_for(85)
    R = datagen.Rel(key=np.arange(0, 100_000_000, 100, dtype=np.int32), rid=None)
    S = datagen.Rel(key=datagen.uniform_keys(g, 20_000_000, 0, 100_000_000), rid=None)
    _check(R, S, "semi-join, 1M x 20M, longer slices")


@gpu
def test_full_stages_semi_join_and_the_ordered_compaction(monkeypatch):
    """Every build row passes S's filter (more passing rows per workgroup than its LDS stage
    holds, so waves write straight out); a probe side too large for a filter (the count pass
    records the semi-join, the write pass visits only matching rows), all and 1% matching; then,
    with the deterministic option, the ordered compaction and the semi-join give the same output
    array on two runs, and the oracle's pairs."""
    need_gpu()
    import torch
    from paper_1904_11201_amd.join import hash_join
    g = datagen.rng_for(84)
    R1 = datagen.Rel(key=datagen.uniform_keys(g, 24_000_000, 0, 100_000), rid=None)
    S1 = datagen.Rel(key=np.arange(100_000, dtype=np.int32), rid=g.permutation(100_000).astype(np.int32))
    _check(R1, S1, "all of 24M build rows pass")
    R2 = datagen.Rel(key=np.arange(100_000, dtype=np.int32), rid=g.permutation(100_000).astype(np.int32))
    S2 = datagen.Rel(key=datagen.uniform_keys(g, 6_000_000, 0, 100_000), rid=None)
    _check(R2, S2, "semi-join, every probe row matches")
    R3 = datagen.Rel(key=np.arange(0, 10_000_000, 100, dtype=np.int32), rid=None)
    S3 = datagen.Rel(key=datagen.uniform_keys(g, 5_000_000, 0, 10_000_000), rid=g.permutation(5_000_000).astype(np.int32))
    _check(R3, S3, "semi-join, 1% of probe rows match")
    hot = np.concatenate([np.full(40_000, 777, np.int32), datagen.uniform_keys(g, 200_000, 0, 10_000_000)])
    R5 = datagen.Rel(key=g.permutation(hot).astype(np.int32), rid=g.permutation(len(hot)).astype(np.int32))
    S5 = datagen.Rel(key=np.concatenate([np.full(50, 777, np.int32),
                                         datagen.uniform_keys(g, 3_000_000, 0, 10_000_000)]).astype(np.int32), rid=None)
    _check(R5, S5, "semi-join, a build partition of several chunks (its units share their S slice)")
    S4 = datagen.Rel(key=datagen.uniform_keys(g, 1_500_000, 0, 10_000_000), rid=None)
    monkeypatch.setenv("JOIN_HASH_DETERMINISTIC", "1")
    for X, Y, label in ((R1, S1, "filtered build side, ordered"), (R3, S3, "semi-join, ordered"),
                        (R3, S4, "filtered probe side, ordered")):
        _check(X, Y, label)
        dX, dY = dev_rel(X), dev_rel(Y)
        a = hash_join(dX, dY, prefilter=True)
        b = hash_join(dX, dY, prefilter=True)
        torch.cuda.synchronize()
        assert a.shape == b.shape and torch.equal(a, b), label
