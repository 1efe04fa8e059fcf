"""Hash equi join (partition -> LDS table count -> scan -> write) on the GPU vs the CPU oracle.

Bit-exact after canonical sorting.  Covers the single-partition path and the partitioned path,
forced fan-outs and forced R-chunking (the LDS-overflow path), skew, duplicates, extreme keys,
payload rids, and the full 16M x 64M workload against its closed form."""
import numpy as np
import pytest
import torch

import oracle
from paper_1904_11201_amd import datagen
from tests.gpu_util import canon_gpu, canon_np, dev_rel, gpu, log, need_gpu

I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1


def _hash(R, S, with_rid=True):
    from paper_1904_11201_amd.join import hash_join
    return hash_join(dev_rel(R, with_rid), dev_rel(S, with_rid))


def _check(R, S, with_rid=True, label=""):
    log(f"hash {label} {R.n}x{S.n}")
    rr = R.rid if with_rid else None
    sr = S.rid if with_rid else None
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=rr, Srid=sr)
    got = canon_gpu(_hash(R, S, with_rid))
    assert len(got) == n, label
    assert np.array_equal(got, ref), label


@gpu
def test_small_equi_c1_full():
    """65,536 x 65,536 keys uniform in [0, 16384): against the brute-force definition."""
    need_gpu()
    R, S = datagen.small_equi(seed=1)
    log("hash C1 64Kx64K")
    n, ref = oracle.equi_nlj(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    got = canon_gpu(_hash(R, S))
    assert len(got) == n and np.array_equal(got, ref)
    assert n == oracle.count_equi(R.key, S.key)


@gpu
@pytest.mark.parametrize("nR,nS", [(1, 1), (1, 1000), (1000, 1), (63, 65), (4097, 333),
                                   (9216, 9217), (30001, 70003)])
def test_ragged_sizes(nR, nS):
    need_gpu()
    R, S = datagen.small_random(nR + 3 * nS, nR, nS, -50, 50, rid_mode="random")
    _check(R, S, label="ragged")


@gpu
def test_rid_none_means_position():
    need_gpu()
    R, S = datagen.small_random(5, 5000, 7000, 0, 100, rid_mode="none")
    _check(R, S, with_rid=False, label="rid=None")


@gpu
def test_extreme_and_negative_keys():
    need_gpu()
    R, S = datagen.small_random(9, 20000, 30000, I32_MIN, I32_MAX, rid_mode="random")
    specials = np.array([I32_MIN, I32_MAX, -1, 0, 1, I32_MIN + 1, I32_MAX - 1], np.int32)
    R.key[: 7 * 50] = np.repeat(specials, 50)
    S.key[: 7 * 40] = np.repeat(specials, 40)
    # also tuples equal to the table's candidate empty markers' bit patterns
    R.key[400:410] = -1
    R.rid[400:410] = -1
    _check(R, S, label="extremes")


@gpu
def test_duplicate_heavy_build_side():
    """Bag semantics: every R duplicate pairs with every matching S tuple."""
    need_gpu()
    g = np.random.default_rng(3)
    R = datagen.Rel(key=np.full(3000, 42, np.int32), rid=np.arange(3000, dtype=np.int32))
    S = datagen.Rel(key=g.choice(np.array([41, 42, 43], np.int32), 2500),
                    rid=np.arange(2500, dtype=np.int32))
    _check(R, S, label="all-equal build keys")


@gpu
def test_partitioned_path_and_fanouts(monkeypatch):
    """The same join through the single-partition path and several forced fan-outs."""
    need_gpu()
    R, S = datagen.small_random(21, 200_000, 600_000, 0, 150_000, rid_mode="random")
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    for bits in ("0", "1", "5", "8", "11"):
        monkeypatch.setenv("JOIN_HASH_BITS", bits)
        log(f"hash fan-out bits={bits}")
        got = canon_gpu(_hash(R, S))
        assert len(got) == n and np.array_equal(got, ref), bits


def _offset_rel(rel, shift, with_rid=True):
    """The relation's columns as device views starting `shift` int32 past a buffer's start, so
    that they are not 16-byte aligned."""
    from paper_1904_11201_amd.join import Relation

    def d(a):
        if a is None:
            return None
        buf = torch.zeros(len(a) + shift, dtype=torch.int32, device="cuda")
        buf[shift:] = torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
        return buf[shift:]

    return Relation(d(rel.key), None, d(rel.rid) if with_rid else None)


@gpu
@pytest.mark.parametrize("kshift,with_rid", [(1, True), (0, True), (3, False), (2, True)])
def test_unaligned_columns_and_partial_tiles(monkeypatch, kshift, with_rid):
    """Columns that start off a 16-byte boundary take the element-by-element loads of the
    histogram and scatter; sizes that are not a whole number of scatter tiles take the partial
    tile path; both at a large and a small fan-out."""
    from paper_1904_11201_amd.join import hash_join
    need_gpu()
    R, S = datagen.small_random(23 + kshift, 70_001, 4 * 16384 * 3 + 4097, 0, 60_000, rid_mode="random")
    rr = R.rid if with_rid else None
    sr = S.rid if with_rid else None
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=rr, Srid=sr)
    for bits in ("11", "3"):
        monkeypatch.setenv("JOIN_HASH_BITS", bits)
        log(f"hash offset views shift={kshift} rid={with_rid} bits={bits}")
        got = canon_gpu(hash_join(_offset_rel(R, kshift, with_rid), _offset_rel(S, kshift, with_rid)))
        assert len(got) == n and np.array_equal(got, ref), (kshift, bits)


@gpu
@pytest.mark.parametrize("with_rid", [False, True])
def test_full_scatter_tiles_with_and_without_rids(with_rid):
    """Sides large enough for whole scatter tiles in every chunk (and a partial tile after
    them), with rid columns and with row positions."""
    from paper_1904_11201_amd.join import hash_join
    need_gpu()
    R, S = datagen.small_random(29, 1_200_001, 5_000_003, 0, 1_000_000,
                                rid_mode="random" if with_rid else "none")
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    log(f"hash 1.2M x 5M rid={with_rid}")
    got = canon_gpu(hash_join(dev_rel(R, with_rid), dev_rel(S, with_rid)))
    assert len(got) == n and np.array_equal(got, ref)


@gpu
def test_partitioned_heavy_duplicates(monkeypatch):
    """A few build keys with about a thousand copies each, through partitioned plans: long chains
    of overflowed buckets in the tables of fan-out 2 and more (marked tables) and of fan-out 1
    (claim counters)."""
    need_gpu()
    g = datagen.rng_for(41)
    keys = g.integers(-2**31, 2**31 - 1, 40, dtype=np.int64).astype(np.int32)
    R = datagen.Rel(key=keys[g.integers(0, 40, 50_000)], rid=g.permutation(50_000).astype(np.int32))
    S = datagen.Rel(key=np.concatenate([keys[g.integers(0, 40, 8_000)],
                                        g.integers(-2**31, 2**31 - 1, 2_000, dtype=np.int64).astype(np.int32)]),
                    rid=np.arange(10_000, dtype=np.int32))
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    for bits in ("1", "2", "3", "6"):
        monkeypatch.setenv("JOIN_HASH_BITS", bits)
        log(f"hash heavy duplicates bits={bits}")
        got = canon_gpu(_hash(R, S))
        assert len(got) == n and np.array_equal(got, ref), bits


@gpu
def test_lds_overflow_chunked_build(monkeypatch):
    """A small table capacity forces several R chunks per partition (each probed by all of the
    partition's S tuples), in both the single and the partitioned path."""
    need_gpu()
    R, S = datagen.small_random(22, 50_000, 80_000, 0, 20_000, rid_mode="random")
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    for cap, bits in (("256", "0"), ("256", "4"), ("1000", "2")):
        monkeypatch.setenv("JOIN_HASH_CAP", cap)
        monkeypatch.setenv("JOIN_HASH_BITS", bits)
        log(f"hash cap={cap} bits={bits}")
        got = canon_gpu(_hash(R, S))
        assert len(got) == n and np.array_equal(got, ref), (cap, bits)


@gpu
def test_many_units_scan_kernels(monkeypatch):
    """Over 8192 work units (64-entry tables at fan-out 8: about 9400 R chunks): the unit counts
    go through the separate scan kernels instead of the count kernel's last workgroup."""
    need_gpu()
    R, S = datagen.small_random(23, 600_000, 800_000, 0, 300_000, rid_mode="random")
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    monkeypatch.setenv("JOIN_HASH_CAP", "64")
    monkeypatch.setenv("JOIN_HASH_BITS", "8")
    log("hash many units cap=64 bits=8")
    got = canon_gpu(_hash(R, S))
    assert len(got) == n and np.array_equal(got, ref)


@gpu
def test_skewed_build_and_probe():
    """Zipf keys on both sides: hot partitions are split into many S slices."""
    need_gpu()
    g = datagen.rng_for(31)
    rk = datagen.zipf_ranks(g, 300_000, 1_000_000).astype(np.int32)
    sk = datagen.zipf_ranks(g, 400_000, 1_000_000).astype(np.int32)
    R = datagen.Rel(key=rk, rid=np.arange(len(rk), dtype=np.int32))
    S = datagen.Rel(key=sk, rid=np.arange(len(sk), dtype=np.int32))
    # Zipf on both sides has a huge hot-key product: count only, plus a sampled exact check.
    from paper_1904_11201_amd.join import JOIN_KIND_HASH, join_count, workspace
    ws = workspace(JOIN_KIND_HASH, R.n, S.n)
    log("hash zipf both sides count")
    got = join_count(JOIN_KIND_HASH, dev_rel(R), dev_rel(S), None, ws)
    assert got == oracle.count_equi(R.key, S.key)
    keep = R.key > 50  # drop the hottest keys so the pairs fit
    R2 = datagen.Rel(key=R.key[keep], rid=R.rid[keep])
    _check(R2, S, label="zipf tail")


def _closed_form_check(zipf: bool):
    R, S, perm = datagen.large_equi(seed=3 if zipf else 2, zipf=zipf)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm), dtype=np.int32)
    log(f"hash 16M x 64M zipf={zipf}")
    pairs = _hash(R, S)
    assert pairs.shape[0] == S.n
    # each S tuple matches exactly one R tuple: order by rid_S and compare rid_R column
    order = torch.sort(pairs[:, 1]).indices
    srt = pairs[order].cpu().numpy()
    assert np.array_equal(srt[:, 1], np.arange(S.n, dtype=np.int32))
    assert np.array_equal(srt[:, 0], inv[S.key])


@gpu
def test_large_equi_uniform_full_closed_form():
    need_gpu()
    _closed_form_check(False)


@gpu
def test_large_equi_zipf_full_closed_form():
    need_gpu()
    _closed_form_check(True)


@gpu
def test_band_zero_theta_equals_hash_join():
    """Two independent GPU paths: |R.a - S.a| <= 0 through the theta kernels and R.a = S.a
    through the hash kernels give the same pairs."""
    need_gpu()
    from paper_1904_11201_amd.join import Pred, theta_join
    R, S = datagen.small_random(77, 20000, 25000, 0, 5000, rid_mode="random")
    a = canon_gpu(_hash(R, S))
    b = canon_gpu(theta_join(dev_rel(R), dev_rel(S), Pred("band", 0)))
    assert np.array_equal(a, b)
    assert len(a) == oracle.count_equi(R.key, S.key)
