"""Theta join (tiled nested loop, count -> scan -> write) on the GPU vs the CPU oracle.

Bit-exact after canonical sorting.  Sizes span several work units and ragged tails (|R| not a
multiple of 512 rows per wave, |S| not a multiple of the 8-row scalar group)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1904_11201_amd import datagen
from tests.gpu_util import canon_gpu, dev_rel, gpu, log, need_gpu

I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1
OPS_A = ["eq", "ne", "lt", "le", "gt", "ge", "band"]
OPS_C = ["none", "eq", "ne", "lt", "le", "gt", "ge"]


def _theta(R, S, op_a, w=0, op_c="none"):
    from paper_1904_11201_amd.join import Pred, theta_join
    return theta_join(dev_rel(R), dev_rel(S), Pred(op_a, w, op_c))


def _oracle(R, S, op_a, w=0, op_c="none"):
    return oracle.theta_nlj(R.key, S.key, op_a, w=w, Rc=R.key2, Sc=S.key2, op_c=op_c,
                            Rrid=R.rid, Srid=S.rid)


@gpu
@pytest.mark.parametrize("op_a", OPS_A)
def test_every_operator_pair(op_a):
    need_gpu()
    R, S = datagen.small_random(100 + OPS_A.index(op_a), 1100, 1037, -40, 40, with_c=True,
                                rid_mode="random")
    for op_c in OPS_C:
        w = 3 if op_a == "band" else 0
        log(f"theta {op_a}/{op_c} 1100x1037")
        n, ref = _oracle(R, S, op_a, w, op_c)
        got = canon_gpu(_theta(R, S, op_a, w, op_c))
        assert len(got) == n, (op_a, op_c)
        assert np.array_equal(got, ref), (op_a, op_c)


@gpu
def test_band_extremes_and_wide_bands():
    """|R.a - S.a| <= w over the whole int32 range: no wrap-around false positives."""
    need_gpu()
    R, S = datagen.small_random(7, 700, 650, I32_MIN, I32_MAX)
    R.key[:64] = I32_MIN
    R.key[64:128] = I32_MAX
    S.key[:50] = I32_MAX
    S.key[50:90] = I32_MIN
    S.key[90:100] = 0
    for w in (0, 1, 12345, 1 << 30, I32_MAX):
        log(f"band extremes w={w}")
        n, ref = _oracle(R, S, "band", w)
        got = canon_gpu(_theta(R, S, "band", w))
        assert len(got) == n and np.array_equal(got, ref), w


@gpu
def test_band_lt_reduced_c3a_shape():
    """The band + inequality workload's distributions at 64K x 64K (several units per side)."""
    need_gpu()
    R, S = datagen.band_theta(seed=4, n=1 << 16)
    log("band_theta 64K x 64K w=8 c<")
    n, ref = oracle.band_window(R.key, S.key, 8, Rc=R.key2, Sc=S.key2, op_c="lt", Rrid=R.rid,
                                Srid=S.rid)
    got = canon_gpu(_theta(R, S, "band", 8, "lt"))
    assert len(got) == n and np.array_equal(got, ref)


@gpu
def test_band_lt_full_c3a():
    """1M x 1M, |R.a-S.a| <= 8 and R.c < S.c: all ~557K pairs against the sorted-window oracle
    (itself pinned against the brute-force definition)."""
    need_gpu()
    R, S = datagen.band_theta(seed=4, n=1 << 20)
    log("band_theta 1M x 1M w=8 c< (full)")
    n, ref = oracle.band_window(R.key, S.key, 8, Rc=R.key2, Sc=S.key2, op_c="lt", Rrid=R.rid,
                                Srid=S.rid)
    got = canon_gpu(_theta(R, S, "band", 8, "lt"))
    assert len(got) == n and np.array_equal(got, ref)
    # a sampled exact check against the brute-force definition itself
    rows = np.random.default_rng(0).choice(R.n, 256, replace=False)
    sub = datagen.Rel(key=R.key[rows], key2=R.key2[rows], rid=R.rid[rows])
    n2, ref2 = oracle.theta_nlj(sub.key, S.key, "band", w=8, Rc=sub.key2, Sc=S.key2, op_c="lt",
                                Rrid=sub.rid, Srid=S.rid)
    mask = np.isin(got[:, 0], rows)
    assert np.array_equal(got[mask], ref2)


@gpu
def test_lt_count_full_c3b():
    """64K x 64K R.a < S.a, count only: exact count against the closed form (uint64)."""
    need_gpu()
    from paper_1904_11201_amd.join import JOIN_KIND_THETA, Pred, join_count, workspace
    R, S = datagen.lt_theta(seed=5, n=1 << 16)
    log("lt_theta 64K x 64K count")
    p = Pred("lt")
    ws = workspace(JOIN_KIND_THETA, R.n, S.n, p)
    got = join_count(JOIN_KIND_THETA, dev_rel(R), dev_rel(S), p, ws)
    assert got == oracle.count_lt(R.key, S.key)
    assert got == oracle.theta_nlj(R.key, S.key, "lt", want_pairs=False)[0]


@gpu
def test_count_beyond_int32():
    """A count above 2^32 (all pairs of 70K x 70K match) stays exact in uint64."""
    need_gpu()
    from paper_1904_11201_amd.join import JOIN_KIND_THETA, Pred, join_count, workspace
    n = 70000
    R = datagen.Rel(key=np.zeros(n, np.int32))
    S = datagen.Rel(key=np.ones(n, np.int32))
    p = Pred("lt")
    ws = workspace(JOIN_KIND_THETA, n, n, p)
    got = join_count(JOIN_KIND_THETA, dev_rel(R, False), dev_rel(S, False), p, ws)
    assert got == n * n and got > (1 << 32)


@gpu
@pytest.mark.parametrize("nR,nS", [(1, 1), (1, 9), (513, 7), (64, 8), (511, 4099), (2000, 1)])
def test_ragged_and_tiny(nR, nS):
    need_gpu()
    R, S = datagen.small_random(nR * 7 + nS, nR, nS, -5, 5, with_c=True, rid_mode="none")
    for op_a, op_c in (("lt", "none"), ("band", "ge"), ("eq", "ne")):
        n, ref = _oracle(R, S, op_a, 2, op_c)
        from paper_1904_11201_amd.join import Pred, theta_join
        got = canon_gpu(theta_join(dev_rel(R, False), dev_rel(S, False), Pred(op_a, 2, op_c)))
        assert len(got) == n and np.array_equal(got, ref), (nR, nS, op_a, op_c)


@gpu
def test_tile_shapes_do_not_change_results(monkeypatch):
    need_gpu()
    R, S = datagen.small_random(55, 3000, 5000, -100, 100, with_c=True)
    n, ref = _oracle(R, S, "band", 4, "lt")
    for ts in ("8", "64", "1000", "100000"):
        monkeypatch.setenv("JOIN_THETA_TS", ts)
        got = canon_gpu(_theta(R, S, "band", 4, "lt"))
        assert len(got) == n and np.array_equal(got, ref), ts


@gpu
def test_theta_output_is_deterministic():
    need_gpu()
    from paper_1904_11201_amd.join import Pred, theta_join
    R, S = datagen.small_random(66, 4000, 3000, -30, 30)
    a = theta_join(dev_rel(R), dev_rel(S), Pred("lt"))
    b = theta_join(dev_rel(R), dev_rel(S), Pred("lt"))
    assert torch.equal(a, b)
