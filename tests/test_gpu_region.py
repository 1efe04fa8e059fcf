"""Theta join with region pruning (JOIN_KIND_THETA_REGION) on the GPU vs the CPU oracle.

Same bar as the plain nested loop: bit-exact after canonical sorting.  The cases stress the
classification: every operator, ties at bucket edges, single-value buckets (all-duplicate keys,
where EQ / NE regions are green or white as a whole), the INT32 extremes, wide bands whose
regions are entirely green, and ragged sizes."""
import numpy as np
import pytest
import torch

import oracle
from paper_1904_11201_amd import datagen
from tests.gpu_util import canon_gpu, dev_rel, gpu, log, need_gpu

I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1
OPS_A = ["eq", "ne", "lt", "le", "gt", "ge", "band"]


def _region(R, S, op_a, w=0, op_c="none", with_rid=True):
    from paper_1904_11201_amd.join import Pred, theta_join
    return theta_join(dev_rel(R, with_rid), dev_rel(S, with_rid), Pred(op_a, w, op_c), region=True)


def _oracle(R, S, op_a, w=0, op_c="none", with_rid=True):
    return oracle.theta_nlj(R.key, S.key, op_a, w=w, Rc=R.key2, Sc=S.key2, op_c=op_c,
                            Rrid=R.rid if with_rid else None, Srid=S.rid if with_rid else None)


@gpu
@pytest.mark.parametrize("op_a", OPS_A)
@pytest.mark.parametrize("op_c", ["none", "lt", "ne"])
def test_region_every_operator(op_a, op_c):
    need_gpu()
    R, S = datagen.small_random(300 + OPS_A.index(op_a), 3100, 2900, -3000, 3000, with_c=True,
                                rid_mode="random")
    w = 25 if op_a == "band" else 0
    log(f"region {op_a}/{op_c}")
    n, ref = _oracle(R, S, op_a, w, op_c)
    got = canon_gpu(_region(R, S, op_a, w, op_c))
    assert len(got) == n and np.array_equal(got, ref), (op_a, op_c)


@gpu
@pytest.mark.parametrize("op_a", OPS_A)
def test_region_duplicates_and_ties(op_a):
    """Few distinct values: buckets hold one value each, so EQ/NE regions are green/white as a
    whole and LT/LE/GT/GE regions tie at every bucket edge."""
    need_gpu()
    R, S = datagen.small_random(400 + OPS_A.index(op_a), 2000, 2500, 0, 6)
    n, ref = _oracle(R, S, op_a, 1 if op_a == "band" else 0)
    got = canon_gpu(_region(R, S, op_a, 1 if op_a == "band" else 0))
    assert len(got) == n and np.array_equal(got, ref), op_a


@gpu
@pytest.mark.parametrize("w", [0, 1, 1000, 1 << 30, I32_MAX])
def test_region_band_extremes(w):
    need_gpu()
    R, S = datagen.small_random(7, 900, 800, I32_MIN, I32_MAX)
    R.key[:64] = I32_MIN
    R.key[64:128] = I32_MAX
    S.key[:50] = I32_MAX
    S.key[50:90] = I32_MIN
    log(f"region band extremes w={w}")
    n, ref = _oracle(R, S, "band", w)
    got = canon_gpu(_region(R, S, "band", w))
    assert len(got) == n and np.array_equal(got, ref), w


@gpu
def test_region_band_lt_full_c3a():
    need_gpu()
    R, S = datagen.band_theta(seed=4, n=1 << 20)
    log("region band_theta 1M x 1M w=8 c<")
    n, ref = oracle.band_window(R.key, S.key, 8, Rc=R.key2, Sc=S.key2, op_c="lt", Rrid=R.rid,
                                Srid=S.rid)
    got = canon_gpu(_region(R, S, "band", 8, "lt"))
    assert len(got) == n and np.array_equal(got, ref)


@gpu
def test_region_lt_count_c3b():
    need_gpu()
    from paper_1904_11201_amd.join import JOIN_KIND_THETA_REGION, Pred, join_count, workspace
    R, S = datagen.lt_theta(seed=5, n=1 << 16)
    p = Pred("lt")
    ws = workspace(JOIN_KIND_THETA_REGION, R.n, S.n, p)
    got = join_count(JOIN_KIND_THETA_REGION, dev_rel(R), dev_rel(S), p, ws)
    assert got == oracle.count_lt(R.key, S.key)


@gpu
def test_region_lt_pairs_with_green_cross_products():
    """R.a < S.a materialised: most pairs come from green regions written as cross products."""
    need_gpu()
    R, S = datagen.small_random(17, 6000, 5000, -100000, 100000, rid_mode="random")
    n, ref = _oracle(R, S, "lt")
    got = canon_gpu(_region(R, S, "lt"))
    assert len(got) == n and np.array_equal(got, ref)


@gpu
@pytest.mark.parametrize("nR,nS", [(1, 1), (1, 700), (700, 1), (513, 9), (5000, 3)])
def test_region_ragged(nR, nS):
    need_gpu()
    R, S = datagen.small_random(nR * 3 + nS, nR, nS, -50, 50, with_c=True, rid_mode="none")
    for op_a, op_c in (("lt", "none"), ("band", "ge"), ("ne", "none"), ("eq", "lt")):
        n, ref = _oracle(R, S, op_a, 3, op_c, with_rid=False)
        got = canon_gpu(_region(R, S, op_a, 3, op_c, with_rid=False))
        assert len(got) == n and np.array_equal(got, ref), (nR, nS, op_a, op_c)


@gpu
def test_region_equals_nested_loop_kind():
    need_gpu()
    from paper_1904_11201_amd.join import Pred, theta_join
    R, S = datagen.band_theta(seed=9, n=50_000, hi=1 << 16)
    a = canon_gpu(theta_join(dev_rel(R), dev_rel(S), Pred("band", 3, "gt")))
    b = canon_gpu(theta_join(dev_rel(R), dev_rel(S), Pred("band", 3, "gt"), region=True))
    assert np.array_equal(a, b)
