"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each pin is independent of the oracle's own code: hand-derived worked examples
(tests/golden/*.json, each with its citation and derivation), library routines (pandas.merge,
numpy.searchsorted, collections.Counter), closed forms, and invariants of the join definitions
of Section 2.3 (trichotomy, mirror symmetry, band w=0 == equality, monotonicity in w,
conjunction == intersection, permutation invariance, empty inputs) and the result-size bound of
Section 3.3.3 (equation rsize).  A dropped term, a wrong sign or comparison, a transposed operand
or a wrap-around in the band arithmetic each fails at least one of them.
"""
import collections
import json
import os

import numpy as np
import pandas as pd
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_1904_11201_amd import datagen

GOLD = os.path.join(os.path.dirname(__file__), "golden")
I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _col(d, k):
    return None if k not in d else np.array(d[k], dtype=np.int64).astype(np.int32)


def _pairs_set(p):
    return collections.Counter(map(tuple, np.asarray(p).tolist()))


# ---------------------------------------------------------------- worked examples (golden) --

def test_golden_equi_duplicates():
    g = _load("equi_duplicates.json")
    exp = np.array(g["expected"], dtype=np.int32)
    for fn in (oracle.equi_nlj, oracle.equi_sortmerge):
        n, p = fn(_col(g["R"], "a"), _col(g["S"], "a"))
        assert n == len(exp)
        assert np.array_equal(p, exp)
    assert oracle.count_equi(_col(g["R"], "a"), _col(g["S"], "a")) == len(exp)


def test_golden_theta_ops():
    g = _load("theta_ops.json")
    for op, exp in g["cases"].items():
        n, p = oracle.theta_nlj(_col(g["R"], "a"), _col(g["S"], "a"), op)
        assert n == len(exp), op
        assert np.array_equal(p, np.array(exp, dtype=np.int32).reshape(-1, 2)), op
    assert oracle.count_lt(_col(g["R"], "a"), _col(g["S"], "a")) == len(g["cases"]["lt"])


def test_golden_band_extremes():
    g = _load("band_extremes.json")
    for w, exp in g["cases"].items():
        exp = np.array(exp, dtype=np.int32)
        n, p = oracle.theta_nlj(_col(g["R"], "a"), _col(g["S"], "a"), "band", w=int(w))
        assert n == len(exp) and np.array_equal(p, exp), w
        n2, p2 = oracle.band_window(_col(g["R"], "a"), _col(g["S"], "a"), int(w))
        assert n2 == len(exp) and np.array_equal(p2, exp), w


def test_golden_band_and_lt_with_payload():
    g = _load("band_and_lt_payload.json")
    R, S, pr = g["R"], g["S"], g["pred"]
    exp = np.array(g["expected"], dtype=np.int32)
    n, p = oracle.theta_nlj(_col(R, "a"), _col(S, "a"), pr["op_a"], w=pr["w"], Rc=_col(R, "c"),
                            Sc=_col(S, "c"), op_c=pr["op_c"], Rrid=_col(R, "rid"),
                            Srid=_col(S, "rid"))
    assert n == 1 and np.array_equal(p, exp)
    n2, p2 = oracle.band_window(_col(R, "a"), _col(S, "a"), pr["w"], Rc=_col(R, "c"),
                                Sc=_col(S, "c"), op_c="lt", Rrid=_col(R, "rid"),
                                Srid=_col(S, "rid"))
    assert n2 == 1 and np.array_equal(p2, exp)


# ------------------------------------------------------------ library routines / closed forms --

small_keys = st.lists(st.integers(-6, 6), min_size=0, max_size=40)


@settings(max_examples=60, deadline=None)
@given(small_keys, small_keys)
def test_equi_count_is_sum_of_multiplicity_products(rk, sk):
    """count(EQ) = sum_k |R_k| * |S_k| (collections.Counter, not the oracle's sort)."""
    cr, cs = collections.Counter(rk), collections.Counter(sk)
    expect = sum(cr[k] * cs[k] for k in cr)
    rk, sk = np.array(rk, dtype=np.int32), np.array(sk, dtype=np.int32)
    assert oracle.equi_nlj(rk, sk, want_pairs=False)[0] == expect
    assert oracle.equi_sortmerge(rk, sk, want_pairs=False)[0] == expect
    assert oracle.count_equi(rk, sk) == expect


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_equi_pairs_equal_pandas_merge(seed):
    R, S = datagen.small_random(seed, 700, 900, -50, 50, rid_mode="random")
    dr = pd.DataFrame({"k": R.key, "r": R.rid})
    ds = pd.DataFrame({"k": S.key, "s": S.rid})
    m = dr.merge(ds, on="k", how="inner")
    ref = np.stack([m["r"].to_numpy(np.int32), m["s"].to_numpy(np.int32)], axis=1)
    ref = ref[np.lexsort((ref[:, 1], ref[:, 0]))]
    for fn in (oracle.equi_nlj, oracle.equi_sortmerge):
        n, p = fn(R.key, S.key, Rrid=R.rid, Srid=S.rid)
        assert n == len(ref)
        assert np.array_equal(p, ref)


@pytest.mark.parametrize("seed", [21, 22])
def test_lt_count_equals_searchsorted(seed):
    R, S = datagen.small_random(seed, 2000, 1500, I32_MIN, I32_MAX)
    ss = np.sort(S.key.astype(np.int64))
    expect = int(np.sum(len(ss) - np.searchsorted(ss, R.key.astype(np.int64), side="right")))
    assert oracle.count_lt(R.key, S.key) == expect
    assert oracle.theta_nlj(R.key, S.key, "lt", want_pairs=False)[0] == expect


def test_lt_pairs_equal_per_row_slices():
    """Each R row pairs with exactly the S rows above it in sorted order (numpy argsort)."""
    R, S = datagen.small_random(23, 300, 400, -30, 30)
    order = np.argsort(S.key, kind="stable")
    sk = S.key[order]
    ref = []
    for i, a in enumerate(R.key):
        lo = np.searchsorted(sk, a, side="right")
        ref.extend((i, int(j)) for j in order[lo:])
    ref = np.array(sorted(ref), dtype=np.int32).reshape(-1, 2)
    n, p = oracle.theta_nlj(R.key, S.key, "lt")
    assert n == len(ref) and np.array_equal(p, ref)


def test_large_equi_closed_form_reduced():
    """R.key is a permutation and R.rid its positions, so EQ = {(invperm[S.key[j]], j)}."""
    for zipf in (False, True):
        R, S, perm = datagen.large_equi(seed=2, nR=1 << 14, nS=1 << 16, zipf=zipf)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(len(perm), dtype=np.int32)
        ref = np.stack([inv[S.key], np.arange(S.n, dtype=np.int32)], axis=1)
        ref = ref[np.lexsort((ref[:, 1], ref[:, 0]))]
        n, p = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
        assert n == S.n and np.array_equal(p, ref)
        assert oracle.count_equi(R.key, S.key) == S.n


# ------------------------------------------------------------------------------ invariants --

@pytest.mark.parametrize("seed", [31, 32, 33])
def test_trichotomy_and_complements(seed):
    R, S = datagen.small_random(seed, 400, 350, -20, 20)
    c = {op: oracle.theta_nlj(R.key, S.key, op, want_pairs=False)[0]
         for op in ("eq", "ne", "lt", "le", "gt", "ge")}
    total = R.n * S.n
    assert c["lt"] + c["eq"] + c["gt"] == total
    assert c["ne"] == total - c["eq"]
    assert c["le"] == c["lt"] + c["eq"]
    assert c["ge"] == c["gt"] + c["eq"]
    assert c["eq"] == oracle.count_equi(R.key, S.key)


@pytest.mark.parametrize("op,mirror", [("lt", "gt"), ("le", "ge"), ("gt", "lt"),
                                        ("ge", "le"), ("eq", "eq"), ("ne", "ne")])
def test_mirror_symmetry(op, mirror):
    R, S = datagen.small_random(41, 120, 150, -15, 15)
    _, a = oracle.theta_nlj(R.key, S.key, op)
    _, b = oracle.theta_nlj(S.key, R.key, mirror)
    b = b[:, ::-1]
    b = b[np.lexsort((b[:, 1], b[:, 0]))]
    assert np.array_equal(a, b)


def test_band_zero_is_equality():
    R, S = datagen.small_random(51, 500, 600, -40, 40)
    _, a = oracle.theta_nlj(R.key, S.key, "band", w=0)
    _, b = oracle.equi_nlj(R.key, S.key)
    assert np.array_equal(a, b)


def test_band_monotone_and_conjunction_is_intersection():
    R, S = datagen.small_random(52, 300, 300, -100, 100, with_c=True)
    prev = None
    for w in (0, 1, 3, 8, 50):
        _, band = oracle.theta_nlj(R.key, S.key, "band", w=w)
        sb = set(map(tuple, band.tolist()))
        if prev is not None:
            assert prev <= sb
        prev = sb
        _, lt = oracle.theta_nlj(R.key2, S.key2, "lt")
        _, both = oracle.theta_nlj(R.key, S.key, "band", w=w, Rc=R.key2, Sc=S.key2, op_c="lt")
        assert set(map(tuple, both.tolist())) == sb & set(map(tuple, lt.tolist()))
        n3, win = oracle.band_window(R.key, S.key, w, Rc=R.key2, Sc=S.key2, op_c="lt")
        assert np.array_equal(win, both)


def test_band_counts_by_direct_window_definition():
    """|a-b| <= w  <=>  b in [a-w, a+w]; count by sorted S and numpy (64-bit bounds)."""
    R, S = datagen.small_random(53, 800, 700, I32_MIN, I32_MAX)
    S.key[:50] = I32_MAX
    S.key[50:100] = I32_MIN
    R.key[:20] = I32_MIN
    R.key[20:40] = I32_MAX
    ss = np.sort(S.key.astype(np.int64))
    for w in (0, 5, 1 << 20, I32_MAX):
        a = R.key.astype(np.int64)
        cnt = np.searchsorted(ss, a + w, side="right") - np.searchsorted(ss, a - w, side="left")
        expect = int(cnt.sum())
        assert oracle.theta_nlj(R.key, S.key, "band", w=w, want_pairs=False)[0] == expect, w
        assert oracle.band_window(R.key, S.key, w, want_pairs=False)[0] == expect, w


def test_permutation_invariance_and_empty():
    R, S = datagen.small_random(61, 200, 250, -10, 10, with_c=True)
    g = np.random.default_rng(5)
    pr, ps = g.permutation(R.n), g.permutation(S.n)
    for op in ("eq", "lt", "band"):
        _, a = oracle.theta_nlj(R.key, S.key, op, w=2, Rc=R.key2, Sc=S.key2, op_c="ge")
        _, b = oracle.theta_nlj(R.key[pr], S.key[ps], op, w=2, Rc=R.key2[pr], Sc=S.key2[ps],
                                op_c="ge", Rrid=R.rid[pr], Srid=S.rid[ps])
        assert np.array_equal(a, b)
    e = np.zeros(0, dtype=np.int32)
    assert oracle.equi_nlj(e, S.key)[0] == 0
    assert oracle.equi_sortmerge(R.key, e)[0] == 0
    assert oracle.theta_nlj(e, e, "lt")[0] == 0
    assert oracle.count_equi(e, S.key) == 0 and oracle.count_lt(R.key, e) == 0
    assert oracle.band_window(R.key, e, 3)[0] == 0


@pytest.mark.parametrize("seed", [71, 72])
def test_sortmerge_and_window_match_bruteforce(seed):
    R, S = datagen.small_random(seed, 1000, 1200, -300, 300, with_c=True, rid_mode="random")
    a = oracle.equi_nlj(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    b = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])
    for w, opc in ((4, "lt"), (0, "none"), (30, "ne")):
        a = oracle.theta_nlj(R.key, S.key, "band", w=w, Rc=R.key2, Sc=S.key2, op_c=opc,
                             Rrid=R.rid, Srid=S.rid)
        b = oracle.band_window(R.key, S.key, w, Rc=R.key2, Sc=S.key2, op_c=opc, Rrid=R.rid,
                               Srid=S.rid)
        assert a[0] == b[0] and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("buckets", [1, 3, 7, 64])
def test_result_size_bound_of_section_3_3_3(buckets):
    """Equation rsize: with tuples grouped into reducers by key (here key mod buckets), the
    allocation sum_i |S_i| * |T_i| bounds the exact count from above and |R|*|S| bounds it; it is
    exact when every non-empty group holds a single distinct key."""
    R, S = datagen.small_random(81, 500, 400, 0, 40)
    exact = oracle.count_equi(R.key, S.key)
    br, bs = np.bincount(R.key % buckets, minlength=buckets), np.bincount(S.key % buckets,
                                                                          minlength=buckets)
    rsize = int(np.sum(br.astype(np.int64) * bs))
    assert exact <= rsize <= R.n * S.n
    if buckets >= 40:
        assert exact == rsize


def test_rid_none_means_position():
    R, S = datagen.small_random(91, 50, 60, 0, 5, rid_mode="none")
    a = oracle.equi_nlj(R.key, S.key)
    b = oracle.equi_nlj(R.key, S.key, Rrid=np.arange(R.n, dtype=np.int32),
                        Srid=np.arange(S.n, dtype=np.int32))
    assert np.array_equal(a[1], b[1])
