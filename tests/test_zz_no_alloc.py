"""join_hash_noalloc: the hash join with its workspace in the library's static device array.

Called through the C ABI and compared with join_hash (the same join with a caller workspace),
pair for pair after canonical sorting, on two calls in a row, the second with a smaller input
(the array keeps the first call's contents), and on a partitioned join before a single-path
one.  Also: the count lands on the device; an output too small receives nothing; a join whose
workspace exceeds the array is refused."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1904_11201_amd import datagen
from tests.gpu_util import canon_gpu, dev_rel, gpu, log, need_gpu


def _noalloc(R, S, cap):
    """Direct C-ABI call; returns (status, count tensor, pairs tensor)."""
    from paper_1904_11201_amd import _native
    pairs = torch.full((max(cap, 1), 2), -7, dtype=torch.int32, device="cuda")
    count = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    rr, sr = R.c(), S.c()
    rc = _native.lib.join_hash_noalloc(ctypes.byref(rr), ctypes.byref(sr),
                                       ctypes.c_void_p(pairs.data_ptr()) if cap else None, cap,
                                       ctypes.c_void_p(count.data_ptr()), None)
    torch.cuda.synchronize()
    return rc, int(count.item()), pairs[:cap]


def _with_workspace(R, S):
    from paper_1904_11201_amd import join as J
    return canon_gpu(J.hash_join(R, S))


@gpu
@pytest.mark.parametrize("sizes", [
    ((1_000_000, 4_000_000, 500_000), (65_536, 65_536, 16_384)),   # partitioned, then single path
    ((120_000, 300_000, 50_000), (5_000, 7_000, 3_000)),           # single path twice, smaller
])
def test_noalloc_matches_join_hash_on_two_calls(sizes):
    need_gpu()
    from paper_1904_11201_amd import _native
    for i, (nR, nS, dom) in enumerate(sizes):
        Rh, Sh = datagen.small_random(90 + i, nR, nS, 0, dom, rid_mode="random")
        R, S = dev_rel(Rh), dev_rel(Sh)
        want = _with_workspace(R, S)
        log(f"noalloc call {i + 1}: {nR} x {nS}, {len(want)} pairs")
        rc, n, pairs = _noalloc(R, S, len(want))
        assert rc == _native.JOIN_OK, _native.last_error()
        assert n == len(want)
        assert np.array_equal(canon_gpu(pairs), want)


@gpu
def test_noalloc_small_output_and_empty_and_too_large():
    need_gpu()
    from paper_1904_11201_amd import _native
    from paper_1904_11201_amd import join as J
    Rh, Sh = datagen.small_random(95, 20_000, 30_000, 0, 10_000)
    R, S = dev_rel(Rh), dev_rel(Sh)
    n_want = len(_with_workspace(R, S))
    log("noalloc capacity one short")
    rc, n, pairs = _noalloc(R, S, n_want - 1)
    assert rc == _native.JOIN_OK and n == n_want
    assert bool((pairs == -7).all()), "an output too small must receive nothing"
    log("noalloc empty side")
    rc, n, _ = _noalloc(R, J.Relation(torch.empty(0, dtype=torch.int32, device="cuda")), 0)
    assert rc == _native.JOIN_OK and n == 0
    log("noalloc above the array")
    big = J.Relation(torch.zeros(8 << 20, dtype=torch.int32, device="cuda"))
    rc, _, _ = _noalloc(big, big, 0)
    assert rc == _native.JOIN_E_WORKSPACE and "scratch" in _native.last_error()
