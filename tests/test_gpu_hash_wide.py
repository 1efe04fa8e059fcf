"""Hash joins whose per-work-unit match counts pass 2^32.

The result-size step of the paper (Section 3.3.3, equation rsize) is computed exactly here, in
64 bits per unit and per wave: a hot build key repeated across a whole LDS table, probed by a
long run of equal probe keys, gives work units of more than 2^32 pairs each.  The expected
counts are closed forms: every R row of the hot key matches every S row of it."""
import numpy as np
import torch

import oracle
from paper_1904_11201_amd import datagen
from tests.gpu_util import dev_rel, gpu, log, need_gpu


def _count(R, S):
    from paper_1904_11201_amd.join import JOIN_KIND_HASH, join_count, workspace
    ws = workspace(JOIN_KIND_HASH, R.n, S.n)
    return join_count(JOIN_KIND_HASH, R, S, None, ws)


@gpu
def test_single_path_units_beyond_2_pow_32():
    """R: 9,216 rows of key 7 (one LDS table, single path), S: 2^28 rows of key 7.  The plan cuts
    S into 512 slices, so every unit holds 9,216 x 524,288 = 4.83e9 pairs."""
    need_gpu()
    from paper_1904_11201_amd.join import Relation
    nR, nS = 9216, 1 << 28
    R = Relation(torch.full((nR,), 7, dtype=torch.int32, device="cuda"))
    S = Relation(torch.full((nS,), 7, dtype=torch.int32, device="cuda"))
    log(f"hash count-only single path {nR} x {nS}, hot key 7")
    got = _count(R, S)
    del S
    torch.cuda.empty_cache()
    assert got == 2_473_901_162_496 == nR * nS


@gpu
def test_partitioned_hot_key_over_16_chunks():
    """Partitioned path: key 7 holds 147,556 build rows (17 LDS chunks of its partition) and
    2^22 probe rows, among 50,000 other build keys and 10^6 other probe keys; the hot
    partition's units hold 9,216 x 524,288 pairs each.  Count = sum over keys of cntR * cntS."""
    need_gpu()
    g = datagen.rng_for(55)
    hot_r, hot_s = 16 * 9216 + 100, 1 << 22
    rk = np.concatenate([np.full(hot_r, 7, np.int32),
                         g.integers(100, 1_000_000, 50_000).astype(np.int32)])
    sk = np.concatenate([g.integers(100, 1_000_000, 1_000_000).astype(np.int32),
                         np.full(hot_s, 7, np.int32)])
    g.shuffle(rk)
    g.shuffle(sk)
    R = datagen.Rel(key=rk, rid=np.arange(len(rk), dtype=np.int32))
    S = datagen.Rel(key=sk, rid=np.arange(len(sk), dtype=np.int32))
    want = oracle.count_equi(R.key, S.key)
    assert want > hot_r * hot_s >= 1 << 39
    log(f"hash count-only partitioned {R.n} x {S.n}, hot key with {hot_r} x {hot_s} rows")
    assert _count(dev_rel(R), dev_rel(S)) == want
