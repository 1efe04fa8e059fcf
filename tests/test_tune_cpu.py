"""Autotuner cache lookups (host logic only; the measurements themselves need a GPU)."""
from paper_1904_11201_amd import tune


class _J:
    def __init__(self, n, bits=-1):
        self.R = type("R", (), {"n": n})()
        self.bits = bits


CACHE = {"hash_bits": {"10": 0, "14": 1, "18": 6, "22": 10}, "theta_ts": {"12": 1024, "16": 4096}}


def test_nearest_bucket_at_or_below():
    assert tune.hash_bits_for(1 << 18, CACHE) == 6
    # bucket 20 -> tuned 18's 6 bits, raised to the 8 that 2^20 rows need with 4608-entry tables
    # (16K-row partitions would take four tables, each probing the partition's S slice)
    assert tune.hash_bits_for((1 << 20) + 5, CACHE) == 8
    assert tune.hash_bits_for((1 << 20) + 5, CACHE, cap=9216) == 7
    assert tune.hash_bits_for(1 << 23, CACHE) == 11
    assert tune.hash_bits_for(100, CACHE) == 0                # below every bucket: the smallest
    assert tune.hash_bits_for(1 << 18, {}) == -1              # nothing tuned: library default


def test_fan_out_keeps_partitions_inside_one_table():
    """The lookup never picks fewer bits than the size needs for a mean partition of at most
    0.9 of the table capacity: fewer would split partitions into several R chunks."""
    import numpy as np
    cap = tune.HASH_CAP
    assert tune.hash_min_bits(int(0.9 * cap), cap) == 0
    assert tune.hash_min_bits(int(0.9 * cap) + 1, cap) == 1
    assert tune.hash_min_bits(3_000_000, cap) == 10         # 3M / 2^10 = 2930 <= 4147 < 5859
    assert tune.hash_min_bits(3_000_000, 9216) == 9         # 3M / 2^9 = 5859 <= 8294 < 11719
    assert tune.hash_min_bits(1 << 40, cap) == tune.HASH_MAX_BITS
    sizes = np.unique(np.logspace(10, 22, 200, base=2).astype(np.int64))
    got = tune.hash_bits_for_sizes(sizes, CACHE)
    assert (sizes / (1 << got.astype(np.int64)) <= 0.9 * cap).all()
    assert (got >= np.array([tune.hash_bits_for(1 << int(np.log2(n)), CACHE) for n in sizes])).all()


def test_theta_tile_clamped_to_probe_side():
    assert tune.theta_ts_for(1 << 16, 1 << 16, CACHE) == 4096
    assert tune.theta_ts_for(1 << 12, 300, CACHE) == 300
    assert tune.theta_ts_for(1 << 16, 1 << 16, {}) == 0


def test_apply_bits_keeps_explicit_choices():
    jobs = [_J(1 << 14), _J(1 << 22, bits=3)]
    tune.apply_bits(jobs, CACHE)
    assert [j.bits for j in jobs] == [2, 3]  # 2^14 rows: tuned 1 bit, raised to fit 4608 entries


def test_bits_for_sizes_matches_the_per_size_lookup():
    import numpy as np
    sizes = np.array([1, 100, 1 << 10, (1 << 14) + 3, 1 << 18, (1 << 20) + 5, 1 << 23, 3 << 21])
    got = tune.hash_bits_for_sizes(sizes, CACHE)
    assert got.tolist() == [tune.hash_bits_for(int(n), CACHE) for n in sizes]
    assert tune.hash_bits_for_sizes(sizes, {}).tolist() == [-1] * len(sizes)


def test_packed_job_table_checks_offsets():
    import numpy as np
    import pytest
    import torch
    from paper_1904_11201_amd import join as J
    k = torch.zeros(10, dtype=torch.int32)
    for roffs, soffs in (([0, 5, 4, 10], [0, 3, 6, 10]),   # falling
                         ([0, 5, 9], [0, 5, 10]),          # does not end at the length
                         ([1, 5, 10], [0, 5, 10]),         # does not start at 0
                         ([0, 5, 10], [0, 10])):           # sides disagree on the join count
        with pytest.raises(ValueError):
            J._packed_array(k, np.array(roffs), k, np.array(soffs))
