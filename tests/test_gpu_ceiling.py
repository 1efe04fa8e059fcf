"""The ceiling kernels behind the measured roofline denominators: the copy moves every byte,
and the VALU spin performs exactly the add/xor chains it counts."""
import numpy as np
import pytest
import torch

from tests.gpu_util import gpu, log, need_gpu


@gpu
@pytest.mark.parametrize("nbytes", [16, 4096, 16 * 1021, (1 << 24) + 16 * 37])
def test_copy_moves_every_byte(nbytes):
    need_gpu()
    from paper_1904_11201_amd import join as J
    log(f"ceiling copy bytes={nbytes}")
    g = np.random.default_rng(nbytes)
    x = torch.from_numpy(g.integers(-2**31, 2**31, size=nbytes // 4, dtype=np.int64)
                         .astype(np.int32)).cuda()
    y = torch.full_like(x, -1)
    J.prof_copy(x, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


@gpu
@pytest.mark.parametrize("mix", [0, 1, 2])
@pytest.mark.parametrize("blocks,iters", [(1, 0), (3, 1), (5, 257)])
def test_valu_spin_results_and_clock(blocks, iters, mix):
    need_gpu()
    from paper_1904_11201_amd import join as J
    log(f"ceiling valu blocks={blocks} iters={iters} mix={mix}")
    sink = torch.full((blocks * 256,), -1, dtype=torch.int32, device="cuda")
    clk = torch.zeros(2, dtype=torch.int64, device="cuda")
    ops = J.prof_valu(blocks, iters, sink, clk, mix=mix)
    torch.cuda.synchronize()
    assert ops == blocks * 256 * (48 if mix == 2 else 32) * iters
    # each lane: a_j = 16 * gid + j, b = 0x9E3779B9 ^ block
    m32 = np.uint64(0xFFFFFFFF)
    gid = np.arange(blocks * 256, dtype=np.uint64)
    b = (np.uint64(0x9E3779B9) ^ (gid // np.uint64(256))) & m32
    a = (gid[:, None] * np.uint64(16) + np.arange(16, dtype=np.uint64)[None, :]) & m32
    if mix == 0:  # a <- (a + b) ^ b, iterated; the lane keeps the xor of its chains
        for _ in range(iters):
            a = ((a + b[:, None]) & m32) ^ b[:, None]
        want = np.bitwise_xor.reduce(a, axis=1).astype(np.uint32).view(np.int32)
    elif mix == 2:  # min over the lane's 16 values of (b - a_j) mod 2^32; all ones if no pass
        d = ((b[:, None] - a) & m32).min(axis=1)
        want = (d if iters > 0 else np.full_like(d, 0xFFFFFFFF)).astype(np.uint32).view(np.int32)
    else:  # wave mask of lanes with some (b - a_j) mod 2^32 <= 2^20; halves xored
        hit = (((b[:, None] - a) & m32) <= np.uint64(1 << 20)).any(axis=1) & (iters > 0)
        w = hit.reshape(-1, 64)
        mask = (w.astype(np.uint64) << np.arange(64, dtype=np.uint64)[None, :]).sum(axis=1,
                                                                                   dtype=np.uint64)
        lanes = ((mask & m32) ^ (mask >> np.uint64(32))).astype(np.uint32).view(np.int32)
        want = np.repeat(lanes, 64)
    assert np.array_equal(sink.cpu().numpy(), want)
    cyc, ticks = clk.cpu().tolist()
    assert cyc >= 0 and ticks >= 0
    assert J.prof_wall_clock_hz() > 0
