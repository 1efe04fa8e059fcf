"""C-ABI behaviour on the GPU: snprintf-style capacity handling, count/materialize split,
workspace reuse, and the device scan primitive against an exclusive prefix sum."""
import numpy as np
import pytest
import torch

import oracle
from paper_1904_11201_amd import datagen
from tests.gpu_util import canon_gpu, dev_rel, gpu, log, need_gpu


@gpu
@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4095, 4096, 4097, 100_000, (1 << 20) + 7])
def test_scan_u64(n):
    need_gpu()
    from paper_1904_11201_amd.join import join_scan_u64
    g = np.random.default_rng(n)
    x = g.integers(0, 1 << 40, size=n, dtype=np.int64)
    log(f"scan n={n}")
    out, total = join_scan_u64(torch.from_numpy(x).cuda())
    ref = np.concatenate([[0], np.cumsum(x)[:-1]]) if n else np.zeros(0, np.int64)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert int(total.item()) == int(x.sum())


@gpu
@pytest.mark.parametrize("kind", ["hash", "theta"])
def test_capacity_too_small_then_materialize(kind):
    need_gpu()
    from paper_1904_11201_amd import join as J
    R, S = datagen.small_random(13, 3000, 4000, 0, 300)
    pred = J.Pred("eq") if kind == "theta" else None
    k = J.JOIN_KIND_THETA if kind == "theta" else J.JOIN_KIND_HASH
    dR, dS = dev_rel(R), dev_rel(S)
    ws = J.workspace(k, R.n, S.n, pred)
    n_exact = oracle.count_equi(R.key, S.key)
    small = torch.full((n_exact - 1, 2), -7, dtype=torch.int32, device="cuda")
    fn = (lambda p: J.join_theta(dR, dS, pred, ws, p)) if kind == "theta" else (
        lambda p: J.join_hash(dR, dS, ws, p))
    with pytest.raises(J.JoinError) as ei:
        fn(small)
    assert ei.value.status == 2 and ei.value.count == n_exact
    torch.cuda.synchronize()
    assert bool((small == -7).all()), "nothing may be written when capacity is too small"
    # the workspace still holds the count: materialize without recounting
    with pytest.raises(J.JoinError):
        J.join_materialize(k, dR, dS, pred, ws, small)
    out = torch.empty((n_exact, 2), dtype=torch.int32, device="cuda")
    J.join_materialize(k, dR, dS, pred, ws, out)
    _, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    assert np.array_equal(canon_gpu(out), ref)


@gpu
def test_workspace_reuse_across_joins():
    need_gpu()
    from paper_1904_11201_amd import join as J
    ws = J.workspace(J.JOIN_KIND_HASH, 300_000, 300_000)
    for seed in (1, 2, 3):
        R, S = datagen.small_random(seed, 200_000 + seed, 250_000, 0, 100_000)
        got = canon_gpu(J.hash_join(dev_rel(R), dev_rel(S), ws=ws))
        n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
        assert len(got) == n and np.array_equal(got, ref)


@gpu
def test_streams_are_respected():
    need_gpu()
    from paper_1904_11201_amd import join as J
    R, S = datagen.small_random(8, 100_000, 100_000, 0, 50_000)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dR, dS = dev_rel(R), dev_rel(S)
        out = J.hash_join(dR, dS, stream=s)
    s.synchronize()
    n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    assert np.array_equal(canon_gpu(out), ref)


@gpu
@pytest.mark.parametrize("kind", ["hash", "theta", "region"])
def test_plan_changed_between_count_and_materialize(kind):
    """The count pass records its plan's signature in the workspace.  A tuning knob changed
    before the write pass: on the same thread join_materialize refuses (JOIN_E_INVAL); from
    another thread, where the host cannot tell, the write kernels refuse and write nothing.
    Counting again under the new plan then works."""
    need_gpu()
    import threading
    from paper_1904_11201_amd import _native
    from paper_1904_11201_amd import join as J
    R, S = datagen.band_theta(seed=31, n=20_000, hi=1 << 14)
    if kind == "hash":
        k, pred, knob, vals = J.JOIN_KIND_HASH, None, "hash.cap", (4096, 2048)
    elif kind == "theta":
        k, pred, knob, vals = J.JOIN_KIND_THETA, J.Pred("band", 8, "lt"), "theta.ts", (512, 1024)
    else:
        k, pred, knob, vals = J.JOIN_KIND_THETA_REGION, J.Pred("band", 8, "lt"), "theta.stash", (64, 32)
    dR, dS = dev_rel(R), dev_rel(S)
    if kind == "hash":
        n_exact, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
    else:
        n_exact, ref = oracle.theta_nlj(R.key, S.key, "band", w=8, Rc=R.key2, Sc=S.key2,
                                        op_c="lt", Rrid=R.rid, Srid=S.rid)
    sizes = []
    for v in vals:
        _native.tune_set(knob, v, local=True)
        sizes.append(J.join_workspace_bytes(k, R.n, S.n, pred))
    ws = torch.empty(max(sizes), dtype=torch.uint8, device="cuda")
    try:
        _native.tune_set(knob, vals[0], local=True)
        log(f"plan stamp {kind}: count under {knob}={vals[0]}")
        assert J.join_count(k, dR, dS, pred, ws) == n_exact
        _native.tune_set(knob, vals[1], local=True)
        out = torch.full((n_exact, 2), -7, dtype=torch.int32, device="cuda")
        with pytest.raises(J.JoinError) as ei:
            J.join_materialize(k, dR, dS, pred, ws, out)
        assert ei.value.status == _native.JOIN_E_INVAL
        # another thread (the host keeps no record there): the device refuses
        errs = []

        def other():
            try:
                _native.tune_set(knob, vals[1], local=True)
                J.join_materialize(k, dR, dS, pred, ws, out)
                torch.cuda.synchronize()
            except Exception as e:  # noqa: BLE001
                errs.append(e)
        t = threading.Thread(target=other)
        t.start()
        t.join()
        assert not errs, errs
        assert bool((out == -7).all()), "a write pass under another plan must write nothing"
        # count again under the new plan, then the write goes through
        assert J.join_count(k, dR, dS, pred, ws) == n_exact
        J.join_materialize(k, dR, dS, pred, ws, out)
        assert np.array_equal(canon_gpu(out), ref)
    finally:
        _native.tune_set(knob, None, local=True)
