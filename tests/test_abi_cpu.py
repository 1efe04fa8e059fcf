"""C-ABI checks that need no GPU: the library loads, exports every symbol include/join.h
declares, sizes workspaces, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]

n = pytest.importorskip("paper_1904_11201_amd._native",
                        reason="libjoin.so not built (python -m paper_1904_11201_amd.build)")


def declared_functions():
    names = []
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w\s\*]*?\b(join_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    decl = declared_functions()
    assert set(decl) == set(n.EXPORTS), decl
    lib = ctypes.CDLL(n.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name


def test_workspace_sizes():
    assert n.lib.join_workspace_bytes(0, 10, 10, None) == 0
    assert n.lib.join_workspace_bytes(n.JOIN_KIND_HASH, -1, 10, None) == 0
    small = n.lib.join_workspace_bytes(n.JOIN_KIND_HASH, 1 << 16, 1 << 16, None)
    big = n.lib.join_workspace_bytes(n.JOIN_KIND_HASH, 1 << 24, 1 << 26, None)
    assert 0 < small < big
    # the partitioned layout holds both sides' key and rid columns
    assert big >= 4 * 2 * ((1 << 24) + (1 << 26))
    assert n.lib.join_workspace_bytes(n.JOIN_KIND_THETA, 1 << 20, 1 << 20, None) > 0
    assert n.lib.join_scan_workspace_bytes(0) > 0
    assert n.lib.join_scan_workspace_bytes(-1) == 0


def _rel(ptr, nrows):
    return n.JoinRel(ptr, None, None, nrows)


def _count(kind, R, S, pred=None, ws=None, ws_bytes=0):
    c = ctypes.c_uint64(7)
    rc = n.lib.join_count(kind, ctypes.byref(R), ctypes.byref(S),
                          ctypes.byref(pred) if pred is not None else None, ws, ws_bytes, None,
                          ctypes.byref(c))
    return rc, c.value


def test_argument_errors():
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    ok = _rel(fake, 10)
    assert _count(9, ok, ok)[0] == n.JOIN_E_INVAL
    assert _count(n.JOIN_KIND_HASH, _rel(fake, -3), ok)[0] == n.JOIN_E_INVAL
    assert _count(n.JOIN_KIND_HASH, _rel(None, 5), ok)[0] == n.JOIN_E_INVAL
    assert _count(n.JOIN_KIND_HASH, _rel(fake, 1 << 31), ok)[0] == n.JOIN_E_UNSUPPORTED
    assert _count(n.JOIN_KIND_THETA, ok, ok, None)[0] == n.JOIN_E_INVAL
    bad = [n.JoinPred(0, 0, 0), n.JoinPred(8, 0, 0), n.JoinPred(3, 0, 7), n.JoinPred(7, -1, 0),
           n.JoinPred(3, 0, -1)]
    for p in bad:
        assert _count(n.JOIN_KIND_THETA, ok, ok, p)[0] == n.JOIN_E_INVAL, (p.op_a, p.w, p.op_c)
    # a condition on column c needs key2 on both sides
    assert _count(n.JOIN_KIND_THETA, ok, ok, n.JoinPred(3, 0, 3))[0] == n.JOIN_E_INVAL
    # workspace missing or too small
    assert _count(n.JOIN_KIND_HASH, ok, ok)[0] == n.JOIN_E_WORKSPACE
    assert _count(n.JOIN_KIND_HASH, ok, ok, ws=fake, ws_bytes=8)[0] == n.JOIN_E_WORKSPACE
    assert "workspace" in n.last_error()
    # count pointer is required
    rc = n.lib.join_count(n.JOIN_KIND_HASH, ctypes.byref(ok), ctypes.byref(ok), None, fake, 1 << 30,
                          None, None)
    assert rc == n.JOIN_E_INVAL
    # scan primitive
    assert n.lib.join_scan_u64(None, None, -1, None, fake, 1 << 20, None) == n.JOIN_E_INVAL
    assert n.lib.join_scan_u64(fake, fake, 10, None, None, 0, None) == n.JOIN_E_WORKSPACE


def test_empty_relations_need_no_device():
    """An empty side has an exact count of 0 without any kernel launch."""
    fake = ctypes.c_void_p(0x1000)
    ws_bytes = n.lib.join_workspace_bytes(n.JOIN_KIND_HASH, 0, 10, None)
    rc, c = _count(n.JOIN_KIND_HASH, _rel(None, 0), _rel(fake, 10), ws=fake, ws_bytes=ws_bytes)
    assert rc == n.JOIN_OK and c == 0
    p = n.JoinPred(n.OPS["lt"], 0, 0)
    ws_bytes = n.lib.join_workspace_bytes(n.JOIN_KIND_THETA, 10, 0, None)
    rc, c = _count(n.JOIN_KIND_THETA, _rel(fake, 10), _rel(None, 0), p, ws=fake, ws_bytes=ws_bytes)
    assert rc == n.JOIN_OK and c == 0


def test_single_hip_runtime_shared_with_torch():
    """libjoin binds to the HIP runtime torch already loaded, so torch's device pointers and
    stream handles are valid inside it."""
    rts = n._hip_runtimes()
    assert len(rts) == 1, rts


def _jobs(specs):
    fake = ctypes.c_void_p(0x1000)  # never dereferenced by the sizing and validation calls
    arr = (n.JoinJob * max(len(specs), 1))()
    for i, (nr, ns, bits, reserved) in enumerate(specs):
        arr[i] = n.JoinJob(_rel(fake if nr else None, nr), _rel(fake if ns else None, ns), bits, reserved)
    return arr


def test_batch_workspace_sizes_and_argument_errors():
    ws = n.lib.join_batch_workspace_bytes
    assert ws(0, _jobs([])) > 0  # an empty batch still has its header
    assert ws(-1, _jobs([])) == 0
    one = ws(1, _jobs([(1000, 2000, -1, 0)]))
    two = ws(2, _jobs([(1000, 2000, -1, 0), (1 << 20, 1 << 22, -1, 0)]))
    assert 0 < one < two
    # the partitioned tuples of both sides are part of the workspace
    assert two >= 8 * (1000 + 2000 + (1 << 20) + (1 << 22))
    assert ws(1, _jobs([(10, 10, 12, 0)])) == 0        # fan-out above 2^11
    assert ws(1, _jobs([(10, 10, -1, 1)])) == 0        # reserved must be 0
    assert ws(1, _jobs([(-1, 10, -1, 0)])) == 0        # negative size
    arr = _jobs([(10, 10, -1, 0)])
    arr[0].R.key = None                                # key NULL with n > 0
    assert ws(1, arr) == 0
    # 32-bit row indices: three probe sides of 2^31 - 1 rows exceed them, two do not
    big = (1 << 31) - 1
    assert ws(2, _jobs([(10, big, -1, 0), (10, big, -1, 0)])) > 0
    assert ws(3, _jobs([(10, big, -1, 0)] * 3)) == 0
    plan = n.JoinBatchPlan()
    rc = n.lib.join_batch_prepare(1, _jobs([(10, 10, 12, 0)]), None, 0, ctypes.byref(plan), None)
    assert rc == n.JOIN_E_INVAL and "bits" in n.last_error()
    rc = n.lib.join_batch_prepare(1, _jobs([(10, 10, -1, 0)]), None, 0, ctypes.byref(plan), None)
    assert rc == n.JOIN_E_WORKSPACE
    assert n.lib.join_batch_count(None, None, 0, None, None) == n.JOIN_E_INVAL
    assert n.lib.join_batch_materialize(None, None, 0, None, 0, None) == n.JOIN_E_INVAL


def test_tuning_knobs_override_environment(monkeypatch):
    monkeypatch.setenv("JOIN_HASH_CAP", "4096")
    assert n.tune_get("hash.cap", 9216) == 4096
    small = n.lib.join_workspace_bytes(n.JOIN_KIND_HASH, 1 << 24, 1 << 26, None)
    n.tune_set("hash.cap", 10240)
    try:
        assert n.tune_get("hash.cap", 9216) == 10240
        # fewer, larger partitions: smaller histogram/offset arrays in the workspace
        assert n.lib.join_workspace_bytes(n.JOIN_KIND_HASH, 1 << 24, 1 << 26, None) != small
    finally:
        n.tune_set("hash.cap", None)
    assert n.tune_get("hash.cap", 9216) == 4096
    monkeypatch.delenv("JOIN_HASH_CAP")
    assert n.tune_get("hash.cap", 9216) == 9216
    with pytest.raises(KeyError):
        n.tune_set("no.such.knob", 1)


def test_thread_local_knobs_win_and_stay_on_their_thread():
    """join_tune_set_local: the calling thread sees its own value over the process-wide one;
    other threads do not see it."""
    import threading
    n.tune_set("theta.ts", 4096)
    try:
        n.tune_set("theta.ts", 512, local=True)
        seen = {}
        t = threading.Thread(target=lambda: seen.setdefault("other", n.tune_get("theta.ts", 0)))
        t.start()
        t.join()
        assert n.tune_get("theta.ts", 0) == 512
        assert seen["other"] == 4096
        n.tune_set("theta.ts", None, local=True)
        assert n.tune_get("theta.ts", 0) == 4096
    finally:
        n.tune_set("theta.ts", None, local=True)
        n.tune_set("theta.ts", None)
    assert n.tune_get("theta.ts", 0) == 0


def test_build_sizes_and_argument_errors():
    assert n.lib.join_build_bytes(-1) == 0
    assert n.lib.join_build_bytes(1 << 31) == 0
    small, big = n.lib.join_build_bytes(1000), n.lib.join_build_bytes(1 << 24)
    assert 0 < small < big and big >= 8 * (1 << 24)
    desc = n.JoinBuild()
    fake = ctypes.c_void_p(0x1000)
    R = _rel(fake, 1000)
    assert n.lib.join_build(ctypes.byref(R), None, 0, ctypes.byref(desc), None) == n.JOIN_E_WORKSPACE
    assert n.lib.join_build(ctypes.byref(_rel(None, 5)), None, 0, ctypes.byref(desc), None) == n.JOIN_E_INVAL
    # a zeroed descriptor is not a build
    assert n.lib.join_probe_workspace_bytes(ctypes.byref(n.JoinBuild()), 10) == 0
    S = _rel(fake, 10)
    c = ctypes.c_uint64(0)
    assert n.lib.join_probe_count(ctypes.byref(n.JoinBuild()), fake, ctypes.byref(S), None, 0, None,
                                  ctypes.byref(c)) == n.JOIN_E_INVAL


def test_ceiling_calls_reject_bad_arguments():
    lib = n.lib
    # size not a multiple of 16, null pointers with bytes > 0, misaligned pointers
    assert lib.join_prof_copy(None, None, 8, None) == 1
    assert lib.join_prof_copy(None, None, 16, None) == 1
    assert lib.join_prof_copy(ctypes.c_void_p(8), ctypes.c_void_p(64), 16, None) == 1
    assert lib.join_prof_copy(None, None, 0, None) == 0
    sink = ctypes.c_void_p(256)
    assert lib.join_prof_valu(0, 1, 0, sink, sink, None) == 1
    assert lib.join_prof_valu((1 << 22) + 1, 1, 0, sink, sink, None) == 1
    assert lib.join_prof_valu(1, 1, 0, None, sink, None) == 1
    assert lib.join_prof_valu(1, 1, 5, sink, sink, None) == 1
    assert "join_prof_valu" in n.last_error()
    assert lib.join_prof_stream(0, None, sink, 16, None) == 1
    assert lib.join_prof_stream(1, None, sink, 16, None) == 1
    assert lib.join_prof_stream(2, None, ctypes.c_void_p(8), 16, None) == 1
    assert lib.join_prof_stream(2, None, sink, 8, None) == 1
    assert lib.join_prof_stream(1, None, None, 0, None) == 0
    assert "join_prof_stream" in n.last_error()
