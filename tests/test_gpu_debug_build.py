"""The checking build (libjoin_debug.so, compiled with JL_DEBUG): every write pass counts the pairs
it writes per work unit and join_materialize compares them with what the count pass counted,
and join_materialize refuses to write when R, S or the workspace changed since join_count.

Run in a child process that loads the checking build (JOIN_LIBRARY), on inputs shaped like the
small equi join (64K x 64K), a partitioned equi join and the band theta join (nested loop and
region pruning), each checked against the oracle; then one call that changes S between the count
and the write, which must be refused."""
import os
import subprocess
import sys

import pytest

from tests.gpu_util import gpu, log, need_gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys
import numpy as np
import torch
import oracle
from paper_1904_11201_amd import _native, datagen
from paper_1904_11201_amd import join as J
from tests.gpu_util import canon_gpu, dev_rel
assert _native.LIB_PATH.endswith("libjoin_debug.so"), _native.LIB_PATH

def check(label, got, n, ref):
    assert len(got) == n and np.array_equal(got, ref), label
    print("ok", label, n, flush=True)

R, S = datagen.small_equi(seed=1)
n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
check("hash 64K x 64K", canon_gpu(J.hash_join(dev_rel(R), dev_rel(S))), n, ref)
R, S = datagen.small_random(71, 1_000_000, 4_000_000, 0, 900_000, rid_mode="random")
n, ref = oracle.equi_sortmerge(R.key, S.key, Rrid=R.rid, Srid=S.rid)
check("hash 1M x 4M partitioned", canon_gpu(J.hash_join(dev_rel(R), dev_rel(S))), n, ref)
R, S = datagen.band_theta(seed=4, n=1 << 18)
n, ref = oracle.band_window(R.key, S.key, 8, Rc=R.key2, Sc=S.key2, op_c="lt", Rrid=R.rid, Srid=S.rid)
p = J.Pred("band", 8, "lt")
dR, dS = dev_rel(R), dev_rel(S)
check("theta band 256K x 256K", canon_gpu(J.theta_join(dR, dS, p)), n, ref)
check("region band 256K x 256K", canon_gpu(J.theta_join(dR, dS, p, region=True)), n, ref)

# S changed between the count and the write: refused, nothing written
ws = J.workspace(J.JOIN_KIND_THETA, R.n, S.n, p)
cnt = J.join_count(J.JOIN_KIND_THETA, dR, dS, p, ws)
dS.key[0] += 1
out = torch.full((cnt, 2), -7, dtype=torch.int32, device="cuda")
try:
    J.join_materialize(J.JOIN_KIND_THETA, dR, dS, p, ws, out)
except J.JoinError as e:
    assert e.status == _native.JOIN_E_INVAL and "changed" in str(e), e
    torch.cuda.synchronize()
    assert bool((out == -7).all())
    print("ok refused", flush=True)
else:
    raise AssertionError("a changed input was not refused")
'''


@gpu
def test_checking_build_counts_and_fingerprints():
    need_gpu()
    lib = os.path.join(ROOT, "paper_1904_11201_amd", "libjoin_debug.so")
    if not os.path.exists(lib):
        pytest.fail("libjoin_debug.so is missing: build it with python -m paper_1904_11201_amd.build --debug")
    env = dict(os.environ, JOIN_LIBRARY="libjoin_debug.so", PYTHONPATH=ROOT)
    log("checking build: child process with libjoin_debug.so")
    r = subprocess.run([sys.executable, "-u", "-c", CHILD], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=240)
    log(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count("ok") == 5
