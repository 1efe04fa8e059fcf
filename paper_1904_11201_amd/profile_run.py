"""A fixed workload to run under a profiler (rocprofv3 --kernel-trace / --pmc).

    python -m paper_1904_11201_amd.profile_run hash    # 16M x 64M uniform hash join, three times
    python -m paper_1904_11201_amd.profile_run theta   # 1M x 1M band (w = 8) and R.c < S.c, once
    python -m paper_1904_11201_amd.profile_run valu    # the five int32 VALU spins, once each
    python -m paper_1904_11201_amd.profile_run copy    # the 1 GiB device copy, three times

Inputs are the seeded synthetic workloads of datagen (seed 2 and seed 4), copied to the device
before the joins; each join is count + exact allocation + write.
"""
from __future__ import annotations

import sys

import numpy as np
import torch

from . import datagen
from . import join as J


def _d(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


def main(argv=None) -> int:
    what = (argv if argv is not None else sys.argv[1:]) or ["hash"]
    if what[0] == "hash":
        R, S, _ = datagen.large_equi(seed=2, zipf=False)
        dR, dS = J.Relation(_d(R.key), rid=_d(R.rid)), J.Relation(_d(S.key), rid=_d(S.rid))
        ws = J.workspace(J.JOIN_KIND_HASH, R.n, S.n)
        for _ in range(3):
            out = J.hash_join(dR, dS, ws=ws)
    elif what[0] == "theta":
        R, S = datagen.band_theta(seed=4, n=1 << 20)
        dR = J.Relation(_d(R.key), _d(R.key2), _d(R.rid))
        dS = J.Relation(_d(S.key), _d(S.key2), _d(S.rid))
        out = J.theta_join(dR, dS, J.Pred("band", 8, "lt"))
    elif what[0] == "valu":
        # the spins of the measured VALU ceilings, at the launch shape the benchmark uses
        props = torch.cuda.get_device_properties(0)
        blocks, iters = props.multi_processor_count * 8, 1 << 14
        sink = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
        clk = torch.zeros(2, dtype=torch.int64, device="cuda")
        for mix in (0, 1, 2, 3, 4):
            J.prof_valu(blocks, iters, sink, clk, mix=mix)
        out = sink
    elif what[0] == "copy":
        src = torch.ones((1 << 30) // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            J.prof_copy(src, dst)
        out = dst
    else:
        print(f"unknown workload {what[0]!r}: hash, theta, valu or copy", file=sys.stderr)
        return 2
    torch.cuda.synchronize()
    print("done", out.shape[0], flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
