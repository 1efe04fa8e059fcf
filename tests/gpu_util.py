"""Helpers for the GPU parity tests: moving seeded relations to the device and putting pair
arrays in canonical order (ascending by (rid_R, rid_S) as signed int32) on either side."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

gpu = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def dev_rel(rel, with_rid=True):
    from paper_1904_11201_amd.join import Relation

    def d(a):
        return None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()

    return Relation(d(rel.key), d(rel.key2), d(rel.rid) if with_rid else None)


def canon_gpu(pairs: torch.Tensor) -> np.ndarray:
    """Sort [n, 2] int32 device pairs canonically on the GPU, return as numpy."""
    if pairs.numel() == 0:
        return np.zeros((0, 2), np.int32)
    a = pairs[:, 0].to(torch.int64)
    b = pairs[:, 1].to(torch.int64) + (1 << 31)
    k = a * (1 << 32) + b
    order = torch.sort(k).indices
    return pairs[order].cpu().numpy()


def canon_np(p: np.ndarray) -> np.ndarray:
    if len(p) == 0:
        return np.zeros((0, 2), np.int32)
    return p[np.lexsort((p[:, 1], p[:, 0]))]
