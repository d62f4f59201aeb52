"""Shared helpers for GPU tests: build library handles from generator output
and compare against the CPU oracle."""
import sys

import numpy as np


def say(*a):
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev_graph(g):
    import paper_2310_11222_amd as nvd
    return nvd.Graph(g.row_ptr, g.col_idx, g.w)


def to_dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = np.where(want != 0, np.abs(want), 1.0)
    return np.abs(got - want) / den
