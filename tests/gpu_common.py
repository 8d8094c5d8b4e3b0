"""Helpers for the GPU tests (not collected): test-side CSR building from a
canonical edge list (numpy; shares nothing with the oracle or the HIP
library) and device transfers."""
from __future__ import annotations

import sys

import numpy as np
import torch


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def csr_np(n: int, eu, ev):
    """Symmetric CSR with sorted rows from an edge list without self-loops
    or duplicates."""
    eu = np.asarray(eu, np.int64)
    ev = np.asarray(ev, np.int64)
    u = np.concatenate([eu, ev])
    v = np.concatenate([ev, eu])
    order = np.lexsort((v, u))
    u, v = u[order], v[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(u, minlength=n), out=row_ptr[1:])
    return row_ptr.astype(np.int32), v.astype(np.int32)


def to_dev(a, dtype=torch.int32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def graph_dev(P, row_ptr, col_idx):
    return P.Graph(to_dev(row_ptr), to_dev(col_idx))
