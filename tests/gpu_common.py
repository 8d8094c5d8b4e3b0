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


def _by_distance(row_ptr, col_idx, order, first_vertices, tail_vertices, tail):
    """Stable re-rank of `tail` (items, with vertices tail_vertices) by the BFS
    distance of their vertex from the highest-degree vertex among
    first_vertices (first on ties): nearest first, distances past 30
    together, unreached last."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    rp = np.asarray(row_ptr, np.int64)
    n = len(rp) - 1
    deg = np.diff(rp)
    probe = int(first_vertices[np.argmax(deg[first_vertices])])
    adj = csr_matrix((np.ones(len(col_idx), np.int8), np.asarray(col_idx), rp), shape=(n, n))
    dist = shortest_path(adj, method="D", unweighted=True, directed=False, indices=probe)
    dt = dist[tail_vertices]
    key = np.where(np.isinf(dt), 31, np.minimum(np.where(np.isinf(dt), 0, dt), 30)).astype(np.int64)
    return tail[np.argsort(key, kind="stable")]


def allsource_batch_order(row_ptr, col_idx, width: int):
    """The order in which all-source batches take their sources: the
    vertices that have arcs, by degree class (rows longer than 64 arcs, then
    64, 32-63, ..., 1), ids ascending inside a class; with more than one
    batch, the batches after the first take the remaining vertices by their
    BFS distance from the first batch's highest-degree vertex (first in that
    order on ties): nearest first, distances past 30 together, the vertices
    it does not reach last, the order above among equals."""
    rp = np.asarray(row_ptr, np.int64)
    deg = np.diff(rp)
    act = np.nonzero(deg)[0]
    cls = np.where(deg[act] > 64, 0, 7 - np.floor(np.log2(np.maximum(deg[act], 1))).astype(np.int64))
    order = act[np.lexsort((act, cls))]
    if len(order) <= width:
        return order
    first = order[:width]
    return np.concatenate([first, _by_distance(row_ptr, col_idx, order, first, order[width:], order[width:])])


def listed_batch_order(row_ptr, col_idx, src, width: int, by_distance: bool):
    """The order (list positions) in which listed-source batches take their
    sources: by their vertex's degree class (a source without arcs with the
    last), positions ascending inside a class; with by_distance and more than
    one batch, the later batches by distance from the first batch's
    highest-degree source, as in allsource_batch_order."""
    rp = np.asarray(row_ptr, np.int64)
    deg = np.diff(rp)[src]
    k = len(src)
    cls = np.where(deg > 64, 0, np.where(deg > 0, 7 - np.floor(np.log2(np.maximum(deg, 1))).astype(np.int64), 7))
    order = np.lexsort((np.arange(k), cls))
    if not by_distance or k <= width:
        return order
    first = order[:width]
    tail = order[width:]
    return np.concatenate([first, _by_distance(row_ptr, col_idx, order, np.asarray(src)[first], np.asarray(src)[tail], tail)])
