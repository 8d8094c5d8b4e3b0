"""Learned candidate proposer for the CC nodes of an AND aggregate.

The exact answer needs one BFS per vertex of the AND graph (Sec. 4).  The
proposer ranks vertices with a small FP32 MLP over per-layer quantities the
Psi step has already produced (degree, closeness and 2-hop count: the
signals CC1 and CC2 build on, Sec. 5.1-5.2), keeps the best `budget` fraction as
candidates, runs exact per-source BFS on the AND graph for those only, and
returns the best of them by exact closeness.  Every step is a kernel of
``libhln.so``; this module only sequences the calls.  The method itself is
not in the paper: it is an accelerator whose answers are exact closeness
values of real vertices, with the exhaustive computation as the fallback
and the reference its precision is measured against.

Training data: for each HoMLN, features from its layers and labels from
the exact closeness of its AND graph (log-rank, 1 = most central).
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


def upload_homln(h, stream=None):
    """Device CSR layers of a HoMLN (edge lists through the ingest kernels)."""
    items = [(h.n, torch.from_numpy(np.ascontiguousarray(eu, dtype=np.int32)).cuda(),
              torch.from_numpy(np.ascontiguousarray(ev, dtype=np.int32)).cuda()) for eu, ev in h.layers]
    return [g.trimmed() for g in L.hln_csr_from_edges_batch(items, stream=stream)]


def psi(plan: L.Plan, graphs, stream=None):
    """All-source closeness and 2-hop counts of each graph (batched)."""
    outs = L.Plan.outputs(graphs, want_h2=True)
    plan.run(graphs, outs, stream=stream)
    return outs


def features(layers, psi_outs, X=None, stream=None):
    return L.hln_proposer_features(layers, [o["S"] for o in psi_outs], [o["R"] for o in psi_outs],
                                   [o["h2"] for o in psi_outs], X=X, stream=stream)


def training_example(plan: L.Plan, h, stream=None):
    """(X [n, 12] float32, label [n] float32) of one HoMLN."""
    layers = upload_homln(h, stream)
    g_and = L.hln_compose_and(layers, stream=stream).trimmed()
    outs = psi(plan, layers + [g_and], stream)
    X = features(layers, outs[:-1], stream=stream)
    lab = L.hln_rank_labels(outs[-1]["cc"], stream=stream)
    return X, lab


class Proposer:
    """FP32 MLP parameters and Adam state on the device."""

    def __init__(self, seed: int = 0, device: str = "cuda"):
        npar = L.mlp_param_count()
        self.params = torch.empty(npar, dtype=torch.float32, device=device)
        self.m = torch.empty_like(self.params)
        self.v = torch.empty_like(self.params)
        L.hln_mlp_init(self.params, self.m, self.v, seed=seed)
        self.step = 0
        self.history = []

    def fit(self, X: torch.Tensor, label: torch.Tensor, steps: int = 3000, lr: float = 2e-3,
            batch: int = 65536, seed: int = 0, log_every: int = 0):
        """Adam on mean squared error over contiguous minibatches of one
        seeded shuffle of the rows; the learning rate is halved at 50%,
        75% and 90% of the steps."""
        n = X.shape[0]
        perm = torch.from_numpy(np.random.default_rng(seed).permutation(n)).to(X.device)
        Xs = X.index_select(0, perm).contiguous()
        ys = label.index_select(0, perm).contiguous()
        batch = min(batch, n)
        nb = max(1, n // batch)
        loss = torch.zeros(1, dtype=torch.float32, device=X.device)
        ws = None
        for s in range(steps):
            b = s % nb
            rate = lr * (0.5 ** sum(s >= f * steps for f in (0.5, 0.75, 0.9)))
            self.step += 1
            ws = L.hln_mlp_train_step(self.params, self.m, self.v, self.step, rate,
                                      Xs[b * batch:(b + 1) * batch], ys[b * batch:(b + 1) * batch],
                                      loss=loss, ws=ws)
            if log_every and (s % log_every == 0 or s == steps - 1):
                self.history.append((s, float(loss.item())))
        return self

    def score(self, X: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        return L.hln_mlp_forward(self.params, X, out, stream=stream)


class Query:
    """Preallocated buffers for the proposer arm on one AND graph:
    features -> MLP scores -> top `n_cand` -> exact per-source BFS on the
    AND graph -> top `k` by exact closeness."""

    def __init__(self, g_and: L.Graph, n_cand: int, k: int, width_bits: int = 4096):
        dev = g_and.row_ptr.device
        n = g_and.n
        self.g, self.n_cand, self.k, self.width = g_and, n_cand, k, width_bits
        self.X = torch.empty((n, 12), dtype=torch.float32, device=dev)
        self.y = torch.empty(n, dtype=torch.float32, device=dev)
        self.cand = torch.empty(max(n_cand, 1), dtype=torch.int32, device=dev)
        self.pos = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
        self.ws_topk = L.workspace(int(L.lib().hln_topk_workspace_size(n)), dev)
        self.bfs = {"S": torch.empty(n_cand, dtype=torch.int64, device=dev),
                    "R": torch.empty(n_cand, dtype=torch.int32, device=dev),
                    "cc": torch.empty(n_cand, dtype=torch.float64, device=dev), "h2": None}
        self.ws_bfs = L.workspace(L.closeness_workspace_size(n, g_and.nnz, n_cand, width_bits), dev)

    def features(self, layers, psi_outs, stream=None):
        features(layers, psi_outs, X=self.X, stream=stream)

    def candidates_from(self, score: torch.Tensor, stream=None):
        """The n_cand best-scored vertices, as ascending ids."""
        L.hln_topk(score, self.n_cand, ids=self.cand, ws=self.ws_topk, stream=stream, as_set=True)

    def refine(self, stream=None):
        """Exact closeness of the candidates on the AND graph, then their
        top k (positions into the candidate list in self.pos).  The
        candidates are in ascending id order, so ties in exact closeness
        are broken by vertex id, as in the exhaustive ranking."""
        L.hln_closeness_layer(self.g, self.cand[:self.n_cand], width_bits=self.width, out=self.bfs,
                              ws=self.ws_bfs, stream=stream)
        L.hln_topk(self.bfs["cc"], self.k, ids=self.pos, ws=self.ws_topk, stream=stream)

    def run(self, proposer: Proposer, layers, psi_outs, stream=None):
        self.features(layers, psi_outs, stream)
        proposer.score(self.X, self.y, stream)
        self.candidates_from(self.y, stream)
        self.refine(stream)

    def result(self):
        """(vertex ids, exact closeness) of the answer, on the host."""
        cand = self.cand[:self.n_cand].cpu().numpy()
        pos = self.pos[:self.k].cpu().numpy()
        return cand[pos], self.bfs["cc"].cpu().numpy()[pos]
