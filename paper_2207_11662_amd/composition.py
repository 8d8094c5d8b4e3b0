"""Composition accuracy and the all-subsets sweep (Theta step, Sec. 4-5).

The decoupling method analyses every layer once (Psi: all-source closeness,
per-layer S and R) and then estimates the CC nodes of any layer subset's AND
aggregate from those per-layer results alone (Theta).  This module measures
how well it does:

* `study_subset`: for one layer subset, the ground truth (AND aggregate,
  exact closeness, Sec. 4) against CC2 (Sec. 5.2, Algorithm 1), CC1 (Sec.
  5.1, Eq. 2-3; a CC-node set, no ranking) and the naive composition
  (intersection of the layers' CC-node sets, Sec. 4), for the above-average
  CC-node sets and, for CC2 and naive, the top-k sets.  Scores: Jaccard
  coefficient (the paper's "accuracy"), precision, recall and F1 (Sec. 5,
  Sec. 6.1).
* `subsets_sweep`: Psi once, then every subset of two or more layers; the
  per-subset ground truth (AND, and OR as the alternative aggregation) is
  timed against the per-subset Theta (Sec. 6.1 performance argument: the
  layer analysis is reused for exponentially many subsets).

Every closeness value, aggregate, score and selection comes from the
library's kernels; only the set comparison runs on the host.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

from . import _lib as L
from .proposer import psi, upload_homln


def set_metrics(pred, truth) -> dict:
    """Jaccard, precision, recall and F1 of a predicted vertex set against
    the true one (empty sets score 1 when both are empty, else 0)."""
    a = set(int(x) for x in pred)
    b = set(int(x) for x in truth)
    inter = len(a & b)
    union = len(a | b)
    p = inter / len(a) if a else float(not b)
    r = inter / len(b) if b else float(not a)
    return {"jaccard": inter / union if union else 1.0, "precision": p, "recall": r,
            "f1": 2 * p * r / (p + r) if p + r > 0 else 0.0, "pred": len(a), "true": len(b)}


def _ids(out) -> np.ndarray:
    ids, _, count = out
    c = int(count.item())
    return ids[:c].cpu().numpy()


def cc_sets_dev(mode: int, n: int, S_list, R_list, k: int, ws=None):
    """Device outputs of the above-average and top-k selections of one
    ranking mode (HLN_RANK_WF for one graph, HLN_RANK_CC2 for a layer
    subset); no synchronisation."""
    above = L.hln_compose_cc_topk(mode, n, S_list, R_list, -1, ws=ws)
    top = L.hln_compose_cc_topk(mode, n, S_list, R_list, k, ws=ws)
    return above, top


def cc_sets(mode: int, n: int, S_list, R_list, k: int, ws=None):
    """(above-average ids, top-k ids) on the host."""
    above, top = cc_sets_dev(mode, n, S_list, R_list, k, ws)
    return _ids(above), _ids(top)


def study_subset(n: int, layer_graphs, layer_outs, subset, k: int, plan: L.Plan, ws=None, cc1_tau=(1, 2)) -> dict:
    """Ground truth, CC2, CC1 and naive CC-node sets of one layer subset."""
    gs = [layer_graphs[i] for i in subset]
    Ss = [layer_outs[i]["S"] for i in subset]
    Rs = [layer_outs[i]["R"] for i in subset]
    g_and = L.hln_compose_and(gs).trimmed()
    gt = L.Plan.outputs([g_and])
    plan.run([g_and], gt)
    t_above, t_top = cc_sets(L.HLN_RANK_WF, n, [gt[0]["S"]], [gt[0]["R"]], k, ws)
    c_above, c_top = cc_sets(L.HLN_RANK_CC2, n, Ss, Rs, k, ws)
    naive_above = _ids(L.hln_compose_cc_topk(L.HLN_RANK_NAIVE, n, Ss, Rs, -1, ws=ws))
    # naive top-k: the intersection of the layers' top-k sets (the naive rule
    # applied to top-k sets; it can hold fewer than k vertices)
    naive_top = _ids(L.hln_compose_cc_topk(L.HLN_RANK_NAIVE, n, Ss, Rs, k, ws=ws))
    ids1, cnt1, _ = L.hln_compose_cc1(gs, Ss, Rs, cc1_tau)
    cc1_above = ids1[:int(cnt1.item())].cpu().numpy()
    return {"subset": list(subset), "and_arcs": int(g_and.nnz),
            "cc2_above": set_metrics(c_above, t_above), "cc2_topk": set_metrics(c_top, t_top),
            "cc1_above": set_metrics(cc1_above, t_above),
            "naive_above": set_metrics(naive_above, t_above), "naive_topk": set_metrics(naive_top, t_top)}


def study_homln(h, k_frac: float = 0.1, pairs: bool = True, plan: L.Plan | None = None) -> list:
    """f1 on one HoMLN: all layers together and, if `pairs`, every pair."""
    plan = plan or L.Plan()
    layers = upload_homln(h)
    outs = psi(plan, layers)
    k = max(1, int(np.ceil(k_frac * h.n)))
    ws = L.workspace(int(L.lib().hln_compose_cc_topk_workspace_size(h.n)), layers[0].row_ptr.device)
    subsets = [tuple(range(len(layers)))]
    if pairs and len(layers) > 2:
        subsets += list(itertools.combinations(range(len(layers)), 2))
    return [study_subset(h.n, layers, outs, s, k, plan, ws) for s in subsets]


def summarise(records) -> dict:
    """Mean of each score over a list of study_subset records."""
    out = {}
    for key in ("cc2_above", "cc2_topk", "cc1_above", "naive_above", "naive_topk"):
        out[key] = {m: float(np.mean([r[key][m] for r in records])) for m in ("jaccard", "precision", "recall", "f1")}
    out["subsets"] = len(records)
    return out


def batched_and_truth(layers, subsets, k: int, width_bits: int = 4096) -> dict:
    """The AND ground truths of all subsets at once: every subset's AND
    graph (one batched composition call), then the closeness of all of them
    through one plan call (graphs above the LDS-tile limit share one
    partitioned persistent launch) and their top-k sets through one batched
    selection call; timed as a whole with HIP events.  Returns the time and
    each subset's top-k ids."""
    dev = layers[0].row_ptr.device
    n = layers[0].n
    ands = L.AndBatch([[layers[i] for i in sub] for sub in subsets])
    graphs = [L.Graph(rp, ci, ci.numel()) for rp, ci in ands.outs]
    plan = L.Plan()
    plan.set_width(n, width_bits)
    outs = L.Plan.outputs(graphs)
    bws = L.workspace(plan.workspace_size(graphs), dev)
    sel = L.TopkBatch([(L.HLN_RANK_WF, n, [o["S"]], [o["R"]], k) for o in outs])

    def run():
        ands.run()
        plan.run(graphs, outs, ws=bws)
        sel.run()

    run()                                   # warm-up
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    run()
    b.record()
    torch.cuda.synchronize()
    L.device_status()
    return {"t_ms": a.elapsed_time(b), "topk": [ids[:k].cpu().numpy() for ids, _, _ in sel.outs]}


def subsets_sweep(h, k_frac: float = 0.01, width_bits: int = 4096, with_or: bool = True) -> dict:
    """f2: Psi once, then every subset of >= 2 layers.  Times (HIP events on
    the current stream): Psi (all-source closeness of every layer), per
    subset the AND ground truth (aggregation + all-source closeness) and the
    OR ground truth, and per subset Theta (CC2 top-k and above-average from
    the layers' S and R)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    n = h.n
    k = max(1, int(np.ceil(k_frac * n)))
    layers = upload_homln(h)
    torch.cuda.synchronize()
    nl = len(layers)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    ws_sel = L.workspace(int(L.lib().hln_compose_cc_topk_workspace_size(n)), dev)
    ws_cc1 = L.workspace(int(L.lib().hln_compose_cc1_workspace_size(n, nl)), dev)
    cc1_out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(1, dtype=torch.int32, device=dev),
               torch.empty(1, dtype=torch.float64, device=dev))
    nnz_max = sum(g.nnz for g in layers)
    ws_cl = L.workspace(L.closeness_workspace_size(n, nnz_max, n, width_bits), dev)
    outs = [{"S": torch.empty(n, dtype=torch.int64, device=dev), "R": torch.empty(n, dtype=torch.int32, device=dev),
             "cc": None, "h2": None} for _ in range(nl)]
    a, b = ev(), ev()
    a.record()
    for g, o in zip(layers, outs):
        L.hln_closeness_layer(g, width_bits=width_bits, want_cc=False, out=o, ws=ws_cl)
    b.record()
    torch.cuda.synchronize()
    L.device_status()
    t_psi = a.elapsed_time(b)
    gt_out = {"S": torch.empty(n, dtype=torch.int64, device=dev), "R": torch.empty(n, dtype=torch.int32, device=dev),
              "cc": None, "h2": None}
    recs = []
    for r in range(2, nl + 1):
        for sub in itertools.combinations(range(nl), r):
            gs = [layers[i] for i in sub]
            # buffers of this subset, allocated before the timed regions
            cap_and = min(g.nnz for g in gs)
            and_buf = (torch.empty(n + 1, dtype=torch.int32, device=dev), torch.empty(cap_and, dtype=torch.int32, device=dev))
            ws_cmp = L.workspace(L.compose_workspace_size(gs), dev)
            e = [ev() for _ in range(6)]
            e[0].record()
            g_and = L.hln_compose_and(gs, ws=ws_cmp, out=and_buf)
            L.hln_closeness_layer(g_and, width_bits=width_bits, want_cc=False, out=gt_out, ws=ws_cl)
            t_dev = cc_sets_dev(L.HLN_RANK_WF, n, [gt_out["S"]], [gt_out["R"]], k, ws_sel)
            e[1].record()
            c_dev = cc_sets_dev(L.HLN_RANK_CC2, n, [outs[i]["S"] for i in sub], [outs[i]["R"] for i in sub], k, ws_sel)
            e[2].record()
            L.hln_compose_cc1(gs, [outs[i]["S"] for i in sub], [outs[i]["R"] for i in sub], ws=ws_cc1, out=cc1_out)
            e[5].record()
            torch.cuda.synchronize()
            L.device_status()
            rec = {"subset": list(sub), "t_and_gt_ms": e[0].elapsed_time(e[1]), "t_theta_ms": e[1].elapsed_time(e[2]),
                   "t_theta_cc1_ms": e[2].elapsed_time(e[5])}
            t_sets = (_ids(t_dev[0]), _ids(t_dev[1]))
            c_sets = (_ids(c_dev[0]), _ids(c_dev[1]))
            rec["cc2_above"] = set_metrics(c_sets[0], t_sets[0])
            rec["cc2_topk"] = set_metrics(c_sets[1], t_sets[1])
            rec["cc1_above"] = set_metrics(cc1_out[0][:int(cc1_out[1].item())].cpu().numpy(), t_sets[0])
            del and_buf, ws_cmp
            if with_or:
                cap_or = sum(g.nnz for g in gs)
                or_buf = (torch.empty(n + 1, dtype=torch.int32, device=dev), torch.empty(cap_or, dtype=torch.int32, device=dev))
                ws_cmp = L.workspace(L.compose_workspace_size(gs), dev)
                e[3].record()
                g_or = L.hln_compose_or(gs, ws=ws_cmp, out=or_buf)
                L.hln_closeness_layer(g_or, width_bits=width_bits, want_cc=False, out=gt_out, ws=ws_cl)
                o_dev = cc_sets_dev(L.HLN_RANK_WF, n, [gt_out["S"]], [gt_out["R"]], k, ws_sel)
                e[4].record()
                torch.cuda.synchronize()
                L.device_status()
                rec["t_or_gt_ms"] = e[3].elapsed_time(e[4])
                rec["or_vs_and_topk"] = set_metrics(_ids(o_dev[1]), t_sets[1])
                del or_buf, ws_cmp
            rec["_gt_topk"] = t_sets[1]
            recs.append(rec)
    batched = batched_and_truth(layers, [x["subset"] for x in recs], k, width_bits)
    for x, ids in zip(recs, batched.pop("topk")):
        assert np.array_equal(ids, x.pop("_gt_topk")), "batched AND ground truth differs"
    t_gt = sum(x["t_and_gt_ms"] for x in recs)
    t_theta = sum(x["t_theta_ms"] for x in recs)
    return {"layers": nl, "subsets": len(recs), "k": k, "t_psi_ms": t_psi, "t_and_gt_total_ms": t_gt,
            "t_theta_total_ms": t_theta, "speedup_decoupled": t_gt / (t_psi + t_theta),
            "t_and_gt_batched_ms": batched["t_ms"],
            "speedup_decoupled_vs_batched_gt": batched["t_ms"] / (t_psi + t_theta),
            "t_theta_cc1_total_ms": sum(x["t_theta_cc1_ms"] for x in recs),
            "cc1_above_mean": {m: float(np.mean([x["cc1_above"][m] for x in recs])) for m in ("jaccard", "precision", "f1")},
            "t_or_gt_total_ms": sum(x.get("t_or_gt_ms", 0.0) for x in recs) if with_or else None,
            "cc2_topk_mean": {m: float(np.mean([x["cc2_topk"][m] for x in recs])) for m in ("jaccard", "precision", "f1")},
            "cc2_above_mean": {m: float(np.mean([x["cc2_above"][m] for x in recs])) for m in ("jaccard", "precision", "f1")},
            "records": recs}
