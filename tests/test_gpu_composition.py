"""Composition study (f1) and subset sweep (f2) on the GPU: every CC-node
set the study scores is the oracle's, element for element."""
import itertools

import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from oracle import oracle as O
from tests.gpu_common import csr_np, say

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")
from paper_2207_11662_amd import composition as CM  # noqa: E402
from paper_2207_11662_amd import proposer as PR  # noqa: E402


def oracle_sets(n, layers_np, subset, k):
    Ls = [layers_np[i] for i in subset]
    A = O.compose("and", Ls)
    _, _, cc = O.closeness_all(*A)
    truth = (np.sort(O.above_mean(cc)), O.topk_desc(cc, k))
    SR = [O.closeness_all(*g) for g in Ls]
    est = O.cc2_est(n, [x[0] for x in SR], [x[1] for x in SR])
    sc = O.cc2_score(n, est)
    cc2 = (np.sort(O.above_mean(sc)), O.topk_desc(sc, k))
    naive = np.sort(O.naive(n, [x[2] for x in SR]))
    cc1 = O.cc1(n, Ls, [x[0] for x in SR], [x[1] for x in SR], (1, 2))
    return truth, cc2, naive, cc1


def test_study_sets_match_oracle_config1():
    h = C.config1()
    n = h.n
    layers_np = [csr_np(n, *e) for e in h.layers]
    k = int(np.ceil(0.1 * n))
    plan = P.Plan()
    layers = PR.upload_homln(h)
    outs = PR.psi(plan, layers)
    ws = P.workspace(int(P.lib().hln_compose_cc_topk_workspace_size(n)))
    subsets = [(0, 1, 2), (0, 1), (0, 2), (1, 2)]
    recs = CM.study_homln(h, k_frac=0.1, pairs=True, plan=plan)
    assert [tuple(r["subset"]) for r in recs] == subsets
    for sub, rec in zip(subsets, recs):
        truth, cc2, naive, cc1 = oracle_sets(n, layers_np, sub, k)
        g_and = P.hln_compose_and([layers[i] for i in sub]).trimmed()
        gt = P.Plan.outputs([g_and])
        plan.run([g_and], gt)
        t_above, t_top = CM.cc_sets(P.HLN_RANK_WF, n, [gt[0]["S"]], [gt[0]["R"]], k, ws)
        c_above, c_top = CM.cc_sets(P.HLN_RANK_CC2, n, [outs[i]["S"] for i in sub], [outs[i]["R"] for i in sub], k, ws)
        assert np.array_equal(np.sort(t_above), truth[0]) and np.array_equal(t_top, truth[1])
        assert np.array_equal(np.sort(c_above), cc2[0]) and np.array_equal(c_top, cc2[1])
        assert rec["cc2_above"] == CM.set_metrics(cc2[0], truth[0])
        assert rec["cc2_topk"] == CM.set_metrics(cc2[1], truth[1])
        assert rec["naive_above"] == CM.set_metrics(naive, truth[0])
        assert rec["cc1_above"] == CM.set_metrics(cc1, truth[0])
        say("subset", sub, "cc2 top-k jaccard %.3f, naive above jaccard %.3f"
            % (rec["cc2_topk"]["jaccard"], rec["naive_above"]["jaccard"]))


@pytest.mark.parametrize("width", [512, 4096])
def test_subsets_sweep_small(width):
    """Also checks, inside the sweep, that the batched AND ground truths (all
    subsets through one plan call: one launch per graph at 512, the
    partitioned multi-graph launch at 4096) give every subset's top-k set."""
    h = C.config2(scale=0.02)
    res = CM.subsets_sweep(h, k_frac=0.05, width_bits=width)
    assert res["subsets"] == 2 ** 4 - 4 - 1
    assert all(r["t_and_gt_ms"] > 0 and r["t_theta_ms"] > 0 for r in res["records"])
    assert res["t_and_gt_batched_ms"] > 0
    # the sweep's CC2 scores agree with the oracle on one subset
    n = h.n
    layers_np = [csr_np(n, *e) for e in h.layers]
    k = res["k"]
    sub = (0, 2, 3)
    truth, cc2, _, cc1 = oracle_sets(n, layers_np, sub, k)
    rec = [r for r in res["records"] if tuple(r["subset"]) == sub][0]
    assert rec["cc2_topk"] == CM.set_metrics(cc2[1], truth[1])
    assert rec["cc1_above"] == CM.set_metrics(cc1, truth[0])
    say("speedup of the decoupled method", res["speedup_decoupled"])
