"""Parity of hln_compose_cc_topk (CC-node selection, CC2 and naive
composition) with the CPU oracle: id lists identical (ties by id), scores
bit-exact."""
import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from oracle import oracle as O
from tests.gpu_common import csr_np, graph_dev, say, to_dev

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")


def select(mode, n, S_list, R_list, k):
    Sd = [to_dev(s, torch.int64) for s in S_list]
    Rd = [to_dev(r, torch.int32) for r in R_list]
    ids, score, count = P.hln_compose_cc_topk(mode, n, Sd, Rd, k)
    torch.cuda.synchronize()
    P.device_status()
    c = int(count.item())
    return ids[:c].cpu().numpy(), score[:c].cpu().numpy()


def synthetic_sums(rng, n, ties):
    """Random (S, R) pairs that a graph could produce, with many exact ties
    when `ties` (closeness values repeat)."""
    R = rng.integers(1, n + 1, size=n).astype(np.int32)
    if ties:
        R = rng.choice([1, n // 2 + 1, n], size=n).astype(np.int32)
    S = np.where(R > 1, R - 1 + rng.integers(0, 3 * n, size=n) * (0 if ties else 1), 0).astype(np.int64)
    if ties:
        S = np.where(R > 1, (R - 1) * rng.choice([1, 2, 3], size=n), 0).astype(np.int64)
    return S, R


@pytest.mark.parametrize("ties", [False, True])
def test_wf_topk_and_above_mean(ties):
    rng = np.random.default_rng(5 + ties)
    for n in (1, 2, 7, 1023, 1024, 1025, 5000):
        S, R = synthetic_sums(rng, n, ties)
        cc = O.closeness_wf(n, S, R)
        for k in sorted({0, 1, min(10, n), n // 3, n}):
            say("wf", n, k, ties)
            ids, sc = select(P.HLN_RANK_WF, n, [S], [R], k)
            ref = O.topk_desc(cc, k)
            assert np.array_equal(ids, ref)
            assert np.array_equal(sc.view(np.int64), cc[ref].view(np.int64))
        ids, sc = select(P.HLN_RANK_WF, n, [S], [R], -1)
        assert np.array_equal(ids, O.above_mean(cc))


@pytest.mark.parametrize("ties", [False, True])
def test_cc2_and_naive(ties):
    rng = np.random.default_rng(11 + ties)
    for n in (3, 500, 4097):
        r = int(rng.integers(2, 6))
        sums = [synthetic_sums(rng, n, ties) for _ in range(r)]
        S_list = [s for s, _ in sums]
        R_list = [x for _, x in sums]
        est = O.cc2_est(n, S_list, R_list)
        score = O.cc2_score(n, est)
        for k in (0, 1, n // 10, n):
            say("cc2", n, r, k)
            ids, sc = select(P.HLN_RANK_CC2, n, S_list, R_list, k)
            ref = O.topk_asc_i64(est, k)
            assert np.array_equal(ids, ref)
            assert np.array_equal(sc.view(np.int64), score[ref].view(np.int64))
        ids, _ = select(P.HLN_RANK_CC2, n, S_list, R_list, -1)
        assert np.array_equal(ids, O.above_mean(score))
        ccs = [O.closeness_wf(n, s, x) for s, x in sums]
        ids, _ = select(P.HLN_RANK_NAIVE, n, S_list, R_list, -1)
        assert np.array_equal(ids, O.naive(n, ccs))
        for k in (0, 1, n // 10, n // 2, n):
            say("naive top-k", n, r, k)
            ids, sc = select(P.HLN_RANK_NAIVE, n, S_list, R_list, k)
            assert np.array_equal(ids, O.naive_topk(n, ccs, k)), k
            assert np.all(sc == 0.0)


def test_end_to_end_config1():
    """HIP closeness -> HIP selection against oracle closeness -> oracle
    selection, on config 1's layers and AND graph (top-10%, K = ceil(0.1 n))."""
    h = C.config1()
    n = h.n
    k = O.topk_count(n, 1, 10)
    layers = [csr_np(n, *e) for e in h.layers]
    A = O.compose("and", layers)
    outs, refs = [], []
    for rp, ci in layers + [A]:
        g = graph_dev(P, rp, ci)
        outs.append(P.hln_closeness_layer(g, width_bits=512))
        refs.append(O.bfs_sums(rp, ci))
    torch.cuda.synchronize()
    for o, (S, R) in zip(outs, refs):
        ids, _, count = P.hln_compose_cc_topk(P.HLN_RANK_WF, n, [o["S"]], [o["R"]], k)
        torch.cuda.synchronize()
        assert np.array_equal(ids[: int(count.item())].cpu().numpy(), O.topk_desc(O.closeness_wf(n, S, R), k))
    ids, _, count = P.hln_compose_cc_topk(P.HLN_RANK_CC2, n, [o["S"] for o in outs[:3]], [o["R"] for o in outs[:3]], k)
    torch.cuda.synchronize()
    est = O.cc2_est(n, [S for S, _ in refs[:3]], [R for _, R in refs[:3]])
    assert np.array_equal(ids[: int(count.item())].cpu().numpy(), O.topk_asc_i64(est, k))


def batch_problems(seed, count, nmax):
    """Mixed WF and CC2 problems (with and without ties, k from 0 to n)."""
    rng = np.random.default_rng(seed)
    probs = []
    for p in range(count):
        n = int(rng.integers(1, nmax))
        ties = bool(p % 2)
        if p % 3 == 0:
            S, R = synthetic_sums(rng, n, ties)
            cc = O.closeness_wf(n, S, R)
            k = int(rng.choice([0, 1, max(n // 10, 0), n]))
            probs.append((P.HLN_RANK_WF, n, [S], [R], k, O.topk_desc(cc, k), cc))
        else:
            r = int(rng.integers(1, 5))
            sums = [synthetic_sums(rng, n, ties) for _ in range(r)]
            est = O.cc2_est(n, [s for s, _ in sums], [x for _, x in sums])
            k = int(rng.choice([0, 1, max(n // 10, 0), n]))
            probs.append((P.HLN_RANK_CC2, n, [s for s, _ in sums], [x for _, x in sums], k, O.topk_asc_i64(est, k),
                          O.cc2_score(n, est)))
    return probs


def check_topk_batch(probs, outs, tag):
    for i, ((mode, n, S_list, R_list, k, ref, score), (ids, sc, cnt)) in enumerate(zip(probs, outs)):
        c = int(cnt.item())
        assert c == k, (tag, i)
        assert np.array_equal(ids[:c].cpu().numpy(), ref), (tag, i, mode, n, k)
        assert np.array_equal(sc[:c].cpu().numpy().view(np.int64), score[ref].view(np.int64)), (tag, i)


def test_topk_batch_against_oracle_and_single_calls():
    """Forty problems of mixed modes and sizes (n from 1 to 6,000, k from 0
    to n, ties) in one call: every problem against the oracle, and against
    the one-problem call bit for bit."""
    probs = batch_problems(21, 40, 6000)
    dev_probs = [(mode, n, [to_dev(s, torch.int64) for s in S], [to_dev(x, torch.int32) for x in R], k)
                 for mode, n, S, R, k, _, _ in probs]
    outs = P.hln_compose_cc_topk_batch(dev_probs)
    torch.cuda.synchronize()
    P.device_status()
    check_topk_batch(probs, outs, "batch")
    for (mode, n, S, R, k), (ids, sc, cnt) in zip(dev_probs, outs):
        i1, s1, c1 = P.hln_compose_cc_topk(mode, n, S, R, k)
        torch.cuda.synchronize()
        assert int(c1.item()) == int(cnt.item())
        assert torch.equal(i1[:k].cpu(), ids[:k].cpu()) and torch.equal(s1[:k].cpu(), sc[:k].cpu())


def test_topk_batch_captured_and_repeated():
    probs = batch_problems(23, 30, 3000)
    dev_probs = [(mode, n, [to_dev(s, torch.int64) for s in S], [to_dev(x, torch.int32) for x in R], k)
                 for mode, n, S, R, k, _, _ in probs]
    tb = P.TopkBatch(dev_probs)
    tb.run()
    torch.cuda.synchronize()
    check_topk_batch(probs, tb.outs, "eager")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        tb.run()
    for rep in range(2):
        for ids, sc, cnt in tb.outs:
            ids.fill_(-3)
            sc.fill_(-3.0)
            cnt.fill_(-3)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        P.device_status()
        check_topk_batch(probs, tb.outs, "replay%d" % rep)


def test_topk_batch_errors():
    L = P.lib()
    assert L.hln_compose_cc_topk_batch(None, 0, None, 0, None) == 0
    assert L.hln_compose_cc_topk_batch(None, 1, None, 0, None) == 1
    S = [torch.zeros(10, dtype=torch.int64, device="cuda")] * 2
    R = [torch.ones(10, dtype=torch.int32, device="cuda")] * 2
    for bad in [(P.HLN_RANK_NAIVE, 10, S, R, 2), (P.HLN_RANK_WF, 10, S, R, 2), (P.HLN_RANK_CC2, 10, S, R, 11),
                (P.HLN_RANK_CC2, 10, S, R, -1), (P.HLN_RANK_CC2, 0, S, R, 0)]:
        with pytest.raises(P.HlnError):
            P.hln_compose_cc_topk_batch([(P.HLN_RANK_CC2, 10, S, R, 3), bad])
    tb = P.TopkBatch([(P.HLN_RANK_CC2, 10, S, R, 3)])
    small = torch.zeros(256, dtype=torch.uint8, device="cuda")
    assert L.hln_compose_cc_topk_batch(tb.arr, 1, P._lib._ptr(small), 256, None) == 2
