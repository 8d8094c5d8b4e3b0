"""Full-size parity in the benchmark's own launch configuration, every
vertex: the config-2 step exactly as bench.py times it (batched ingest of 4
Chung-Lu layers over 100,000 vertices, AND aggregation, all-source closeness
of the 4 layers and the AND graph at W = 4096 with 2-hop counts and levels
per batch, one batched top-10% / CC2 top-10% selection call, the naive
composition), and config 5's exhaustive AND-graph closeness with its top-1%
set (the precision reference of the learned proposer).

The oracle runs one plain BFS per source on the host cores (about 15 s per
10^5-vertex layer on 16 cores), on CSRs it builds itself from the same
seeded edge lists.  Bars (Sec. 4, Eq. 1 with the Wasserman-Faust form):
CSR, S, R, h2, levels and every id set bit-exact; closeness and selection
scores compared as FP64 bit patterns (0 ulp)."""
import numpy as np
import pytest
import torch

import bench
from homln_inputs import configs as C
from oracle import oracle as O
from tests.gpu_common import allsource_batch_order, say

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")

W_BENCH = 4096          # the benchmark's source-batch width


def levels_ref(rp, ci, ecc, width):
    """Per-batch levels: 1 + the largest eccentricity of each batch's sources
    in the all-source batch order (allsource_batch_order)."""
    act = allsource_batch_order(rp, ci, width)
    nb = (len(rp) - 1 + width - 1) // width
    na = (len(act) + width - 1) // width
    return [1 + int(ecc[act[b * width:(b + 1) * width]].max()) for b in range(na)] + [0] * (nb - na)


@pytest.fixture(scope="module")
def cfg2_step():
    """The bench's config-2 step run once on the GPU; host copies of every
    output, plus a cache of the oracle's per-graph results."""
    h = C.config2()
    say("cfg2 bench step: n=%d, W=%d" % (h.n, W_BENCH))
    cs = bench.Cfg2Step(h, W_BENCH)
    cs.step()
    torch.cuda.synchronize()
    P.device_status()
    host = {
        "csr": [(rp.cpu().numpy(), ci.cpu().numpy()) for rp, ci in cs.csr_bufs],
        "and": (cs.and_buf[0].cpu().numpy(), cs.and_buf[1].cpu().numpy()),
        "outs": [{k: v.cpu().numpy() for k, v in o.items()} for o in cs.outs],
        "levels": [lv.cpu().numpy() for lv in cs.levels],
        "sel": [(a.cpu().numpy(), b.cpu().numpy(), int(c.item())) for a, b, c in cs.sel],
    }
    # the oracle's own CSRs from the same edge lists
    layers = [O.csr_from_edges(h.n, eu, ev) for eu, ev in h.layers]
    graphs = layers + [O.compose("and", layers)]
    return dict(h=h, n=h.n, K=cs.K, G=cs.G, L=cs.L, host=host, graphs=graphs, oracle={})


def oracle_of(st, gi):
    if gi not in st["oracle"]:
        rp, ci = st["graphs"][gi]
        say("oracle: graph %d (n=%d, arcs=%d)" % (gi, len(rp) - 1, len(ci)))
        S, R, H2, ecc, _ = O.bfs_sums(rp, ci, extras=True)
        st["oracle"][gi] = dict(S=S, R=R, H2=H2, ecc=ecc, cc=O.closeness_wf(st["n"], S, R))
    return st["oracle"][gi]


@pytest.mark.parametrize("gi", [0, 1, 2, 3, 4], ids=["layer0", "layer1", "layer2", "layer3", "and"])
def test_config2_bench_step_every_vertex(cfg2_step, gi):
    st = cfg2_step
    n = st["n"]
    host = st["host"]
    # the step's CSR (GPU ingest / GPU AND) is the oracle's
    rp, ci = st["graphs"][gi]
    grp, gci = host["and"] if gi == st["L"] else host["csr"][gi]
    nnz = int(grp[n])
    assert np.array_equal(grp, rp), "row_ptr differs"
    assert np.array_equal(gci[:nnz], ci), "col_idx differs"
    ref = oracle_of(st, gi)
    got = host["outs"][gi]
    say("compare graph %d: every vertex" % gi)
    bad = np.nonzero(got["S"] != ref["S"])[0]
    assert len(bad) == 0, ("S", gi, bad[:10])
    assert np.array_equal(got["R"], ref["R"]), ("R", gi)
    assert np.array_equal(got["h2"], ref["H2"]), ("h2", gi)
    assert np.array_equal(got["cc"].view(np.int64), ref["cc"].view(np.int64)), ("cc bits", gi)
    # levels per batch = 1 + the largest eccentricity of the batch's sources
    assert host["levels"][gi].tolist() == levels_ref(rp, ci, ref["ecc"], W_BENCH)


def test_config2_bench_step_selection(cfg2_step):
    """Every graph's top-10% (ids in rank order and score bits), CC2's
    top-10% of the layers and the naive composition (intersection of the
    layers' above-average sets), id for id."""
    st = cfg2_step
    n, K, G, L = st["n"], st["K"], st["G"], st["L"]
    sel = st["host"]["sel"]
    refs = [oracle_of(st, gi) for gi in range(G)]
    for gi in range(G):
        ids, sc, cnt = sel[gi]
        want = O.topk_desc(refs[gi]["cc"], K)
        assert cnt == K
        assert np.array_equal(ids[:K], want), ("top-10%", gi)
        assert np.array_equal(sc[:K].view(np.int64), refs[gi]["cc"][want].view(np.int64)), ("top-10% scores", gi)
    est = O.cc2_est(n, [refs[l]["S"] for l in range(L)], [refs[l]["R"] for l in range(L)])
    want = O.topk_asc_i64(est, K)
    ids, sc, cnt = sel[G]
    assert cnt == K
    assert np.array_equal(ids[:K], want), "CC2 top-10%"
    assert np.array_equal(sc[:K].view(np.int64), O.cc2_score(n, est)[want].view(np.int64)), "CC2 scores"
    naive = O.naive(n, [refs[l]["cc"] for l in range(L)])
    ids, _, cnt = sel[G + 1]
    assert cnt == len(naive)
    assert np.array_equal(ids[:cnt], naive), "naive set"


def test_config5_exhaustive_and_top1pct():
    """Config 5 (5 Chung-Lu layers over 200,000 vertices): the exhaustive
    arm of the proposer benchmark -- GPU ingest, GPU AND, all-source
    closeness of the AND graph at W = 4096, top-1% (K = 2,000) -- against
    the oracle on every vertex and id for id."""
    from paper_2207_11662_amd import proposer as PR
    h = C.config5()
    n = h.n
    k = n // 100
    say("cfg5 exhaustive: n=%d, K=%d" % (n, k))
    layers = PR.upload_homln(h)
    g_and = P.hln_compose_and(layers).trimmed()
    ex = P.hln_closeness_layer(g_and, None, width_bits=W_BENCH)
    ids = P.hln_topk(ex["cc"], k)
    torch.cuda.synchronize()
    P.device_status()
    o_layers = [O.csr_from_edges(n, eu, ev) for eu, ev in h.layers]
    rp, ci = O.compose("and", o_layers)
    assert np.array_equal(g_and.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(g_and.col_idx.cpu().numpy(), ci)
    say("oracle: cfg5 AND graph (arcs=%d)" % len(ci))
    S, R = O.bfs_sums(rp, ci)
    cc = O.closeness_wf(n, S, R)
    assert np.array_equal(ex["S"].cpu().numpy(), S)
    assert np.array_equal(ex["R"].cpu().numpy(), R)
    assert np.array_equal(ex["cc"].cpu().numpy().view(np.int64), cc.view(np.int64))
    assert np.array_equal(ids[:k].cpu().numpy(), O.topk_desc(cc, k))
