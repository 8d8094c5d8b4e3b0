"""Config 4 at full size: 6 R-MAT layers over 1,000,000 vertices and their
AND graph, 16,384 seeded sources per graph, listed-source closeness at
W = 512: the 7 graphs through one batched call (the launch configuration
bench.py times) and one single-graph call each.  Sampled sources are
checked against one oracle BFS each (S, R bit-exact, closeness bit-exact);
R of every source is checked against the connected components; the batched
and single-graph outputs are identical."""
import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from oracle import oracle as O
from tests.gpu_common import csr_np, say, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

P = pytest.importorskip("paper_2207_11662_amd")
from paper_2207_11662_amd import proposer as PR  # noqa: E402


@pytest.fixture(scope="module")
def cfg4():
    h = C.config4(workers=8, progress=lambda s: say(s))
    layers = [csr_np(h.n, *e) for e in h.layers]
    say("host CSR built")
    A = O.compose("and", layers)
    say("AND graph: %d arcs" % len(A[1]))
    return h, layers + [A]


@pytest.mark.timeout(1200)
def test_config4_listed_sources_sampled(cfg4):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    h, host = cfg4
    n = h.n
    dev_layers = PR.upload_homln(h)
    g_and = P.hln_compose_and(dev_layers).trimmed()
    graphs = dev_layers + [g_and]
    srcs = [C.config4_sources(gi, np.diff(rp)) for gi, (rp, _) in enumerate(host)]
    dsrc = [to_dev(s) for s in srcs]
    say("batched call: 7 graphs, listed sources, W = 512")
    plan = P.Plan()
    plan.set_width(n, 512)
    bouts = P.Plan.outputs_listed(graphs, dsrc)
    plan.run(graphs, bouts, sources=dsrc)
    torch.cuda.synchronize()
    P.device_status()
    rng = np.random.default_rng(44)
    for gi, (g, (rp, ci)) in enumerate(zip(graphs, host)):
        assert g.nnz == len(ci)
        src = srcs[gi]
        say("graph", gi, "sources", len(src))
        out = P.hln_closeness_layer(g, sources=dsrc[gi], width_bits=512)
        torch.cuda.synchronize()
        P.device_status()
        for key in ("S", "R", "cc"):
            assert torch.equal(bouts[gi][key], out[key]), (gi, key)
        S_g = out["S"].cpu().numpy()
        R_g = out["R"].cpu().numpy()
        cc_g = out["cc"].cpu().numpy()
        pos = np.sort(rng.choice(len(src), size=160, replace=False))
        S, R = O.bfs_sums(rp, ci, sources=src[pos])
        cc = O.closeness_wf(n, S, R)
        assert np.array_equal(S_g[pos], S), gi
        assert np.array_equal(R_g[pos], R), gi
        assert np.array_equal(cc_g[pos].view(np.int64), cc.view(np.int64)), gi
        adj = sp.csr_matrix((np.ones(len(ci), np.int8), ci, rp), shape=(n, n))
        _, lab = connected_components(adj, directed=False)
        assert np.array_equal(R_g, np.bincount(lab)[lab[src]]), gi


@pytest.mark.timeout(1200)
def test_config4_sample_estimate_sampled(cfg4):
    """Per-vertex sums over each graph's 16,384-source sample and the
    estimate for all 1,000,000 vertices: sampled vertices against one oracle
    BFS each (sums bit-exact, estimate bit-exact through the oracle's
    estimator); over all vertices, the sums add up to the per-source sums of
    the listed-source mode."""
    h, host = cfg4
    n = h.n
    dev_layers = PR.upload_homln(h)
    g_and = P.hln_compose_and(dev_layers).trimmed()
    graphs = dev_layers + [g_and]
    rng = np.random.default_rng(45)
    for gi in (0, 3, 6):
        g, (rp, ci) = graphs[gi], host[gi]
        deg = np.diff(rp)
        src = C.config4_sources(gi, deg)
        n_pop = int((deg > 0).sum())
        say("graph", gi, "sample", len(src), "population", n_pop)
        dsrc = to_dev(src)
        pv = P.hln_closeness_layer(g, sources=dsrc, width_bits=512, per_vertex=True)
        cc = P.hln_closeness_estimate(n, n_pop, dsrc, pv["S"], pv["R"])
        ps = P.hln_closeness_layer(g, sources=dsrc, width_bits=512, want_cc=False)
        torch.cuda.synchronize()
        P.device_status()
        S_g, R_g, cc_g = pv["S"].cpu().numpy(), pv["R"].cpu().numpy(), cc.cpu().numpy()
        assert int(S_g.sum()) == int(ps["S"].sum().item()), gi
        assert int(R_g.sum()) == int(ps["R"].to(torch.int64).sum().item()), gi
        assert R_g.max() <= len(src)
        verts = np.sort(np.concatenate([rng.choice(n, size=20, replace=False), src[:4]])).astype(np.int32)
        SQ, RQ = O.sample_sums_at(rp, ci, src, verts)
        assert np.array_equal(S_g[verts], SQ), gi
        assert np.array_equal(R_g[verts], RQ), gi
        SQf = np.zeros(n, np.int64)
        RQf = np.zeros(n, np.int32)
        SQf[verts], RQf[verts] = SQ, RQ
        exp = O.sample_estimate(n, n_pop, src, SQf, RQf)
        assert np.array_equal(cc_g[verts].view(np.int64), exp[verts].view(np.int64)), gi
