"""The batched step of config 3, end to end and captured as the bench
captures it (batched ingest + batched AND + LDS-tile graphs, the persistent graphs
through a second plan pinned to the same widths, batched CC2 top-10%), on
eight HoMLNs at a tenth of config 3's sizes, replayed twice: every CSR, AND
graph, S, R, closeness and CC2 top-10% set against the CPU oracle."""
import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from oracle import oracle as O
from tests.gpu_common import say

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")


def build_step(hs, tuned):
    """The bench's config-3 step over the HoMLNs hs: three callables (batched
    ingest + batched AND + tile graphs; the persistent graphs through a plan
    pinned to the same widths; batched CC2 top-k) and their buffers.  tuned:
    widths from the autotuner (as the bench); else the largest size class is
    sent to the persistent kernel and the rest to tiles."""
    dev = torch.device("cuda")
    items, ing_items, ing_outs, all_graphs = [], [], [], []
    for h in hs:
        n = h.n
        lay = [(torch.from_numpy(eu.astype(np.int32)).to(dev), torch.from_numpy(ev.astype(np.int32)).to(dev))
               for eu, ev in h.layers]
        bufs = [(torch.empty(n + 1, dtype=torch.int32, device=dev), torch.empty(max(2 * len(eu), 1), dtype=torch.int32,
                                                                                 device=dev)) for eu, _ in lay]
        ms = [len(eu) for eu, _ in lay]
        abuf = (torch.empty(n + 1, dtype=torch.int32, device=dev),
                torch.empty(max(1, min(2 * m for m in ms)), dtype=torch.int32, device=dev))
        graphs = [P.Graph(rp, ci, 2 * m) for (rp, ci), m in zip(bufs, ms)]
        gand = P.Graph(abuf[0], abuf[1], abuf[1].numel())
        ing_items += [(n, eu, ev) for eu, ev in lay]
        ing_outs += bufs
        all_graphs += graphs + [gand]
        items.append(dict(h=h, n=n, graphs=graphs, abuf=abuf, k=(n + 9) // 10, nl=len(lay),
                          sel=(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.float64, device=dev),
                               torch.empty(1, dtype=torch.int32, device=dev))))
    iws = P.workspace(P.csr_from_edges_batch_workspace_size(ing_items))

    ands = P.AndBatch([it["graphs"] for it in items], outs=[it["abuf"] for it in items])

    def ingest_compose():
        P.hln_csr_from_edges_batch(ing_items, ws=iws, outs=ing_outs)
        ands.run()

    outs = P.Plan.outputs(all_graphs, want_h2=False)
    ingest_compose()
    torch.cuda.synchronize()
    plan = P.Plan()
    if tuned:
        plan.tune(all_graphs, outs)
    else:
        # the largest size class goes to the persistent kernel, the rest to tiles
        plan.set_width(max(g.n for g in all_graphs), 4096)
    coop = [i for i, g in enumerate(all_graphs) if plan.width(g.n) >= 512]
    tile = [i for i, g in enumerate(all_graphs) if plan.width(g.n) < 512]
    assert coop and tile
    plan_c = P.Plan()
    for i in coop:
        plan_c.set_width(all_graphs[i].n, plan.width(all_graphs[i].n))
    tg, to = [all_graphs[i] for i in tile], [outs[i] for i in tile]
    cg, co = [all_graphs[i] for i in coop], [outs[i] for i in coop]
    bws = P.workspace(max(plan.workspace_size(tg), plan_c.workspace_size(cg)))
    plan.reserve(tg)
    plan_c.reserve(cg)
    probs, o = [], 0
    for it in items:
        probs.append((P.HLN_RANK_CC2, it["n"], [outs[o + i]["S"] for i in range(it["nl"])],
                      [outs[o + i]["R"] for i in range(it["nl"])], it["k"]))
        o += it["nl"] + 1
    topk = P.TopkBatch(probs, outs=[it["sel"] for it in items])
    parts = (lambda: (ingest_compose(), plan.run(tg, to, ws=bws)), lambda: plan_c.run(cg, co, ws=bws), topk.run)
    for f in parts:
        f()
    torch.cuda.synchronize()
    P.device_status()
    return dict(items=items, ing_outs=ing_outs, all_graphs=all_graphs, outs=outs, parts=parts, coop=coop)


def test_config3_step_captured_against_oracle():
    hs = C.config3(count=8, scale=0.1)
    st = build_step(hs, tuned=False)
    items, ing_outs, all_graphs, outs, parts, coop = (st[k] for k in ("items", "ing_outs", "all_graphs", "outs",
                                                                       "parts", "coop"))
    caps = []
    for f in parts:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            f()
        caps.append(g)

    # the oracle side, from the edge lists alone
    ref = []
    for it in items:
        h, n = it["h"], it["n"]
        layers = [O.csr_from_edges(n, eu, ev) for eu, ev in h.layers]
        A = O.compose("and", layers)
        sums = [O.bfs_sums(rp, ci) for rp, ci in layers + [A]]
        est = O.cc2_est(n, [S for S, _ in sums[:-1]], [R for _, R in sums[:-1]])
        ref.append((layers + [A], sums, O.topk_asc_i64(est, it["k"])))

    for rep in range(2):
        for o_ in outs:
            o_["S"].fill_(-1)
            o_["R"].fill_(-1)
            o_["cc"].fill_(-1.0)
        for it in items:
            it["sel"][0].fill_(-1)
            it["abuf"][0].fill_(-1)
        for rp, ci in ing_outs:
            rp.fill_(-1)
        torch.cuda.synchronize()
        for g in caps:
            g.replay()
        torch.cuda.synchronize()
        P.device_status()
        o = 0
        for hi, (it, (csrs, sums, top)) in enumerate(zip(items, ref)):
            n = it["n"]
            gs = it["graphs"] + [P.Graph(it["abuf"][0], it["abuf"][1], it["abuf"][1].numel())]
            for gi, ((rp, ci), (S, R), g) in enumerate(zip(csrs, sums, gs)):
                grp = g.row_ptr.cpu().numpy()
                assert np.array_equal(grp, rp), (rep, hi, gi)
                assert np.array_equal(g.col_idx[:int(grp[-1])].cpu().numpy(), ci), (rep, hi, gi)
                assert np.array_equal(outs[o + gi]["S"].cpu().numpy(), S), (rep, hi, gi)
                assert np.array_equal(outs[o + gi]["R"].cpu().numpy(), R), (rep, hi, gi)
                cc = O.closeness_wf(n, S, R)
                assert np.array_equal(outs[o + gi]["cc"].cpu().numpy().view(np.int64), cc.view(np.int64)), (rep, hi, gi)
            c = int(it["sel"][2].item())
            assert c == it["k"] and np.array_equal(it["sel"][0][:c].cpu().numpy(), top), (rep, hi)
            o += it["nl"] + 1
        say("replay", rep, "ok:", len(items), "HoMLNs,", len(all_graphs), "graphs,", len(coop), "persistent")


def test_config3_full_size_sampled():
    """All 64 HoMLNs of config 3 at full size, in the bench's launch
    configuration (autotuned widths, the persistent graphs in one partitioned
    multi-graph launch): every layer's CSR and every AND graph equal the
    oracle's; on every graph, 64 sampled vertices' S, R and closeness bits
    equal the oracle's BFS from them and R of every vertex equals its
    component's size; every vertex of every graph of seven HoMLNs (the four
    smallest, whose graphs run as LDS tiles, and the three smallest with
    graphs on the persistent kernel) and their CC2 top-10% sets equal the
    oracle's from its own all-source sums."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    hs = C.config3()
    st = build_step(hs, tuned=True)
    items, outs, coop = st["items"], st["outs"], set(st["coop"])
    say("graphs", len(st["all_graphs"]), "persistent", len(coop))
    assert len(coop) > 100
    rng = np.random.default_rng(77)
    # graph index ranges per HoMLN, and which HoMLNs get every vertex checked
    first, o = [], 0
    for it in items:
        first.append(o)
        o += it["nl"] + 1
    order = np.argsort([it["n"] for it in items])
    with_coop = [hi for hi in order if any(first[hi] + gi in coop for gi in range(items[hi]["nl"] + 1))]
    full = set(order[:4].tolist()) | set(with_coop[:3])
    say("every vertex for HoMLNs", sorted(int(x) for x in full))
    for hi, it in enumerate(items):
        h, n = it["h"], it["n"]
        layers = [O.csr_from_edges(n, eu, ev) for eu, ev in h.layers]
        csrs = layers + [O.compose("and", layers)]
        gs = it["graphs"] + [P.Graph(it["abuf"][0], it["abuf"][1], it["abuf"][1].numel())]
        sums = []
        for gi, ((rp, ci), g) in enumerate(zip(csrs, gs)):
            o = first[hi] + gi
            grp = g.row_ptr.cpu().numpy()
            assert np.array_equal(grp, rp), (hi, gi)
            assert np.array_equal(g.col_idx[:int(grp[-1])].cpu().numpy(), ci), (hi, gi)
            S_g, R_g = outs[o]["S"].cpu().numpy(), outs[o]["R"].cpu().numpy()
            cc_g = outs[o]["cc"].cpu().numpy()
            if hi in full:
                S, R = O.bfs_sums(rp, ci)
                sums.append((S, R))
                assert np.array_equal(S_g, S), (hi, gi)
                assert np.array_equal(R_g, R), (hi, gi)
                assert np.array_equal(cc_g.view(np.int64), O.closeness_wf(n, S, R).view(np.int64)), (hi, gi)
            else:
                src = np.sort(rng.choice(n, size=min(n, 64), replace=False)).astype(np.int32)
                S, R = O.bfs_sums(rp, ci, sources=src)
                assert np.array_equal(S_g[src], S), (hi, gi)
                assert np.array_equal(R_g[src], R), (hi, gi)
                assert np.array_equal(cc_g[src].view(np.int64), O.closeness_wf(n, S, R).view(np.int64)), (hi, gi)
            adj = sp.csr_matrix((np.ones(len(ci), np.int8), ci, rp), shape=(n, n))
            _, lab = connected_components(adj, directed=False)
            assert np.array_equal(R_g, np.bincount(lab)[lab]), (hi, gi)
        if hi in full:
            est = O.cc2_est(n, [S for S, _ in sums[:-1]], [R for _, R in sums[:-1]])
            top = O.topk_asc_i64(est, it["k"])
            c = int(it["sel"][2].item())
            assert c == it["k"] and np.array_equal(it["sel"][0][:c].cpu().numpy(), top), hi
