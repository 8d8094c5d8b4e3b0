"""Parity of the batched path (hln_closeness_batch: persistent LDS tiles,
hipGraph capture and replay, autotuned widths) with the CPU oracle."""
import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from homln_inputs import generators as G
from oracle import oracle as O
from tests.gpu_common import csr_np, graph_dev, say

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")


def check(graphs_np, outs, tag):
    for i, ((rp, ci), o) in enumerate(zip(graphs_np, outs)):
        n = len(rp) - 1
        S, R, H2, _, _ = O.bfs_sums(rp, ci, extras=True)
        cc = O.closeness_wf(n, S, R)
        assert np.array_equal(o["S"].cpu().numpy(), S), (tag, i)
        assert np.array_equal(o["R"].cpu().numpy(), R), (tag, i)
        assert np.array_equal(o["cc"].cpu().numpy().view(np.int64), cc.view(np.int64)), (tag, i)
        if o.get("h2") is not None:
            assert np.array_equal(o["h2"].cpu().numpy(), H2), (tag, i)


def mixed_graphs(seed, sizes):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        m = int(n * rng.choice([0.4, 1.0, 3.0, 6.0]))
        keys = G.take_distinct(G.er_draw(n), min(m, n * (n - 1) // 2), n, rng)
        out.append(csr_np(n, *G.keys_to_edges(keys, n)))
    return out


def test_batch_mixed_sizes_all_width_classes():
    # sizes chosen so that the widest fitting word is 64, 32, 16 and 8 bits
    sizes = [1, 2, 5, 63, 64, 65, 700, 3000, 9000, 20000, 38000, 60000]
    gnp = mixed_graphs(1, sizes)
    plan = P.Plan()
    say("widths", [plan.width(n) for n in sizes])
    graphs = [graph_dev(P, rp, ci) for rp, ci in gnp]
    outs = P.Plan.outputs(graphs, want_h2=True)
    plan.run(graphs, outs)
    torch.cuda.synchronize()
    P.device_status()
    check(gnp, outs, "mixed")


def test_batch_config1_and_named():
    h = C.config1()
    layers = [csr_np(h.n, *e) for e in h.layers]
    gnp = layers + [O.compose("and", layers), O.compose("or", layers)]
    for kind, arg in [("star", 500), ("path", 300), ("complete", 90), ("hypercube", 9)]:
        n, eu, ev = G.named_graph(kind, arg)
        gnp.append(csr_np(n, *G.to_edges(n, eu, ev)))
    plan = P.Plan()
    graphs = [graph_dev(P, rp, ci) for rp, ci in gnp]
    outs = P.Plan.outputs(graphs, want_h2=True)
    plan.run(graphs, outs)
    torch.cuda.synchronize()
    P.device_status()
    check(gnp, outs, "cfg1")


def test_batch_config3_subset():
    gnp = []
    for hh in range(3):
        hm = C.config3_homln(hh, scale=0.25)
        layers = [csr_np(hm.n, *e) for e in hm.layers]
        gnp += layers + [O.compose("and", layers)]
    say("cfg3 subset graphs", len(gnp), [len(g[0]) - 1 for g in gnp])
    plan = P.Plan()
    graphs = [graph_dev(P, rp, ci) for rp, ci in gnp]
    outs = P.Plan.outputs(graphs)
    plan.run(graphs, outs)
    torch.cuda.synchronize()
    P.device_status()
    check(gnp, outs, "cfg3")


def test_batch_capture_replay_and_tune():
    gnp = mixed_graphs(7, [100, 1500, 5000, 12000])
    graphs = [graph_dev(P, rp, ci) for rp, ci in gnp]
    plan = P.Plan()
    outs = P.Plan.outputs(graphs)
    plan.tune(graphs, outs)
    say("tuned widths", [plan.width(g.n) for g in graphs])
    assert all(plan.width(g.n) in (8, 16, 32, 64, 1024, 2048, 4096) for g in graphs)
    ws = P.workspace(plan.workspace_size(graphs))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.capture(graphs, outs, ws, stream)
    for rep in range(3):
        for o in outs:                          # eager work between replays
            o["S"].fill_(-1)
            o["R"].fill_(-1)
            o["cc"].fill_(-1.0)
        torch.cuda.synchronize()
        plan.replay(stream)
        stream.synchronize()
        P.device_status()
        check(gnp, outs, "replay%d" % rep)


def test_batch_large_graphs_use_the_persistent_kernel():
    """Graphs too large for LDS tiles (n > 65,535) go through the persistent
    cooperative kernel inside the same batch call."""
    gnp = mixed_graphs(3, [70000, 1200])
    plan = P.Plan()
    assert plan.width(70000) >= 512 and plan.width(1200) <= 64
    graphs = [graph_dev(P, rp, ci) for rp, ci in gnp]
    outs = P.Plan.outputs(graphs, want_h2=True)
    plan.run(graphs, outs)
    torch.cuda.synchronize()
    P.device_status()
    check(gnp, outs, "large")


def test_batch_several_persistent_graphs_share_one_launch():
    """Six graphs above the LDS-tile limit go through one multi-graph launch
    whose partitions of the grid run them concurrently (longest work first),
    eagerly and captured in a hipGraph; every output against the oracle."""
    rng = np.random.default_rng(11)
    sizes = [66000, 70500, 68000, 72000, 67000, 69000]
    gnp = []
    for n in sizes:
        m = int(n * rng.choice([0.7, 1.0, 1.5]))
        keys = G.take_distinct(G.er_draw(n), m, n, rng)
        gnp.append(csr_np(n, *G.keys_to_edges(keys, n)))
    gnp.append(mixed_graphs(12, [900])[0])
    plan = P.Plan()
    assert all(plan.width(n) >= 512 for n in sizes)
    graphs = [graph_dev(P, rp, ci) for rp, ci in gnp]
    outs = P.Plan.outputs(graphs, want_h2=True)
    plan.run(graphs, outs)
    torch.cuda.synchronize()
    P.device_status()
    check(gnp, outs, "multi")
    ws = P.workspace(plan.workspace_size(graphs))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.capture(graphs, outs, ws, stream)
    for rep in range(2):
        for o in outs:
            o["S"].fill_(-1)
            o["R"].fill_(-1)
        torch.cuda.synchronize()
        plan.replay(stream)
        stream.synchronize()
        P.device_status()
        check(gnp, outs, "multi-replay%d" % rep)


def test_plan_set_width_pins_the_choice():
    """Widths set by hand: every tile width and every persistent width
    (512 runs one launch per graph, 1024-4096 the multi-graph launch) give
    the oracle's outputs; a tile width wider than fits is narrowed; bad
    widths are rejected and change nothing."""
    sizes = [3000, 5000, 9000]             # classes 2^11, 2^12, 2^13
    gnp = mixed_graphs(21, sizes)
    graphs = [graph_dev(P, rp, ci) for rp, ci in gnp]
    for ws in [(8, 16, 32), (64, 64, 64), (512, 1024, 4096), (2048, 2048, 16), (0, 0, 0)]:
        plan = P.Plan()
        for n, w in zip(sizes, ws):
            plan.set_width(n, w)
        got = [plan.width(n) for n in sizes]
        say("set", ws, "->", got)
        fit = [P.Plan().width(n) for n in sizes]
        for w, g, f in zip(ws, got, fit):
            assert g == (f if w == 0 else min(w, f) if w <= 64 else w)
        outs = P.Plan.outputs(graphs, want_h2=True)
        plan.run(graphs, outs)
        torch.cuda.synchronize()
        P.device_status()
        check(gnp, outs, "set%s" % (ws,))
    plan = P.Plan()
    plan.set_width(3000, 1024)
    for bad in [(3000, 128), (3000, 4), (3000, 8192), (0, 64), (-5, 64)]:
        with pytest.raises(P.HlnError):
            plan.set_width(*bad)
    assert plan.width(3000) == 1024


def check_listed(gnp, sources, outs, tag):
    for i, ((rp, ci), src, o) in enumerate(zip(gnp, sources, outs)):
        n = len(rp) - 1
        if src is None:
            S, R = O.bfs_sums(rp, ci)
        else:
            s = src.cpu().numpy()
            if len(s) == 0:
                continue
            S, R = O.bfs_sums(rp, ci, sources=s)
        cc = O.closeness_wf(n, S, R)
        k = len(S)
        assert np.array_equal(o["S"][:k].cpu().numpy(), S), (tag, i)
        assert np.array_equal(o["R"][:k].cpu().numpy(), R), (tag, i)
        assert np.array_equal(o["cc"][:k].cpu().numpy().view(np.int64), cc.view(np.int64)), (tag, i)


def listed_case(seed):
    """Graphs of many sizes, some with listed sources (hubs among them,
    counts below, at and above one batch of every width, an empty list, a
    whole-vertex-set list), the rest with all their vertices."""
    sizes = [40, 700, 3000, 9000, 20000, 70000, 5000, 1200]
    gnp = mixed_graphs(seed, sizes)
    h = C.config2(scale=0.05)
    gnp.append(csr_np(h.n, *h.layers[0]))
    rng = np.random.default_rng(seed)
    counts = [40, 65, None, 513, 4097, 300, 0, None, 2000]
    sources = []
    for (rp, ci), k in zip(gnp, counts):
        n = len(rp) - 1
        if k is None:
            sources.append(None)
            continue
        hubs = np.argsort(-np.diff(rp))[:min(5, k)]
        rest = rng.choice(n, size=min(n, k + 10), replace=False)
        src = np.unique(np.concatenate([hubs, rest]))[:k]
        rng.shuffle(src)                     # outputs follow the caller's order
        sources.append(torch.from_numpy(src.astype(np.int32)).cuda())
    return gnp, sources


def test_batch_listed_sources():
    """hln_closeness_batch with per-graph listed sources (outputs indexed by
    list position) next to all-source graphs: one call, one persistent
    launch per (width, mode) group; against the oracle."""
    gnp, sources = listed_case(11)
    graphs = [graph_dev(P, rp, ci) for rp, ci in gnp]
    for plan_kind in ("untuned", "pinned512", "pinned4096"):
        plan = P.Plan()
        if plan_kind != "untuned":
            w = int(plan_kind[6:])
            for g in graphs:
                plan.set_width(g.n, w)
        say("listed batch", plan_kind, [None if s is None else s.numel() for s in sources])
        outs = P.Plan.outputs_listed(graphs, sources)
        plan.run(graphs, outs, sources=sources)
        torch.cuda.synchronize()
        P.device_status()
        check_listed(gnp, sources, outs, plan_kind)
        coop, ordinary = plan.launch_paths()
        assert coop >= 1 and ordinary == 0


def test_batch_listed_capture_replay():
    gnp, sources = listed_case(12)
    graphs = [graph_dev(P, rp, ci) for rp, ci in gnp]
    plan = P.Plan()
    outs = P.Plan.outputs_listed(graphs, sources)
    ws = P.workspace(plan.workspace_size(graphs))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.capture(graphs, outs, ws, stream, sources=sources)
    for rep in range(2):
        for o in outs:
            o["S"].fill_(-1)
            o["R"].fill_(-1)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            plan.replay(stream)
        stream.synchronize()
        P.device_status()
        check_listed(gnp, sources, outs, "replay%d" % rep)
    # a second capture of another batch into a graph of the caller's, with a
    # staging buffer of its own: the plan's first graph still replays right
    plan.reserve(graphs[:3])
    outs2 = P.Plan.outputs_listed(graphs[:3], sources[:3])
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        plan.run(graphs[:3], outs2, ws=ws, sources=sources[:3])
    g2.replay()
    torch.cuda.synchronize()
    check_listed(gnp[:3], sources[:3], outs2, "caller-graph")
    for o in outs:
        o["S"].fill_(-1)
    with torch.cuda.stream(stream):
        plan.replay(stream)
    stream.synchronize()
    P.device_status()
    check_listed(gnp, sources, outs, "replay-after-second-capture")


def test_batch_listed_argument_errors():
    gnp, sources = listed_case(13)
    graphs = [graph_dev(P, rp, ci) for rp, ci in gnp]
    plan = P.Plan()
    outs = P.Plan.outputs_listed(graphs, sources)
    bad = list(sources)
    bad[0] = torch.arange(graphs[0].n + 1, dtype=torch.int32, device="cuda")      # n_src > n
    with pytest.raises(P.HlnError):
        plan.run(graphs, outs, sources=bad)
    outs_h2 = [dict(o) for o in outs]
    outs_h2[0]["h2"] = torch.empty(graphs[0].n, dtype=torch.int32, device="cuda")   # h2 with listed sources
    with pytest.raises(P.HlnError) as e:
        plan.run(graphs, outs_h2, sources=sources)
    assert "h2" in str(e.value)
    # capturing without reserved staging is refused
    g = torch.cuda.CUDAGraph()
    with pytest.raises(P.HlnError):
        with torch.cuda.graph(g):
            plan.run(graphs, outs, sources=sources)
    torch.cuda.synchronize()
    P.device_status()
