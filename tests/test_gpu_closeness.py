"""Parity of hln_closeness_layer (HIP, through the C ABI) with the CPU oracle:
S and R bit-exact, closeness bit-exact in FP64, 2-hop counts exact."""
import ctypes

import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from homln_inputs import generators as G
from oracle import oracle as O
from tests.gpu_common import allsource_batch_order, csr_np, graph_dev, listed_batch_order, say, to_dev

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")

WIDTHS = [64, 128, 256, 512, 1024, 2048, 4096]


def run_all(rp, ci, width, want_h2=True, direction=0):
    g = graph_dev(P, rp, ci)
    out = P.hln_closeness_layer(g, width_bits=width, want_h2=want_h2, direction=direction)
    torch.cuda.synchronize()
    P.device_status()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def check_all(n, rp, ci, width, tag, direction=0):
    say(tag, "n=%d nnz=%d W=%d direction=%d" % (n, len(ci), width, direction))
    got = run_all(rp, ci, width, direction=direction)
    S, R, H2, _, _ = O.bfs_sums(rp, ci, extras=True)
    cc = O.closeness_wf(n, S, R)
    assert np.array_equal(got["S"], S), (tag, np.nonzero(got["S"] != S)[0][:10])
    assert np.array_equal(got["R"], R), tag
    assert np.array_equal(got["h2"], H2), tag
    assert np.array_equal(got["cc"].view(np.int64), cc.view(np.int64)), tag


NAMED = [("path", 300), ("star", 1000), ("cycle", 257), ("complete", 150), ("hypercube", 8), ("bipartite", 70, 130)]


@pytest.mark.parametrize("width", WIDTHS)
@pytest.mark.parametrize("named", NAMED, ids=["%s%s" % (x[0], x[1]) for x in NAMED])
def test_named_graphs(named, width):
    n, eu, ev = G.named_graph(*named)
    eu, ev = G.to_edges(n, eu, ev)
    rp, ci = csr_np(n, eu, ev)
    check_all(n, rp, ci, width, "named-%s" % (named,))


@pytest.mark.parametrize("width", WIDTHS)
def test_degenerate(width):
    # one vertex; all isolated; a single edge plus isolated vertices
    for n, eu, ev in [(1, [], []), (5, [], []), (7, [2], [5])]:
        rp, ci = csr_np(n, np.array(eu, np.int64), np.array(ev, np.int64))
        check_all(n, rp, ci, width, "degenerate-n%d" % n)


def test_empty_source_list():
    """An empty source list (n_src = 0, with a NULL or a real pointer)
    enqueues nothing and leaves the outputs alone; in per-vertex mode it
    writes zero sums for every vertex."""
    rp, ci = csr_np(9, np.array([0, 1, 2], np.int64), np.array([1, 2, 3], np.int64))
    g = graph_dev(P, rp, ci)
    L = P.lib()
    o = P._lib.hln_opts(512, 0, 0, None)
    S = torch.full((4,), -7, dtype=torch.int64, device="cuda")
    R = torch.full((4,), -7, dtype=torch.int32, device="cuda")
    need = P.closeness_workspace_size(9, len(ci), 0, 512)
    ws = P.workspace(need)
    gc = g.c()
    real = to_dev(np.array([3], np.int32))
    for src in (None, real.data_ptr()):
        st = L.hln_closeness_layer(ctypes.byref(gc), src, 0, ctypes.byref(o), S.data_ptr(), R.data_ptr(), None, None,
                                   ws.data_ptr(), ws.numel(), None)
        assert st == 0, L.hln_last_error()
    torch.cuda.synchronize()
    P.device_status()
    assert S.tolist() == [-7] * 4 and R.tolist() == [-7] * 4
    out = P.hln_closeness_layer(g, sources=torch.empty(0, dtype=torch.int32, device="cuda"), width_bits=512)
    assert out["S"].numel() == 0 and out["R"].numel() == 0 and out["cc"].numel() == 0
    pv = P.hln_closeness_layer(g, sources=torch.empty(0, dtype=torch.int32, device="cuda"), width_bits=512,
                               per_vertex=True)
    torch.cuda.synchronize()
    P.device_status()
    assert pv["S"].cpu().tolist() == [0] * 9 and pv["R"].cpu().tolist() == [0] * 9


@pytest.mark.parametrize("width", WIDTHS)
def test_random_disconnected(width):
    rng = np.random.default_rng(100 + width)
    for trial in range(6):
        n = int(rng.integers(2, 2500))
        m = int(n * rng.choice([0.3, 0.6, 1.0, 3.0]))
        keys = G.take_distinct(G.er_draw(n), min(m, n * (n - 1) // 2), n, rng)
        eu, ev = G.keys_to_edges(keys, n)
        rp, ci = csr_np(n, eu, ev)
        check_all(n, rp, ci, width, "random-%d" % trial)


@pytest.fixture(scope="module")
def cfg1():
    h = C.config1()
    layers = [csr_np(h.n, *e) for e in h.layers]
    return h.n, layers, O.compose("and", layers), O.compose("or", layers)


@pytest.mark.parametrize("width", WIDTHS)
def test_config1_layers_and_or(cfg1, width):
    n, layers, A, B = cfg1
    for i, (rp, ci) in enumerate(layers + [A, B]):
        check_all(n, rp, ci, width, "cfg1-graph%d" % i)


@pytest.mark.parametrize("width", [64, 512])
def test_config2_scaled(width):
    h = C.config2(scale=0.04)
    rp, ci = csr_np(h.n, *h.layers[0])
    check_all(h.n, rp, ci, width, "cfg2-scaled-layer0")


@pytest.mark.parametrize("width", WIDTHS)
def test_listed_sources(width):
    rng = np.random.default_rng(7)
    h = C.config1()
    rp, ci = csr_np(h.n, *h.layers[1])
    A = O.compose("and", [csr_np(h.n, *e) for e in h.layers])
    for (gr, gc), tag in [((rp, ci), "layer1"), (A, "and")]:
        for count in (1, 63, 64, 65, 300, h.n):
            src = rng.choice(h.n, size=count, replace=False).astype(np.int32)   # any order: outputs follow it
            if count in (63, 300):
                src = np.sort(src)
            say("listed", tag, count, width)
            g = graph_dev(P, gr, gc)
            out = P.hln_closeness_layer(g, sources=to_dev(src), width_bits=width)
            torch.cuda.synchronize()
            P.device_status()
            S, R = O.bfs_sums(gr, gc, sources=src)
            cc = O.closeness_wf(h.n, S, R)
            assert np.array_equal(out["S"].cpu().numpy(), S)
            assert np.array_equal(out["R"].cpu().numpy(), R)
            assert np.array_equal(out["cc"].cpu().numpy().view(np.int64), cc.view(np.int64))


def test_determinism():
    h = C.config2(scale=0.02)
    rp, ci = csr_np(h.n, *h.layers[2])
    a = run_all(rp, ci, 256)
    b = run_all(rp, ci, 256)
    for k in ("S", "R", "cc", "h2"):
        assert np.array_equal(a[k], b[k])


def test_config2_full_size_sampled():
    """Full-size config-2 layers at W = 512 (the narrower code path: 32-bit
    word masks, lane groups of 8; the benchmark's own W = 4096 launch is
    compared on every vertex in test_gpu_fullsize.py): sampled vertices
    against one oracle BFS each (by symmetry S[v] is the BFS sum from v), R
    against the connected components of every vertex."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    h = C.config2()
    n = h.n
    rng = np.random.default_rng(3)
    for li in (0, 3):
        rp, ci = csr_np(n, *h.layers[li])
        say("cfg2-full layer", li)
        got = run_all(rp, ci, 512)
        sample = np.sort(rng.choice(n, size=96, replace=False)).astype(np.int32)
        S, R, H2, _, _ = O.bfs_sums(rp, ci, sources=sample, extras=True)
        assert np.array_equal(got["S"][sample], S)
        assert np.array_equal(got["R"][sample], R)
        assert np.array_equal(got["h2"][sample], H2)
        cc = O.closeness_wf(n, S, R)
        assert np.array_equal(got["cc"][sample].view(np.int64), cc.view(np.int64))
        adj = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
        ncomp, lab = connected_components(adj, directed=False)
        sizes = np.bincount(lab)
        assert np.array_equal(got["R"], sizes[lab])


@pytest.mark.parametrize("width", [64, 512, 2048, 4096])
def test_levels_per_batch(width):
    """The kernel's per-batch level count is 1 + the largest eccentricity of
    the batch's sources (the L_b of the byte model), from the oracle; the
    all-source batches take the vertices that have arcs, largest degree class
    first, ids ascending inside a class, and the batches after the first by
    distance from the first batch's hub (allsource_batch_order)."""
    h = C.config1()
    n = h.n
    for rp, ci in [csr_np(n, *h.layers[0]), O.compose("and", [csr_np(n, *e) for e in h.layers])]:
        nb = (n + width - 1) // width
        lv = torch.zeros(nb, dtype=torch.int32, device="cuda")
        g = graph_dev(P, rp, ci)
        P.hln_closeness_layer(g, width_bits=width, levels=lv)
        torch.cuda.synchronize()
        _, _, _, ecc, _ = O.bfs_sums(rp, ci, extras=True)
        act = allsource_batch_order(rp, ci, width)
        na = (len(act) + width - 1) // width
        ref = [1 + int(ecc[act[b * width:(b + 1) * width]].max()) for b in range(na)] + [0] * (nb - na)
        assert lv.cpu().numpy().tolist() == ref


@pytest.mark.parametrize("width", [64, 512, 2048, 4096])
def test_levels_per_batch_listed(width):
    """Listed sources are batched by their vertex's degree class (a source
    without arcs with the last class), list positions ascending inside a
    class, and below W = 4096 the batches after the first by distance from
    the first batch's hub (listed_batch_order): each batch's level count is 1
    + the largest eccentricity of its sources (oracle), and the per-source
    outputs stay at the caller's positions."""
    h = C.config1()
    n = h.n
    rng = np.random.default_rng(90 + width)
    for rp, ci in [csr_np(n, *h.layers[0]), O.compose("and", [csr_np(n, *e) for e in h.layers])]:
        src = rng.permutation(n)[:int(rng.integers(n // 2, n))].astype(np.int32)
        k = len(src)
        nb = (k + width - 1) // width
        lv = torch.zeros(nb, dtype=torch.int32, device="cuda")
        g = graph_dev(P, rp, ci)
        out = P.hln_closeness_layer(g, sources=to_dev(src), width_bits=width, levels=lv)
        torch.cuda.synchronize()
        P.device_status()
        S, R, _, ecc, _ = O.bfs_sums(rp, ci, sources=src, extras=True)
        assert np.array_equal(out["S"].cpu().numpy(), S)
        assert np.array_equal(out["R"].cpu().numpy(), R)
        order = listed_batch_order(rp, ci, src, width, by_distance=width < 4096)
        ref = [1 + int(ecc[order[b * width:(b + 1) * width]].max()) for b in range(nb)]
        assert lv.cpu().numpy().tolist() == ref


@pytest.mark.parametrize("width", [64, 512])
def test_levels_listed_duplicates_and_arcless(width):
    """Listed sources with repeated vertices and vertices without arcs, over
    a graph of several components: the per-source sums at every list
    position (oracle), and the per-batch levels in the order
    listed_batch_order gives (the later batches by distance from the first
    batch's hub; a repeated vertex keeps its place among equals)."""
    h = C.config1()
    n = h.n
    rp, ci = O.compose("and", [csr_np(n, *e) for e in h.layers])
    deg = np.diff(rp)
    rng = np.random.default_rng(5 + width)
    pool = np.concatenate([rng.choice(n, size=300, replace=False), np.nonzero(deg == 0)[0][:40]])
    src = rng.choice(pool, size=900, replace=True).astype(np.int32)
    nb = (len(src) + width - 1) // width
    lv = torch.zeros(nb, dtype=torch.int32, device="cuda")
    g = graph_dev(P, rp, ci)
    out = P.hln_closeness_layer(g, sources=to_dev(src), width_bits=width, levels=lv)
    torch.cuda.synchronize()
    P.device_status()
    S, R, _, ecc, _ = O.bfs_sums(rp, ci, sources=src, extras=True)
    assert np.array_equal(out["S"].cpu().numpy(), S)
    assert np.array_equal(out["R"].cpu().numpy(), R)
    order = listed_batch_order(rp, ci, src, width, by_distance=True)
    assert lv.cpu().numpy().tolist() == [1 + int(ecc[order[b * width:(b + 1) * width]].max()) for b in range(nb)]


@pytest.mark.parametrize("width", [64, 256, 2048, 4096])
@pytest.mark.parametrize("direction", [1, 2], ids=["top_down", "bottom_up"])
def test_forced_direction(direction, width):
    """Every level top-down (push) or every level bottom-up (pull)."""
    for named in [("path", 300), ("star", 1000), ("complete", 150), ("bipartite", 70, 130)]:
        n, eu, ev = G.named_graph(*named)
        rp, ci = csr_np(n, *G.to_edges(n, eu, ev))
        check_all(n, rp, ci, width, "named-%s" % (named,), direction)
    rng = np.random.default_rng(500 + width + direction)
    for trial in range(4):
        n = int(rng.integers(2, 3000))
        m = int(n * rng.choice([0.3, 1.0, 4.0]))
        keys = G.take_distinct(G.er_draw(n), min(m, n * (n - 1) // 2), n, rng)
        rp, ci = csr_np(n, *G.keys_to_edges(keys, n))
        check_all(n, rp, ci, width, "random-%d" % trial, direction)
    h = C.config2(scale=0.05)
    rp, ci = csr_np(h.n, *h.layers[1])
    check_all(h.n, rp, ci, width, "cfg2-scaled", direction)
    # listed sources, with hubs among them
    src = np.unique(np.concatenate([np.argsort(-np.diff(rp))[:20], rng.choice(h.n, 300, replace=False)]))
    src = src.astype(np.int32)
    g = graph_dev(P, rp, ci)
    out = P.hln_closeness_layer(g, sources=to_dev(src), width_bits=width, direction=direction)
    torch.cuda.synchronize()
    P.device_status()
    S, R = O.bfs_sums(rp, ci, sources=src)
    assert np.array_equal(out["S"].cpu().numpy(), S)
    assert np.array_equal(out["R"].cpu().numpy(), R)


def test_auto_direction_takes_both():
    """The automatic choice runs sparse levels top-down and the dense middle
    bottom-up; the trace records each level's direction and new pairs."""
    h = C.config2(scale=0.1)
    rp, ci = csr_np(h.n, *h.layers[0])
    g = graph_dev(P, rp, ci)
    tr = torch.zeros((4096, 4), dtype=torch.int64, device="cuda")
    lv = torch.zeros((h.n + 511) // 512, dtype=torch.int32, device="cuda")
    out = P.hln_closeness_layer(g, width_bits=512, want_h2=True, levels=lv, trace=tr)
    torch.cuda.synchronize()
    P.device_status()
    rows = int(lv.sum().item())
    t = tr[:rows].cpu().numpy()
    dirs = t[:, 3]
    say("levels", rows, "top-down", int(dirs.sum()))
    assert 0 < dirs.sum() < rows
    S, R, H2, _, _ = O.bfs_sums(rp, ci, extras=True)
    assert np.array_equal(out["S"].cpu().numpy(), S)
    assert np.array_equal(out["h2"].cpu().numpy(), H2)
    # top-down levels are the sparse ones
    pairs = t[:, 2]
    assert np.median(pairs[dirs == 1]) < np.median(pairs[dirs == 0])


def test_auto_direction_at_4096_is_bottom_up():
    """At W = 4096 the automatic choice runs every level bottom-up (the
    trace's direction column is all zero) and the sums stay exact."""
    h = C.config2(scale=0.1)
    rp, ci = csr_np(h.n, *h.layers[0])
    g = graph_dev(P, rp, ci)
    tr = torch.zeros((4096, 4), dtype=torch.int64, device="cuda")
    lv = torch.zeros((h.n + 4095) // 4096, dtype=torch.int32, device="cuda")
    out = P.hln_closeness_layer(g, width_bits=4096, want_h2=True, levels=lv, trace=tr)
    torch.cuda.synchronize()
    P.device_status()
    rows = int(lv.sum().item())
    t = tr[:rows].cpu().numpy()
    assert rows > 0 and not t[:, 3].any()
    S, R, H2, _, _ = O.bfs_sums(rp, ci, extras=True)
    assert np.array_equal(out["S"].cpu().numpy(), S)
    assert np.array_equal(out["R"].cpu().numpy(), R)
    assert np.array_equal(out["h2"].cpu().numpy(), H2)


@pytest.mark.parametrize("width", [64, 4096])
def test_distance_sums_past_the_32_bit_window(width, monkeypatch):
    """Levels from HLN_S32_LEVELS on add to S with 64-bit atomics instead of
    the per-batch 32-bit sums; forcing it from level 3 runs both paths in
    one BFS (long paths and a random graph)."""
    monkeypatch.setenv("HLN_S32_LEVELS", "3")
    for named in [("path", 700), ("cycle", 513)]:
        n, eu, ev = G.named_graph(*named)
        rp, ci = csr_np(n, *G.to_edges(n, eu, ev))
        check_all(n, rp, ci, width, "s64-%s" % (named,))
    h = C.config2(scale=0.03)
    rp, ci = csr_np(h.n, *h.layers[0])
    check_all(h.n, rp, ci, width, "s64-cfg2-scaled")


@pytest.mark.parametrize("width", [64, 256, 4096])
def test_saturation_probe_components(width):
    """Vertices that hold every bit they can receive skip later levels; what
    they can receive is judged against the component of the first batch's
    highest-degree source.  Cases: that probe in a small component (a star
    hub outranking a long cycle), the probe isolated (the first batch all
    isolated vertices), and a listed first batch from another component than
    later batches.  Sums against the oracle."""
    rng = np.random.default_rng(81 + width)
    W = width
    # star (hub degree 3W/2) first, then a cycle and random chords, isolated tail
    n_star = 3 * W // 2 + 1
    n_cyc = 5 * W + 17
    eu = [0] * (n_star - 1)
    ev = list(range(1, n_star))
    base = n_star
    for i in range(n_cyc):
        eu.append(base + i)
        ev.append(base + (i + 1) % n_cyc)
    for _ in range(n_cyc // 3):
        a, b = rng.choice(n_cyc, size=2, replace=False)
        eu.append(base + int(a))
        ev.append(base + int(b))
    n = base + n_cyc + 40
    keys = sorted({(min(a, b), max(a, b)) for a, b in zip(eu, ev) if a != b})
    u = np.array([k[0] for k in keys])
    v = np.array([k[1] for k in keys])
    rp, ci = csr_np(n, u, v)
    check_all(n, rp, ci, width, "star-probe")
    # first batch made of isolated vertices: relabel so they come first
    perm = np.concatenate([np.arange(base + n_cyc, n), np.arange(0, base + n_cyc)])
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    rp2, ci2 = csr_np(n, inv[u], inv[v])
    check_all(n, rp2, ci2, width, "isolated-probe")
    # listed sources: first batch inside the star, later ones on the cycle
    src = np.concatenate([np.arange(0, min(W, n_star)), base + rng.choice(n_cyc, size=2 * W + 5, replace=False)])
    src = src.astype(np.int32)
    g = graph_dev(P, rp, ci)
    out = P.hln_closeness_layer(g, sources=to_dev(src), width_bits=width)
    torch.cuda.synchronize()
    P.device_status()
    S, R = O.bfs_sums(rp, ci, sources=src)
    assert np.array_equal(out["S"].cpu().numpy(), S)
    assert np.array_equal(out["R"].cpu().numpy(), R)
    pv = P.hln_closeness_layer(g, sources=to_dev(src), width_bits=width, per_vertex=True)
    torch.cuda.synchronize()
    SQ, RQ = O.sample_sums(rp, ci, src)
    assert np.array_equal(pv["S"].cpu().numpy(), SQ)
    assert np.array_equal(pv["R"].cpu().numpy(), RQ)


def test_all_sources_many_segments_per_wave():
    """All sources at W = 4096 on a graph with more segments than 64 per wave
    (n = 450,000: about 100 per wave of the 4,096 the grid holds), so the
    sweep takes each wave's segments in several windows of 64: a sparse
    random component over 400,000 vertices, a path of 10,000 vertices (deep
    BFS, saturation over many levels) and 40,000 isolated vertices.  S, R, h2
    and closeness bits of 96 sampled vertices against one oracle BFS each, R
    of every vertex against the components."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    n, nr, npath = 450_000, 400_000, 10_000
    rng = np.random.default_rng(11)
    m = 2 * nr
    eu = rng.integers(0, nr, size=m)
    ev = rng.integers(0, nr, size=m)
    pu = np.arange(nr, nr + npath - 1)
    eu = np.concatenate([eu, pu])
    ev = np.concatenate([ev, pu + 1])
    keep = eu != ev
    a, b = np.minimum(eu[keep], ev[keep]), np.maximum(eu[keep], ev[keep])
    key = np.unique(a * n + b)
    rp, ci = csr_np(n, key // n, key % n)
    say("many windows: n=%d arcs=%d" % (n, len(ci)))
    got = run_all(rp, ci, 4096)
    sample = np.unique(np.concatenate([rng.choice(n, size=90, replace=False),
                                       [0, nr, nr + npath // 2, nr + npath - 1, n - 1, n - 2]])).astype(np.int32)
    S, R, H2, _, _ = O.bfs_sums(rp, ci, sources=sample, extras=True)
    assert np.array_equal(got["S"][sample], S)
    assert np.array_equal(got["R"][sample], R)
    assert np.array_equal(got["h2"][sample], H2)
    assert np.array_equal(got["cc"][sample].view(np.int64), O.closeness_wf(n, S, R).view(np.int64))
    adj = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
    _, lab = connected_components(adj, directed=False)
    assert np.array_equal(got["R"], np.bincount(lab)[lab])


def test_largest_graph_at_width_4096():
    """The largest vertex count W = 4096 allows: n = 2^22 - 1, so a bitset
    is n * W / 8 = 2^31 - 512 bytes and the kernel's 32-bit buffer offsets
    run almost to their end.  A sparse graph (a cycle through all but the
    last 1,000 vertices, which stay isolated, plus random chords) with 4,100
    listed sources in shuffled order: two batches, the second holding the
    lowest-degree sources, among them isolated vertices at the very end of
    the id range.  The oracle takes about 0.1 s of one core per source here,
    so it checks 150 sampled list positions plus every position whose vertex
    is one of the last ids; every isolated source has S = 0, R = 1 and
    closeness 0.  One vertex more is refused (HLN_EUNSUPPORTED) before
    anything is enqueued."""
    n = (1 << 22) - 1
    live = n - 1000
    rng = np.random.default_rng(5)
    base = np.arange(live, dtype=np.int64)
    eu = np.concatenate([base, rng.integers(0, live, size=live)])
    ev = np.concatenate([(base + 1) % live, rng.integers(0, live, size=live)])
    keep = eu != ev
    a, b = np.minimum(eu[keep], ev[keep]), np.maximum(eu[keep], ev[keep])
    key = np.unique(a * n + b)
    rp, ci = csr_np(n, key // n, key % n)
    say("largest graph: n=%d arcs=%d" % (n, len(ci)))
    tail = np.concatenate([np.arange(live - 5, live), np.arange(n - 5, n)])
    src = np.unique(np.concatenate([rng.choice(live - 5, size=4090, replace=False), tail])).astype(np.int32)
    rng.shuffle(src)
    g = graph_dev(P, rp, ci)
    out = P.hln_closeness_layer(g, sources=to_dev(src), width_bits=4096)
    torch.cuda.synchronize()
    P.device_status()
    gS, gR, gcc = out["S"].cpu().numpy(), out["R"].cpu().numpy(), out["cc"].cpu().numpy()
    iso = src >= live
    assert iso.sum() == 5
    assert np.all(gS[iso] == 0) and np.all(gR[iso] == 1) and np.all(gcc[iso] == 0.0)
    pos = np.union1d(rng.choice(len(src), size=150, replace=False), np.nonzero(np.isin(src, tail))[0])
    say("oracle: %d sampled sources" % len(pos))
    S, R = O.bfs_sums(rp, ci, sources=src[pos])
    assert np.array_equal(gS[pos], S)
    assert np.array_equal(gR[pos], R)
    assert np.array_equal(gcc[pos].view(np.int64), O.closeness_wf(n, S, R).view(np.int64))
    del out
    rp2 = np.append(rp, rp[-1]).astype(np.int32)           # one more (isolated) vertex: 2^22
    g2 = P.Graph(to_dev(rp2), g.col_idx)
    with pytest.raises(P.HlnError) as e:
        P.hln_closeness_layer(g2, sources=to_dev(src[:10]), width_bits=4096)
    assert e.value.status == 4          # HLN_EUNSUPPORTED
    torch.cuda.synchronize()
    P.device_status()
