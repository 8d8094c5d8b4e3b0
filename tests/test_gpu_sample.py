"""Sampling estimate of closeness (HIP, through the C ABI) against the CPU
oracle: per-vertex sample sums (listed sources, HLN_FLAG_PER_VERTEX) bit
for bit against one oracle BFS per sampled source, and the FP64 estimate
bit for bit against the oracle's estimator on the same sums."""
import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from homln_inputs import generators as G
from oracle import oracle as O
from tests.gpu_common import csr_np, graph_dev, say, to_dev

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")

WIDTHS = [64, 512, 4096]


def gpu_sums(rp, ci, src, width, direction=0):
    g = graph_dev(P, rp, ci)
    out = P.hln_closeness_layer(g, sources=to_dev(src), width_bits=width, per_vertex=True, direction=direction)
    torch.cuda.synchronize()
    P.device_status()
    assert out["cc"] is None and out["h2"] is None
    return out["S"].cpu().numpy(), out["R"].cpu().numpy()


def gpu_estimate(n, n_pop, src, S, R):
    cc = P.hln_closeness_estimate(n, n_pop, to_dev(src), to_dev(S, torch.int64), to_dev(R))
    torch.cuda.synchronize()
    P.device_status()
    return cc.cpu().numpy()


def check(rp, ci, src, width, n_pop, tag, direction=0):
    n = len(rp) - 1
    say(tag, "n=%d nnz=%d k=%d W=%d direction=%d" % (n, len(ci), len(src), width, direction))
    S, R = gpu_sums(rp, ci, src, width, direction)
    SQ, RQ = O.sample_sums(rp, ci, src)
    assert np.array_equal(S, SQ), (tag, np.nonzero(S != SQ)[0][:10])
    assert np.array_equal(R, RQ), tag
    cc = gpu_estimate(n, n_pop, src, S, R)
    exp = O.sample_estimate(n, n_pop, src, SQ, RQ)
    assert np.array_equal(cc.view(np.int64), exp.view(np.int64)), tag


@pytest.mark.parametrize("width", WIDTHS)
def test_random_graphs_several_batches(width):
    """Sample sizes around the batch width and a ragged tail; graphs with
    several components and isolated vertices."""
    rng = np.random.default_rng(900 + width)
    for trial in range(4):
        n = int(rng.integers(300, 9000))
        m = int(n * rng.choice([0.6, 1.0, 3.0]))
        keys = G.take_distinct(G.er_draw(n), min(m, n * (n - 1) // 2), n, rng)
        rp, ci = csr_np(n, *G.keys_to_edges(keys, n))
        for k in sorted({1, min(n, width - 1), min(n, width + 1), min(n, 2 * width + 37), min(n, 777)}):
            src = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)
            check(rp, ci, src, width, n, "random-%d-k%d" % (trial, k))


@pytest.mark.parametrize("direction", [1, 2])
def test_forced_direction(direction):
    h = C.config2(scale=0.02)
    rp, ci = csr_np(h.n, *h.layers[1])
    src = np.sort(np.random.default_rng(5).choice(h.n, size=1500, replace=False)).astype(np.int32)
    for width in (256, 4096):
        check(rp, ci, src, width, h.n, "cfg2-small-dir%d" % direction, direction=direction)


def test_config1_population_of_nonisolated():
    """Config 4's recipe at config 1's size: the sample is drawn from the
    vertices of degree >= 1 of each graph, n_pop = their count."""
    h = C.config1()
    layers = [csr_np(h.n, *e) for e in h.layers]
    A = O.compose("and", layers)
    for gi, (rp, ci) in enumerate(layers + [A]):
        deg = np.diff(rp)
        src = C.config4_sources(gi, deg, count=max(1, h.n // 8))
        check(rp, ci, src, 512, int((deg > 0).sum()), "cfg1-graph%d" % gi)


def test_full_sample_is_the_exact_closeness():
    """Every vertex sampled: the sums are the all-source sums and the
    estimate is the exact closeness of hln_closeness_layer, bit for bit."""
    h = C.config1()
    rp, ci = O.compose("and", [csr_np(h.n, *e) for e in h.layers])
    n = h.n
    src = np.arange(n, dtype=np.int32)
    S, R = gpu_sums(rp, ci, src, 512)
    g = graph_dev(P, rp, ci)
    ex = P.hln_closeness_layer(g, width_bits=512)
    torch.cuda.synchronize()
    assert np.array_equal(S, ex["S"].cpu().numpy())
    assert np.array_equal(R, ex["R"].cpu().numpy())
    cc = gpu_estimate(n, n, src, S, R)
    assert np.array_equal(cc.view(np.int64), ex["cc"].cpu().numpy().view(np.int64))


def test_edge_cases():
    n, eu, ev = G.named_graph("path", 50)
    eu, ev = G.to_edges(n, eu, ev)
    rp, ci = csr_np(n, eu, ev)
    # empty sample: zero sums, zero estimate
    S, R = gpu_sums(rp, ci, np.zeros(0, np.int32), 512)
    assert not S.any() and not R.any()
    assert not gpu_estimate(n, n, np.zeros(0, np.int32), S, R).any()
    # a repeated id counts each time, as repeated draws
    src = np.array([3, 3, 17], np.int32)
    S, R = gpu_sums(rp, ci, src, 64)
    SQ, RQ = O.sample_sums(rp, ci, src)
    assert np.array_equal(S, SQ) and np.array_equal(R, RQ)
    # one vertex graph, sampled
    rp1, ci1 = csr_np(1, np.zeros(0, np.int64), np.zeros(0, np.int64))
    check(rp1, ci1, np.array([0], np.int32), 64, 1, "n1")
    # isolated vertices outside the population get 0
    rp2, ci2 = csr_np(6, np.array([0, 1]), np.array([1, 2]))
    check(rp2, ci2, np.array([0, 2], np.int32), 64, 3, "isolated")


def test_argument_errors():
    n, eu, ev = G.named_graph("cycle", 20)
    rp, ci = csr_np(n, *G.to_edges(n, eu, ev))
    g = graph_dev(P, rp, ci)
    src = to_dev(np.array([1, 2], np.int32))
    L = P.lib()
    S = torch.zeros(n, dtype=torch.int64, device="cuda")
    R = torch.zeros(n, dtype=torch.int32, device="cuda")
    cc = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(P.HlnError):      # per-vertex sums need listed sources
        P.hln_closeness_layer(g, per_vertex=True)
    o = P._lib.hln_opts(512, 0, 1, None, None, 0)
    ws = P.workspace(P.closeness_workspace_size(n, g.nnz, 2, 512), torch.device("cuda"))
    import ctypes
    gc = g.c()
    args = (ctypes.byref(gc), P._lib._ptr(src), 2, ctypes.byref(o), P._lib._ptr(S), P._lib._ptr(R))
    # cc with per-vertex sums, unknown flag bits
    assert L.hln_closeness_layer(*args, P._lib._ptr(cc), None, P._lib._ptr(ws), ws.numel(), None) == 1
    o.flags = 6
    assert L.hln_closeness_layer(*args, None, None, P._lib._ptr(ws), ws.numel(), None) == 1
    for bad in [(0, 1, 2), (n, 0, 2), (n, n + 1, 2), (n, 1, 2), (n, n, -1)]:
        assert L.hln_closeness_estimate(bad[0], bad[1], P._lib._ptr(src), bad[2], P._lib._ptr(S), P._lib._ptr(R),
                                        P._lib._ptr(cc), None) == 1, bad
    assert L.hln_closeness_estimate(n, n, None, 2, P._lib._ptr(S), P._lib._ptr(R), P._lib._ptr(cc), None) == 1
    torch.cuda.synchronize()
    P.device_status()
