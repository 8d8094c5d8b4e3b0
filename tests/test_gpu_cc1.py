"""Heuristic CC1 (HIP, through the C ABI) against the CPU oracle: the kept
ids equal, and Eq. 3's average bit for bit, on small random HoMLNs, on
config 1 and on scaled configs 2 and 5 (every input, S and R included,
computed by the oracle for the oracle side).  At config 2's full size,
properties that hold at any size."""
import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from oracle import oracle as O
from tests.gpu_common import csr_np, graph_dev, say, to_dev

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")

TAUS = [(1, 2), (0, 1), (1, 3), (3, 4), (1, 1)]


def gpu_cc1(graphs, S_list, R_list, tau):
    ids, count, avg = P.hln_compose_cc1(graphs, S_list, R_list, tau)
    torch.cuda.synchronize()
    P.device_status()
    c = int(count.item())
    return ids[:c].cpu().numpy(), float(avg.item())


def check_homln(n, layers, tag, taus=TAUS):
    sums = [O.bfs_sums(rp, ci)[:2] for rp, ci in layers]
    graphs = [graph_dev(P, rp, ci) for rp, ci in layers]
    S_d = [to_dev(S, torch.int64) for S, _ in sums]
    R_d = [to_dev(R) for _, R in sums]
    for tau in taus:
        want, avg = O.cc1(n, layers, [S for S, _ in sums], [R for _, R in sums], tau, with_avg=True)
        got, gavg = gpu_cc1(graphs, S_d, R_d, tau)
        say(tag, "r=%d tau=%s kept=%d" % (len(layers), tau, len(want)))
        assert np.array_equal(got, want), (tag, tau)
        assert np.float64(gavg).view(np.int64) == np.float64(avg).view(np.int64), (tag, tau)


def random_homln(rng, n, r, p_base, p_own):
    iu, iv = np.triu_indices(n, 1)
    base = rng.random(len(iu)) < p_base
    layers = []
    for _ in range(r):
        keep = base | (rng.random(len(iu)) < p_own)
        layers.append(csr_np(n, iu[keep], iv[keep]))
    return layers


def test_random_small_homlns():
    rng = np.random.default_rng(61)
    for trial in range(12):
        n = int(rng.integers(10, 400))
        r = int(rng.integers(2, 5))
        check_homln(n, random_homln(rng, n, r, 3.0 / n, 2.0 / n), "random-%d" % trial)


def test_config1_all_layers_and_pairs():
    h = C.config1()
    layers = [csr_np(h.n, *e) for e in h.layers]
    check_homln(h.n, layers, "cfg1-all")
    for i in range(len(layers)):
        for j in range(i + 1, len(layers)):
            check_homln(h.n, [layers[i], layers[j]], "cfg1-%d%d" % (i, j), taus=[(1, 2)])


@pytest.mark.parametrize("cfg,scale", [(2, 0.04), (5, 0.1)])
def test_scaled_configs(cfg, scale):
    h = C.make_config(cfg, scale)
    layers = [csr_np(h.n, *e) for e in h.layers]
    check_homln(h.n, layers, "cfg%d-x%g" % (cfg, scale), taus=[(1, 2), (1, 1)])
    check_homln(h.n, layers[:2], "cfg%d-x%g-pair" % (cfg, scale), taus=[(1, 2)])


def test_edge_cases():
    # one layer: the pair (G, G) and G alone agree (identical layers overlap fully)
    rng = np.random.default_rng(67)
    (g,) = random_homln(rng, 120, 1, 0.02, 0.01)
    check_homln(120, [g], "single", taus=[(1, 2)])
    check_homln(120, [g, g], "twice", taus=[(1, 2)])
    # no edges at all: no ratio anywhere, nothing kept
    empty = csr_np(30, np.zeros(0, np.int64), np.zeros(0, np.int64))
    check_homln(30, [empty, empty], "empty", taus=[(0, 1)])
    # one vertex
    one = csr_np(1, np.zeros(0, np.int64), np.zeros(0, np.int64))
    check_homln(1, [one, one], "n1", taus=[(1, 2)])
    # cycles: every ratio equals the average, nothing is central
    u = np.arange(16)
    cyc = csr_np(16, u, (u + 1) % 16)
    check_homln(16, [cyc, cyc], "cycle", taus=[(0, 1)])


def test_argument_errors():
    rng = np.random.default_rng(3)
    layers = random_homln(rng, 50, 2, 0.05, 0.02)
    graphs = [graph_dev(P, rp, ci) for rp, ci in layers]
    S = [torch.zeros(50, dtype=torch.int64, device="cuda")] * 2
    R = [torch.ones(50, dtype=torch.int32, device="cuda")] * 2
    for tau in [(-1, 2), (1, 0)]:
        with pytest.raises(P.HlnError):
            P.hln_compose_cc1(graphs, S, R, tau)
    other = graph_dev(P, *csr_np(51, np.array([0]), np.array([1])))
    with pytest.raises(P.HlnError):
        P.hln_compose_cc1([graphs[0], other], S, R)
    assert P.lib().hln_compose_cc1_workspace_size(50, 65) == 0


def test_config2_full_size_properties():
    """n = 100,000, 4 layers: CC1 keeps only common CC nodes (naive), keeps
    fewer as the threshold rises, nothing above 1, and is deterministic."""
    h = C.config2()
    layers = [P.hln_csr_from_edges(h.n, to_dev(eu), to_dev(ev)).trimmed() for eu, ev in h.layers]
    outs = [P.hln_closeness_layer(g, width_bits=4096, want_cc=False) for g in layers]
    Ss, Rs = [o["S"] for o in outs], [o["R"] for o in outs]
    naive = P.hln_compose_cc_topk(P.HLN_RANK_NAIVE, h.n, Ss, Rs, -1)
    torch.cuda.synchronize()
    nv = set(naive[0][:int(naive[2].item())].cpu().numpy().tolist())
    prev = None
    for tau in [(0, 1), (1, 4), (1, 2), (3, 4), (1, 1), (5, 4)]:
        got, avg = gpu_cc1(layers, Ss, Rs, tau)
        say("cfg2-full tau", tau, "kept", len(got), "avg", avg)
        assert np.all(np.diff(got) > 0)
        s = set(got.tolist())
        assert s <= nv
        if prev is not None:
            assert s <= prev
        prev = s
    assert not prev
    a, _ = gpu_cc1(layers, Ss, Rs, (1, 2))
    b, _ = gpu_cc1(layers, Ss, Rs, (1, 2))
    assert np.array_equal(a, b) and len(a) > 0
