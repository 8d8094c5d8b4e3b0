"""Pins for the CPU oracle: checks against facts that do not come from the
oracle itself (closed forms, Floyd-Warshall, union-find, NetworkX's
closeness routine -- the one the paper uses, Sec. 4 -- Python set algebra,
brute-force sorting, exact rational arithmetic and the paper's printed CC2
example, Sec. 5.2).

Each pin takes an oracle handle ``o`` (the ``oracle.oracle`` module or a
``Variant`` with a planted mistake) and raises AssertionError on a mismatch.
``test_oracle_pins.py`` runs them on the real oracle; ``test_oracle_mutants``
runs them on planted-mistake builds and requires every mistake to be caught.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np

from homln_inputs import generators as G

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# --------------------------------------------------------------------------
# independent helpers (no oracle code)
# --------------------------------------------------------------------------

def adjacency_sets(n, eu, ev):
    adj = [set() for _ in range(n)]
    for a, b in zip(np.asarray(eu).tolist(), np.asarray(ev).tolist()):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def floyd_warshall(n, adj):
    """All-pairs hop distances (inf = unreachable)."""
    D = np.full((n, n), np.inf)
    np.fill_diagonal(D, 0.0)
    for u in range(n):
        for v in adj[u]:
            D[u, v] = 1.0
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def components(n, adj):
    """Union-find component sizes per vertex."""
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for u in range(n):
        for v in adj[u]:
            a, b = find(u), find(v)
            if a != b:
                parent[a] = b
    roots = [find(u) for u in range(n)]
    size = {}
    for r in roots:
        size[r] = size.get(r, 0) + 1
    return np.array([size[r] for r in roots])


def random_graph(rng, n, p):
    iu, iv = np.triu_indices(n, 1)
    keep = rng.random(len(iu)) < p
    return iu[keep], iv[keep]


def csr_of(o, n, eu, ev):
    return o.csr_from_edges(n, eu, ev)


def nx_graph(n, adj):
    import networkx as nx
    g = nx.Graph()
    g.add_nodes_from(range(n))
    for u in range(n):
        for v in adj[u]:
            if u < v:
                g.add_edge(u, v)
    return g


# --------------------------------------------------------------------------
# pins
# --------------------------------------------------------------------------

def pin_closed_forms(o):
    """Textbook distance sums, reach, 2-hop counts and eccentricities."""
    cases = []
    n = 9
    i = np.arange(n)
    cases.append(("path", (n,), i * (i + 1) // 2 + (n - 1 - i) * (n - i) // 2,
                  (i >= 2).astype(int) + (n - 1 - i >= 2).astype(int), np.maximum(i, n - 1 - i)))
    n = 7
    cases.append(("star", (n,), np.array([n - 1] + [2 * n - 3] * (n - 1)),
                  np.array([0] + [n - 2] * (n - 1)), np.array([1] + [2] * (n - 1))))
    for n in (7, 8):
        s = (n * n - 1) // 4 if n % 2 else n * n // 4
        cases.append(("cycle", (n,), np.full(n, s), np.full(n, 2), np.full(n, n // 2)))
    n = 6
    cases.append(("complete", (n,), np.full(n, n - 1), np.zeros(n, int), np.ones(n, int)))
    a, b = 3, 5
    cases.append(("bipartite", (a, b), np.array([b + 2 * (a - 1)] * a + [a + 2 * (b - 1)] * b),
                  np.array([a - 1] * a + [b - 1] * b), np.full(a + b, 2)))
    k = 5
    cases.append(("hypercube", (k,), np.full(1 << k, k * (1 << (k - 1))),
                  np.full(1 << k, k * (k - 1) // 2), np.full(1 << k, k)))
    for kind, args, S_ref, H2_ref, ecc_ref in cases:
        n, eu, ev = G.named_graph(kind, *args)
        rp, ci = csr_of(o, n, eu, ev)
        S, R, H2, ecc, _ = o.bfs_sums(rp, ci, extras=True)
        assert np.array_equal(S, S_ref), (kind, S, S_ref)
        assert np.array_equal(R, np.full(n, n)), (kind, R)
        assert np.array_equal(H2, H2_ref), (kind, H2, H2_ref)
        assert np.array_equal(ecc, ecc_ref), (kind, ecc, ecc_ref)


def pin_disjoint_union(o):
    """Per-component closed forms; R is the component size; isolated
    vertices have S = 0, R = 1, cc = 0 and penalised sum n(n-1)."""
    # path on 0..4, star centred at 5 with leaves 6..9, isolated 10, 11
    n = 12
    eu = [0, 1, 2, 3, 5, 5, 5, 5]
    ev = [1, 2, 3, 4, 6, 7, 8, 9]
    rp, ci = csr_of(o, n, eu, ev)
    S, R = o.bfs_sums(rp, ci)
    i = np.arange(5)
    S_ref = np.concatenate([i * (i + 1) // 2 + (4 - i) * (5 - i) // 2, [4], [7] * 4, [0, 0]])
    R_ref = np.array([5] * 5 + [5] * 5 + [1, 1])
    assert np.array_equal(S, S_ref), (S, S_ref)
    assert np.array_equal(R, R_ref), R
    cc = o.closeness_wf(n, S, R)
    assert cc[10] == 0.0 and cc[11] == 0.0
    # Wasserman-Faust: ((R-1)/S) * ((R-1)/(n-1)); centre of the star: (4/4)*(4/11)
    assert cc[5] == (4 / 4) * (4 / 11), cc[5]
    P = o.penalised(n, S, R)
    assert P[10] == n * (n - 1)
    assert P[5] == 4 + n * (n - 5)


def pin_floyd_warshall(o):
    """BFS sums, reach, 2-hop counts and eccentricity against Floyd-Warshall
    on random graphs, many of them disconnected."""
    rng = np.random.default_rng(11662)
    for trial in range(40):
        n = int(rng.integers(1, 48))
        p = float(rng.choice([0.02, 0.05, 0.1, 0.3]))
        eu, ev = random_graph(rng, n, p)
        adj = adjacency_sets(n, eu, ev)
        D = floyd_warshall(n, adj)
        fin = np.isfinite(D)
        S_ref = np.where(fin, D, 0).sum(1).astype(np.int64)
        R_ref = fin.sum(1)
        H2_ref = (D == 2).sum(1)
        ecc_ref = np.where(fin, D, 0).max(1).astype(int) if n else np.zeros(0, int)
        rp, ci = csr_of(o, n, eu, ev)
        S, R, H2, ecc, ce = o.bfs_sums(rp, ci, extras=True)
        assert np.array_equal(S, S_ref), (trial, S, S_ref)
        assert np.array_equal(R, R_ref), (trial, R, R_ref)
        assert np.array_equal(H2, H2_ref), (trial, H2, H2_ref)
        assert np.array_equal(ecc, ecc_ref), (trial, ecc, ecc_ref)
        assert np.array_equal(R, components(n, adj)), trial
        deg = np.array([len(a) for a in adj])
        ce_ref = np.array([deg[fin[u]].sum() // 2 for u in range(n)])
        assert np.array_equal(ce, ce_ref), trial
        # a subset of sources gives the same per-source values
        if n:
            src = rng.choice(n, size=min(n, 5), replace=False).astype(np.int32)
            S2, R2 = o.bfs_sums(rp, ci, sources=src)
            assert np.array_equal(S2, S_ref[src]) and np.array_equal(R2, R_ref[src])


def pin_networkx(o):
    """Closeness bit-identical to networkx.closeness_centrality, the routine
    the paper uses (Sec. 4), including disconnected graphs."""
    import networkx as nx
    rng = np.random.default_rng(2207)
    for trial in range(30):
        n = int(rng.integers(1, 60))
        p = float(rng.choice([0.03, 0.08, 0.2]))
        eu, ev = random_graph(rng, n, p)
        adj = adjacency_sets(n, eu, ev)
        ref = nx.closeness_centrality(nx_graph(n, adj))
        ref = np.array([ref[i] for i in range(n)], np.float64)
        rp, ci = csr_of(o, n, eu, ev)
        S, R = o.bfs_sums(rp, ci)
        cc = o.closeness_wf(n, S, R)
        assert np.array_equal(cc.view(np.int64), ref.view(np.int64)), (trial, cc, ref)


def pin_networkx_config1(o):
    """Closeness bit-identical to networkx.closeness_centrality on every
    graph of the small three-layer HoMLN (1,000 vertices): its layers and
    their AND and OR aggregates (Sec. 3.1), the aggregates built here with
    Python set algebra.  The AND graph has hundreds of components, so the
    Wasserman-Faust form (Sec. 4) is exercised throughout."""
    import networkx as nx
    from homln_inputs import configs as C
    h = C.config1()
    n = h.n
    sets = [{(min(a, b), max(a, b)) for a, b in zip(eu.tolist(), ev.tolist()) if a != b} for eu, ev in h.layers]
    graphs = [(eu, ev) for eu, ev in h.layers]
    for agg in (set.intersection(*sets), set.union(*sets)):
        pairs = sorted(agg)
        graphs.append((np.array([a for a, _ in pairs], np.int64), np.array([b for _, b in pairs], np.int64)))
    for gi, (eu, ev) in enumerate(graphs):
        g = nx.Graph()
        g.add_nodes_from(range(n))
        g.add_edges_from(zip(np.asarray(eu).tolist(), np.asarray(ev).tolist()))
        ref = nx.closeness_centrality(g)
        ref = np.array([ref[i] for i in range(n)], np.float64)
        rp, ci = csr_of(o, n, eu, ev)
        S, R = o.bfs_sums(rp, ci)
        cc = o.closeness_wf(n, S, R)
        bad = np.nonzero(cc.view(np.int64) != ref.view(np.int64))[0]
        assert len(bad) == 0, (gi, bad[:10])


def pin_cc2_score(o):
    """CC2's score (n-1)/est (Sec. 5.2, then Eq. 1) by two routes that do
    not use the oracle's closeness: with identical connected layers the
    estimate is the exact distance sum, so the score equals NetworkX's
    closeness bit for bit (Sec. 4: the decoupled method is exact when the
    layers agree); on arbitrary layers it equals (n-1)/P with P taken from
    Floyd-Warshall distances, unreachable vertices at distance n (Sec. 5.1),
    the largest over the layers (one IEEE division)."""
    import networkx as nx
    rng = np.random.default_rng(31)
    for trial in range(12):
        n = int(rng.integers(3, 45))
        # a connected layer: a random spanning tree plus random edges
        par = [int(rng.integers(0, i)) for i in range(1, n)]
        eu = np.arange(1, n, dtype=np.int64)
        ev = np.array(par, np.int64)
        xu, xv = random_graph(rng, n, 0.08)
        eu, ev = np.concatenate([eu, xu]), np.concatenate([ev, xv])
        adj = adjacency_sets(n, eu, ev)
        ref = nx.closeness_centrality(nx_graph(n, adj))
        ref = np.array([ref[i] for i in range(n)], np.float64)
        S, R = o.bfs_sums(*csr_of(o, n, eu, ev))
        r = int(rng.integers(1, 4))
        est = o.cc2_est(n, [S] * r, [R] * r)
        sc = o.cc2_score(n, est)
        assert np.array_equal(sc.view(np.int64), ref.view(np.int64)), (trial, sc, ref)
    for trial in range(12):
        n = int(rng.integers(2, 40))
        r = int(rng.integers(2, 4))
        Ps, Ss, Rs = [], [], []
        for _l in range(r):
            u, v = random_graph(rng, n, float(rng.choice([0.04, 0.1])))
            adj = adjacency_sets(n, u, v)
            D = floyd_warshall(n, adj)
            Ps.append([int(np.where(np.isinf(D[x]), n, D[x]).sum()) for x in range(n)])
            S, R = o.bfs_sums(*csr_of(o, n, u, v))
            Ss.append(S)
            Rs.append(R)
        P = np.array(Ps, np.int64).max(0)
        sc = o.cc2_score(n, o.cc2_est(n, Ss, Rs))
        ref = np.array([(n - 1) / int(p) if p > 0 else 0.0 for p in P.tolist()], np.float64)
        assert np.array_equal(sc.view(np.int64), ref.view(np.int64)), (trial, sc, ref)


def pin_networkx_printed(o):
    """Values NetworkX prints for P5 and K1,4 (stored fixture)."""
    with open(os.path.join(GOLDEN, "networkx_closeness_small.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    for kind, arg, *vals in rows:
        n, eu, ev = G.named_graph(kind, int(arg))
        rp, ci = csr_of(o, n, eu, ev)
        S, R = o.bfs_sums(rp, ci)
        cc = o.closeness_wf(n, S, R)
        ref = np.array([float(x) for x in vals])
        assert np.array_equal(cc, ref), (kind, cc, ref)


def pin_wiener_tree(o):
    """On a tree, sum_u S(u) = 2 * sum over edges of n1*n2 (Wiener index)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = int(rng.integers(2, 80))
        parent = [int(rng.integers(0, v)) for v in range(1, n)]
        eu = np.array(parent)
        ev = np.arange(1, n)
        # subtree sizes
        size = np.ones(n, int)
        for v in range(n - 1, 0, -1):
            size[parent[v - 1]] += size[v]
        wiener = sum(int(size[v]) * (n - int(size[v])) for v in range(1, n))
        rp, ci = csr_of(o, n, eu, ev)
        S, R = o.bfs_sums(rp, ci)
        assert int(S.sum()) == 2 * wiener


def pin_csr_normalisation(o):
    """Self-loops dropped, duplicates merged, both orientations, rows sorted."""
    rng = np.random.default_rng(7)
    for _ in range(30):
        n = int(rng.integers(1, 40))
        m = int(rng.integers(0, 120))
        eu = rng.integers(0, n, size=m)
        ev = rng.integers(0, n, size=m)
        adj = adjacency_sets(n, eu, ev)
        rp, ci = csr_of(o, n, eu, ev)
        assert len(rp) == n + 1 and rp[0] == 0
        for u in range(n):
            row = ci[rp[u]:rp[u + 1]].tolist()
            assert row == sorted(adj[u]), (u, row, sorted(adj[u]))


def pin_compose_sets(o):
    """AND / OR aggregation (Sec. 3.1) against Python set algebra, plus
    AND within every layer within OR, idempotence and the empty layer."""
    rng = np.random.default_rng(9)
    for _ in range(25):
        n = int(rng.integers(2, 40))
        r = int(rng.integers(1, 5))
        layers, sets = [], []
        base_u, base_v = random_graph(rng, n, 0.15)
        for _l in range(r):
            u, v = random_graph(rng, n, 0.1)
            keep = rng.random(len(base_u)) < 0.8
            eu = np.concatenate([u, base_u[keep]])
            ev = np.concatenate([v, base_v[keep]])
            layers.append(csr_of(o, n, eu, ev))
            sets.append({(min(a, b), max(a, b)) for a, b in zip(eu.tolist(), ev.tolist()) if a != b})
        and_ref = set.intersection(*sets)
        or_ref = set.union(*sets)
        for mode, ref in (("and", and_ref), ("or", or_ref)):
            rp, ci = o.compose(mode, layers)
            got = {(u, int(v)) for u in range(n) for v in ci[rp[u]:rp[u + 1]] if u < v}
            assert got == ref, (mode, got ^ ref)
            sym = {(int(v), u) for u in range(n) for v in ci[rp[u]:rp[u + 1]] if u > v}
            assert sym == ref
        rp, ci = o.compose("and", [layers[0], layers[0]])
        assert np.array_equal(rp, layers[0][0]) and np.array_equal(ci, layers[0][1])
        rp, ci = o.compose("or", [layers[0], layers[0], layers[0]])
        assert np.array_equal(rp, layers[0][0]) and np.array_equal(ci, layers[0][1])
        empty = (np.zeros(n + 1, np.int32), np.zeros(0, np.int32))
        rp, ci = o.compose("and", [layers[0], empty])
        assert rp[-1] == 0


def pin_mean_exact(o):
    """Fixed-shape mean within 4 ulp of the exact rational mean."""
    rng = np.random.default_rng(13)
    for size in (1, 2, 7, 1023, 1024, 1025, 5000):
        x = rng.random(size) * rng.choice([1e-3, 1.0, 10.0])
        exact = sum(Fraction(float(v)) for v in x) / size
        got = o.mean_fixed_shape(x)
        assert abs(Fraction(got) - exact) <= 4 * Fraction(math.ulp(float(exact))), (size, got, float(exact))


def pin_above_mean(o):
    """'Same or above average' (Sec. 4): a vertex-transitive graph makes
    every vertex a CC node; on a star only the centre is."""
    for kind, arg, expect in (("cycle", 9, list(range(9))), ("star", 6, [0]), ("hypercube", 3, list(range(8)))):
        n, eu, ev = G.named_graph(kind, arg)
        rp, ci = csr_of(o, n, eu, ev)
        S, R = o.bfs_sums(rp, ci)
        cc = o.closeness_wf(n, S, R)
        assert o.above_mean(cc).tolist() == expect, (kind, o.above_mean(cc))
    rng = np.random.default_rng(17)
    for _ in range(20):
        x = rng.integers(0, 5, size=int(rng.integers(1, 50))).astype(np.float64) / 4.0
        mean = Fraction(sum(Fraction(float(v)) for v in x)) / len(x)
        ref = [i for i, v in enumerate(x.tolist()) if Fraction(v) >= mean]
        assert o.above_mean(x).tolist() == ref


def pin_topk(o):
    """Top-k by score descending, ties by ascending id (brute force)."""
    rng = np.random.default_rng(19)
    for _ in range(30):
        size = int(rng.integers(1, 200))
        x = rng.integers(0, 6, size=size).astype(np.float64) / 3.0
        k = int(rng.integers(0, size + 3))
        ref = sorted(range(size), key=lambda i: (-x[i], i))[:k]
        assert o.topk_desc(x, k).tolist() == ref
        key = rng.integers(0, 6, size=size).astype(np.int64)
        ref = sorted(range(size), key=lambda i: (key[i], i))[:k]
        assert o.topk_asc_i64(key, k).tolist() == ref


def pin_cc2_worked_example(o):
    """Sec. 5.2: node A with layer sums 9 and 7 gets the estimate 9."""
    with open(os.path.join(GOLDEN, "cc2_worked_example.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    for n, s_x, s_y, want in rows:
        n = int(n)
        # connected layers: R = n, so the penalty term vanishes
        est = o.cc2_est(n, [np.full(n, int(s_x)), np.full(n, int(s_y))], [np.full(n, n), np.full(n, n)])
        assert np.all(est == int(want)), (est, want)


def pin_cc2_bounds(o):
    """Sec. 5.2: the AND graph's (penalised) distance sum of u is at least
    max over layers; dually the OR graph's is at most the min; with
    identical layers the estimate is exact (Sec. 4, naive = ground truth)."""
    rng = np.random.default_rng(23)
    for _ in range(20):
        n = int(rng.integers(2, 50))
        r = int(rng.integers(2, 4))
        base_u, base_v = random_graph(rng, n, 0.12)
        layers = []
        for _l in range(r):
            u, v = random_graph(rng, n, 0.06)
            layers.append(csr_of(o, n, np.concatenate([u, base_u]), np.concatenate([v, base_v])))
        sums = [o.bfs_sums(*g) for g in layers]
        est = o.cc2_est(n, [s for s, _ in sums], [x for _, x in sums])
        Ps = np.array([o.penalised(n, s, x) for s, x in sums])
        assert np.array_equal(est, Ps.max(0))
        Sa, Ra = o.bfs_sums(*o.compose("and", layers))
        assert np.all(o.penalised(n, Sa, Ra) >= est)
        So, Ro = o.bfs_sums(*o.compose("or", layers))
        assert np.all(o.penalised(n, So, Ro) <= Ps.min(0))
        est_same = o.cc2_est(n, [sums[0][0]] * 2, [sums[0][1]] * 2)
        assert np.array_equal(est_same, o.penalised(n, *sums[0]))


def pin_naive(o):
    """Naive composition (Sec. 4) = intersection of the layers' CC-node
    sets; with identical layers it equals that layer's set."""
    rng = np.random.default_rng(29)
    for _ in range(15):
        n = int(rng.integers(2, 60))
        r = int(rng.integers(2, 4))
        ccs = []
        for _l in range(r):
            u, v = random_graph(rng, n, 0.1)
            S, R = o.bfs_sums(*csr_of(o, n, u, v))
            ccs.append(o.closeness_wf(n, S, R))
        sets = [set(o.above_mean(c).tolist()) for c in ccs]
        assert o.naive(n, ccs).tolist() == sorted(set.intersection(*sets))
        assert o.naive(n, [ccs[0], ccs[0]]).tolist() == o.above_mean(ccs[0]).tolist()


def pin_naive_topk(o):
    """Naive composition of top-k sets: the intersection of the layers'
    top-k sets (brute force: sort each layer by (-score, id), cut at k,
    intersect); identical layers give that layer's top k; k = n keeps every
    vertex, k = 0 none."""
    rng = np.random.default_rng(31)
    for _ in range(25):
        n = int(rng.integers(1, 120))
        r = int(rng.integers(1, 5))
        ccs = [rng.integers(0, 7, size=n).astype(np.float64) / 5.0 for _l in range(r)]
        k = int(rng.integers(0, n + 1))
        tops = [set(sorted(range(n), key=lambda i, c=c: (-c[i], i))[:k]) for c in ccs]
        assert o.naive_topk(n, ccs, k).tolist() == sorted(set.intersection(*tops))
        assert o.naive_topk(n, [ccs[0], ccs[0]], k).tolist() == sorted(o.topk_desc(ccs[0], k).tolist())
        assert o.naive_topk(n, ccs, n).tolist() == list(range(n))
        assert o.naive_topk(n, ccs, 0).tolist() == []


def pin_sample_sums(o):
    """Sample sums against Floyd-Warshall (sum and count over the sampled
    rows of each column), both the per-source and the per-vertex routes."""
    rng = np.random.default_rng(2004)
    for trial in range(30):
        n = int(rng.integers(2, 48))
        eu, ev = random_graph(rng, n, float(rng.choice([0.03, 0.08, 0.3])))
        adj = adjacency_sets(n, eu, ev)
        D = floyd_warshall(n, adj)
        k = int(rng.integers(1, n + 1))
        src = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)
        fin = np.isfinite(D[src])
        SQ_ref = np.where(fin, D[src], 0).sum(0).astype(np.int64)
        RQ_ref = fin.sum(0)
        rp, ci = csr_of(o, n, eu, ev)
        SQ, RQ = o.sample_sums(rp, ci, src)
        assert np.array_equal(SQ, SQ_ref), trial
        assert np.array_equal(RQ, RQ_ref), trial
        verts = rng.choice(n, size=min(n, 7), replace=False).astype(np.int32)
        S2, R2 = o.sample_sums_at(rp, ci, src, verts)
        assert np.array_equal(S2, SQ_ref[verts]) and np.array_equal(R2, RQ_ref[verts]), trial


def pin_sample_estimate_full_sample(o):
    """With every vertex sampled the estimate is the exact closeness, bit for
    bit (Floyd-Warshall sums through the closed form of Sec. 4, Eq. 1 in the
    Wasserman-Faust form), on connected and disconnected graphs."""
    rng = np.random.default_rng(7)
    for trial in range(25):
        n = int(rng.integers(2, 40))
        eu, ev = random_graph(rng, n, float(rng.choice([0.03, 0.1, 0.4])))
        adj = adjacency_sets(n, eu, ev)
        D = floyd_warshall(n, adj)
        fin = np.isfinite(D)
        S = np.where(fin, D, 0).sum(1)
        R = fin.sum(1)
        exact = np.array([((R[v] - 1) / S[v]) * ((R[v] - 1) / (n - 1)) if R[v] > 1 else 0.0 for v in range(n)])
        rp, ci = csr_of(o, n, eu, ev)
        src = np.arange(n, dtype=np.int32)
        SQ, RQ = o.sample_sums(rp, ci, src)
        est = o.sample_estimate(n, n, src, SQ, RQ)
        assert np.array_equal(est.view(np.int64), exact.view(np.int64)), trial
        # isolated vertices outside the population: sampling every vertex of
        # degree >= 1 (n_pop of them) still gives the exact closeness
        deg = np.array([len(a) for a in adj])
        pop = np.flatnonzero(deg > 0).astype(np.int32)
        if 1 < len(pop) < n:
            SQ, RQ = o.sample_sums(rp, ci, pop)
            est = o.sample_estimate(n, len(pop), pop, SQ, RQ)
            assert np.allclose(est, exact, rtol=1e-13, atol=0), trial


def pin_sample_estimate_bound(o):
    """Mean-distance estimate within Hoeffding's bound on a connected graph:
    |SQ/q - S/(n-1)| <= diam * sqrt(ln(2n/delta) / (2k)) for every vertex,
    delta = 1e-3 (k sources sampled uniformly without replacement), and the
    estimated closeness is then the exact one scaled by at most that error."""
    rng = np.random.default_rng(2211)
    n, k = 600, 150
    eu, ev = random_graph(rng, n, 0.004)
    eu = np.concatenate([eu, np.arange(n - 1)])            # a path keeps it connected
    ev = np.concatenate([ev, np.arange(1, n)])
    adj = adjacency_sets(n, eu, ev)
    D = floyd_warshall(n, adj)
    diam = D.max()
    src = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)
    rp, ci = csr_of(o, n, eu, ev)
    SQ, RQ = o.sample_sums(rp, ci, src)
    mask = np.zeros(n, bool)
    mask[src] = True
    q = RQ - mask
    mean_est = SQ / q
    mean_true = D.sum(1) / (n - 1)
    eps = diam * math.sqrt(math.log(2 * n / 1e-3) / (2 * k))
    assert np.all(np.abs(mean_est - mean_true) <= eps)
    est = o.sample_estimate(n, n, src, SQ, RQ)
    exact = 1.0 / mean_true                                   # connected: WF factor 1
    assert np.allclose(est, (1.0 / mean_est) * (q / (k - mask)), rtol=1e-12)
    assert np.all(np.abs(1.0 / est - 1.0 / exact) <= eps + 1e-9)


def cc1_brute(n, adjs, tau):
    """CC1 from the definitions in Sec. 5.1 (Eq. 2-3) with exact rationals:
    distances from Floyd-Warshall, sets as Python sets.  Returns (ids, tie)
    where tie says some comparison sat within 1e-9 of its threshold (the
    FP64 result may then round the other way)."""
    r = len(adjs)
    Ds = [floyd_warshall(n, a) for a in adjs]
    m = [min(len(a[u]) for a in adjs) for u in range(n)]
    ratios, avgs, ch = [], [], []
    tie = False
    for D, a in zip(Ds, adjs):
        P = [int(sum(d if np.isfinite(d) else n for j, d in enumerate(D[u]) if j != u)) for u in range(n)]
        ratio = [Fraction(P[u], m[u]) if m[u] > 0 else None for u in range(n)]
        valid = [x for x in ratio if x is not None]
        avgs.append(sum(valid, Fraction(0)) / len(valid) if valid else Fraction(0))
        ratios.append(ratio)
        reach = [int(np.isfinite(D[u]).sum()) for u in range(n)]
        S = [int(sum(d for d in D[u] if np.isfinite(d))) for u in range(n)]
        cc = [Fraction((reach[u] - 1) ** 2, S[u] * (n - 1)) if reach[u] > 1 and S[u] > 0 and n > 1 else Fraction(0)
              for u in range(n)]
        mean = sum(cc, Fraction(0)) / n
        tie |= any(x != mean and abs(x - mean) <= mean * Fraction(1, 10 ** 9) for x in cc)
        ch.append({u for u in range(n) if cc[u] >= mean})
    avg = max(avgs)
    central = [{u for u in range(n) if ratios[l][u] is not None and ratios[l][u] < avg} for l in range(r)]
    tie |= any(x is not None and x != avg and abs(x - avg) <= avg * Fraction(1, 10 ** 9) for rl in ratios for x in rl)
    out = []
    for c in sorted(set.intersection(*ch)):
        sets = [adjs[l][c] & central[l] for l in range(r)]
        small = min(len(x) for x in sets)
        inter = len(set.intersection(*sets))
        if small > 0 and Fraction(inter, small) >= Fraction(*tau):
            out.append(c)
    return out, tie


def pin_cc1_brute_force(o):
    """CC1 (Sec. 5.1) on small random HoMLNs of 2-3 layers (shared base plus
    private edges, often disconnected) against the definitions with exact
    rationals, for several overlap thresholds."""
    rng = np.random.default_rng(31)
    checked = 0
    for trial in range(40):
        n = int(rng.integers(8, 40))
        r = int(rng.integers(2, 4))
        bu, bv = random_graph(rng, n, 0.08)
        edges = []
        for _l in range(r):
            u, v = random_graph(rng, n, 0.07)
            edges.append((np.concatenate([u, bu]), np.concatenate([v, bv])))
        adjs = [adjacency_sets(n, u, v) for u, v in edges]
        layers = [csr_of(o, n, u, v) for u, v in edges]
        sums = [o.bfs_sums(*g) for g in layers]
        for tau in ((1, 2), (0, 1), (1, 3), (1, 1)):
            want, tie = cc1_brute(n, adjs, tau)
            if tie:
                continue
            got = o.cc1(n, layers, [x[0] for x in sums], [x[1] for x in sums], tau)
            assert got.tolist() == want, (trial, tau)
            checked += 1
    assert checked >= 100


def pin_cc1_vertex_transitive(o):
    """Two identical cycles: every vertex has the same ratio, which is then
    the average itself (exact in FP64 here), so no neighbour lies strictly
    below it and CC1 is empty at every threshold, 0 included."""
    for n in (8, 16, 32):
        u = np.arange(n)
        g = csr_of(o, n, u, (u + 1) % n)
        S, R = o.bfs_sums(*g)
        for tau in ((0, 1), (1, 2), (1, 1)):
            ids, avg = o.cc1(n, [g, g], [S, S], [R, R], tau, with_avg=True)
            assert avg == n * n / 8.0
            assert len(ids) == 0


def pin_cc1_properties(o):
    """CC1 keeps only common CC nodes (a subset of the naive composition,
    Sec. 4); raising the threshold never adds a node; the overlap is at most
    1, so a threshold above 1 keeps nothing; identical layers overlap fully,
    so every threshold up to 1 keeps the same set."""
    rng = np.random.default_rng(37)
    for trial in range(15):
        n = int(rng.integers(10, 60))
        bu, bv = random_graph(rng, n, 0.1)
        edges = []
        for _l in range(2):
            u, v = random_graph(rng, n, 0.06)
            edges.append((np.concatenate([u, bu]), np.concatenate([v, bv])))
        layers = [csr_of(o, n, u, v) for u, v in edges]
        sums = [o.bfs_sums(*g) for g in layers]
        Ss, Rs = [x[0] for x in sums], [x[1] for x in sums]
        naive = set(o.naive(n, [o.closeness_wf(n, S, R) for S, R in zip(Ss, Rs)]).tolist())
        prev = None
        for tau in ((0, 1), (1, 4), (1, 2), (3, 4), (1, 1), (5, 4)):
            got = set(o.cc1(n, layers, Ss, Rs, tau).tolist())
            assert got <= naive
            if prev is not None:
                assert got <= prev
            prev = got
        assert not prev
        same = [set(o.cc1(n, [layers[0]] * 2, [Ss[0]] * 2, [Rs[0]] * 2, tau).tolist())
                for tau in ((0, 1), (1, 2), (1, 1))]
        assert same[0] == same[1] == same[2]


PINS = [pin_closed_forms, pin_disjoint_union, pin_floyd_warshall, pin_networkx, pin_networkx_printed,
        pin_wiener_tree, pin_csr_normalisation, pin_compose_sets, pin_mean_exact, pin_above_mean,
        pin_topk, pin_cc2_worked_example, pin_cc2_bounds, pin_naive, pin_sample_sums,
        pin_sample_estimate_full_sample, pin_sample_estimate_bound, pin_cc1_brute_force, pin_cc1_vertex_transitive,
        pin_cc1_properties, pin_cc2_score, pin_networkx_config1, pin_naive_topk]
