"""Seeded synthetic graph generators for homogeneous multilayer networks.

This module is shared by the CPU oracle side and the HIP side, and for that
reason it holds none of the method's arithmetic: it draws edges and nothing
else (no BFS, no distance sums, no closeness, no aggregation, no ranking).

Every graph is returned as a canonical undirected edge list: two int32
arrays ``(eu, ev)`` with ``eu < ev``, no duplicates, sorted by ``(eu, ev)``.
The paper's layers are simple undirected graphs over one shared vertex set
(Sec. 1, Problem Statement); its own data sets (PaRMAT R-MAT layers whose
edges are split between layers, Sec. 6, Table 1) are not available, so these
generators stand in for them with the same structure: every layer of a
HoMLN contains a common base edge set plus private edges.
"""
from __future__ import annotations

import math
import numpy as np

SEED_ROOT = 220711662


def rng_for(cfg: int, homln: int, stream: int) -> np.random.Generator:
    """PCG64 seeded by SeedSequence([220711662, cfg, homln, stream]).

    stream: layer index for a layer's private edges; 255 the shared base;
    254 the label permutation; 253 per-HoMLN parameters; 512+g source
    samples of graph g."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, cfg, homln, stream])))


# ---------------------------------------------------------------------------
# distinct-edge streams
# ---------------------------------------------------------------------------

def _canon_keys(u: np.ndarray, v: np.ndarray, n: int) -> np.ndarray:
    u = u.astype(np.int64)
    v = v.astype(np.int64)
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    keys = lo * n + hi
    return keys[lo != hi]


def _first_distinct(keys: np.ndarray) -> np.ndarray:
    """Keys in order of first appearance, duplicates removed."""
    if len(keys) == 0:
        return keys
    _, idx = np.unique(keys, return_index=True)
    return keys[np.sort(idx)]


def take_distinct(draw, want: int, n: int, rng: np.random.Generator,
                  exclude: np.ndarray | None = None, max_rounds: int = 200) -> np.ndarray:
    """First ``want`` distinct canonical edge keys of the stream ``draw``.

    draw(rng, k) -> (u, v) candidate endpoints (self-loops allowed, they are
    dropped).  Keys in ``exclude`` (sorted) are skipped.  Returns int64 keys
    in stream order."""
    out = np.zeros(0, np.int64)
    seen = np.zeros(0, np.int64) if exclude is None else np.asarray(exclude, np.int64)
    rounds = 0
    while len(out) < want:
        rounds += 1
        if rounds > max_rounds:
            raise RuntimeError("edge stream exhausted: asked for %d distinct edges on n=%d" % (want, n))
        need = want - len(out)
        k = int(need * 1.25) + 1024
        u, v = draw(rng, k)
        keys = _first_distinct(_canon_keys(u, v, n))
        if len(seen):
            keys = keys[~np.isin(keys, seen, assume_unique=False)]
        keys = keys[:need]
        out = np.concatenate([out, keys])
        seen = np.union1d(seen, keys)
    return out


def keys_to_edges(keys: np.ndarray, n: int, perm: np.ndarray | None = None):
    """Canonical, sorted (eu, ev) int32 arrays from edge keys, after an
    optional vertex relabelling ``perm`` (old id -> new id)."""
    keys = np.asarray(keys, np.int64)
    u = keys // n
    v = keys % n
    if perm is not None:
        u = perm[u]
        v = perm[v]
    k = np.unique(_canon_keys(u, v, n))
    return (k // n).astype(np.int32), (k % n).astype(np.int32)


# ---------------------------------------------------------------------------
# families
# ---------------------------------------------------------------------------

def er_draw(n: int):
    """Uniform vertex pairs (Erdos-Renyi G(n, M) when taken distinct)."""
    def draw(rng, k):
        return rng.integers(0, n, size=k), rng.integers(0, n, size=k)
    return draw


def chung_lu_weights(n: int, gamma: float) -> np.ndarray:
    """w_i proportional to (i+1)^(-1/(gamma-1)): expected degrees follow a
    power law with exponent gamma."""
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (gamma - 1.0))
    return w / w.sum()


def chung_lu_draw(n: int, gamma: float):
    """Both endpoints drawn independently with probability proportional to
    the Chung-Lu weight."""
    cdf = np.cumsum(chung_lu_weights(n, gamma))
    cdf[-1] = 1.0

    def draw(rng, k):
        a = np.searchsorted(cdf, rng.random(k), side="right")
        b = np.searchsorted(cdf, rng.random(k), side="right")
        return np.minimum(a, n - 1), np.minimum(b, n - 1)
    return draw


def rmat_draw(n: int, a: float = 0.57, b: float = 0.19, c: float = 0.19):
    """R-MAT: one quadrant choice per bit of a 2^scale x 2^scale adjacency
    matrix, no noise.  Endpoints >= n are rejected (n need not be a power of
    two)."""
    scale = max(1, int(math.ceil(math.log2(max(n, 2)))))

    def draw(rng, k):
        u = np.zeros(k, np.int64)
        v = np.zeros(k, np.int64)
        for _ in range(scale):
            r = rng.random(k)
            bu = (r >= a + b).astype(np.int64)                 # lower half: quadrants c, d
            bv = ((r >= a) & (r < a + b)) | (r >= a + b + c)   # right half: quadrants b, d
            u = (u << 1) | bu
            v = (v << 1) | bv.astype(np.int64)
        keep = (u < n) & (v < n)
        return u[keep], v[keep]
    return draw


def barabasi_albert_keys(n: int, m_ba: int, rng: np.random.Generator) -> np.ndarray:
    """Preferential attachment: a clique on m_ba+1 vertices, then every new
    vertex attaches to m_ba distinct earlier vertices chosen with probability
    proportional to degree.  Returns canonical keys in creation order."""
    m0 = m_ba + 1
    if n <= m0:
        iu, iv = np.triu_indices(n, 1)
        return iu.astype(np.int64) * n + iv
    iu, iv = np.triu_indices(m0, 1)
    keys = [iu.astype(np.int64) * n + iv]
    ends = np.zeros(2 * (len(iu) + (n - m0) * m_ba), np.int64)
    ne = 2 * len(iu)
    ends[:ne:2] = iu
    ends[1:ne:2] = iv
    for t in range(m0, n):
        chosen: list[int] = []
        while len(chosen) < m_ba:
            cand = ends[rng.integers(0, ne, size=2 * m_ba)]
            for x in cand.tolist():
                if x not in chosen:
                    chosen.append(x)
                    if len(chosen) == m_ba:
                        break
        ch = np.array(chosen, np.int64)
        keys.append(ch * n + t)
        ends[ne:ne + m_ba] = ch
        ends[ne + m_ba:ne + 2 * m_ba] = t
        ne += 2 * m_ba
    return np.concatenate(keys)


# ---------------------------------------------------------------------------
# small named graphs (closed-form fixtures)
# ---------------------------------------------------------------------------

def named_graph(kind: str, *args):
    """Edge lists of textbook graphs on ids 0..n-1 (not canonicalised beyond
    u < v)."""
    if kind == "path":
        (n,) = args
        u = np.arange(n - 1)
        return n, u, u + 1
    if kind == "star":
        (n,) = args
        return n, np.zeros(n - 1, np.int64), np.arange(1, n)
    if kind == "cycle":
        (n,) = args
        u = np.arange(n)
        v = (u + 1) % n
        return n, np.minimum(u, v), np.maximum(u, v)
    if kind == "complete":
        (n,) = args
        iu, iv = np.triu_indices(n, 1)
        return n, iu, iv
    if kind == "bipartite":
        a, b = args
        iu = np.repeat(np.arange(a), b)
        iv = a + np.tile(np.arange(b), a)
        return a + b, iu, iv
    if kind == "hypercube":
        (k,) = args
        n = 1 << k
        us, vs = [], []
        for x in range(n):
            for bit in range(k):
                y = x ^ (1 << bit)
                if x < y:
                    us.append(x)
                    vs.append(y)
        return n, np.array(us), np.array(vs)
    raise ValueError(kind)


def to_edges(n: int, u, v):
    """Canonical sorted (eu, ev) of an arbitrary edge list."""
    k = np.unique(_canon_keys(np.asarray(u), np.asarray(v), n))
    return (k // n).astype(np.int32), (k % n).astype(np.int32)
