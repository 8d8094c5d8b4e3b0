"""The five seeded workloads, as HoMLNs of canonical edge lists.

Config 1  3 layers x 1,000 vertices: shared Erdos-Renyi base (avg degree 6),
          each layer keeps a base edge with probability 0.5 and adds private
          ER edges up to avg degree 8.
Config 2  4 layers x 100,000 vertices: Chung-Lu power law (exponent 2.5,
          avg degree 10), 30% of each layer's edges from a common base.
Config 3  64 HoMLNs, 2-8 layers, n log-uniform in [2,000, 50,000]; layers
          alternate ER (avg degree 4-16) and Barabasi-Albert (m = 3-8) with
          20-50% shared base edges.
Config 4  6 layers x 1,000,000 vertices: R-MAT (0.57, 0.19, 0.19, 0.05), avg
          degree 16, 25% shared base; 16,384 sampled sources per graph.
Config 5  5 layers x 200,000 vertices: Chung-Lu (exponent 2.2-2.8, avg degree
          8-20), 30% shared base.

Every HoMLN gets one seeded vertex relabelling applied to all of its layers,
so vertex ids carry no generator locality (hubs are not the low ids).
``scale`` shrinks vertex counts for quick tests while keeping the recipe.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
import numpy as np

from . import generators as G


@dataclass
class HoMLN:
    name: str
    n: int
    layers: list                      # list of (eu, ev) canonical int32 arrays
    meta: dict = field(default_factory=dict)

    @property
    def m(self):
        return [len(e[0]) for e in self.layers]


def _assemble(cfg: int, h: int, n: int, base_keys: np.ndarray, private: list, name: str, meta=None):
    perm = G.rng_for(cfg, h, 254).permutation(n)
    layers = []
    for keys in private:
        allk = np.concatenate([base_keys, keys]) if len(base_keys) else keys
        layers.append(G.keys_to_edges(allk, n, perm))
    return HoMLN(name, n, layers, meta or {})


def config1(scale: float = 1.0) -> HoMLN:
    n = max(8, int(round(1000 * scale)))
    base_m = n * 6 // 2
    m = n * 8 // 2
    base = G.take_distinct(G.er_draw(n), base_m, n, G.rng_for(1, 0, 255))
    priv = []
    for l in range(3):
        rng = G.rng_for(1, 0, l)
        kept = base[rng.random(len(base)) < 0.5]
        extra = G.take_distinct(G.er_draw(n), m - len(kept), n, rng, exclude=np.sort(kept))
        priv.append(np.concatenate([kept, extra]))
    return _assemble(1, 0, n, np.zeros(0, np.int64), priv, "cfg1-er-3x%d" % n,
                     {"layers": 3, "family": "ER"})


def _shared_homln(cfg: int, h: int, n: int, base_draw, base_m: int, layer_specs, name: str, meta=None):
    """layer_specs: list of ("stream", draw, m) or ("ba", m_ba)."""
    base = G.take_distinct(base_draw, base_m, n, G.rng_for(cfg, h, 255)) if base_m > 0 else np.zeros(0, np.int64)
    base_sorted = np.sort(base)
    priv = []
    for l, spec in enumerate(layer_specs):
        rng = G.rng_for(cfg, h, l)
        if spec[0] == "stream":
            _, draw, m = spec
            priv.append(G.take_distinct(draw, max(0, m - len(base)), n, rng, exclude=base_sorted))
        else:
            _, m_ba = spec
            ba = G.barabasi_albert_keys(n, m_ba, rng)
            priv.append(ba[~np.isin(ba, base_sorted)])
    return _assemble(cfg, h, n, base, priv, name, meta)


def config2(scale: float = 1.0) -> HoMLN:
    n = max(64, int(round(100_000 * scale)))
    m = n * 10 // 2
    draw = G.chung_lu_draw(n, 2.5)
    specs = [("stream", draw, m) for _ in range(4)]
    return _shared_homln(2, 0, n, draw, int(math.ceil(0.30 * m)), specs, "cfg2-chunglu-4x%d" % n,
                         {"layers": 4, "family": "Chung-Lu", "gamma": 2.5, "avg_degree": 10, "shared": 0.30})


def config3_params(h: int, scale: float = 1.0):
    rng = G.rng_for(3, h, 253)
    nl = int(rng.integers(2, 9))
    n = int(round(math.exp(rng.uniform(math.log(2000), math.log(50000)))))
    n = max(32, int(round(n * scale)))
    f = float(rng.uniform(0.2, 0.5))
    kinds = []
    for j in range(nl):
        if j % 2 == 0:
            kinds.append(("er", int(rng.integers(4, 17))))
        else:
            kinds.append(("ba", int(rng.integers(3, 9))))
    return nl, n, f, kinds


def config3_homln(h: int, scale: float = 1.0) -> HoMLN:
    nl, n, f, kinds = config3_params(h, scale)
    ms = [n * d // 2 if k == "er" else n * d for k, d in kinds]
    base_m = int(math.ceil(f * min(ms)))
    specs = []
    for (k, d), m in zip(kinds, ms):
        specs.append(("stream", G.er_draw(n), m) if k == "er" else ("ba", d))
    return _shared_homln(3, h, n, G.er_draw(n), base_m, specs, "cfg3-h%02d-%dx%d" % (h, nl, n),
                         {"layers": nl, "kinds": kinds, "shared": f})


def config3(count: int = 64, scale: float = 1.0) -> list:
    return [config3_homln(h, scale) for h in range(count)]


def _rmat_private(n: int, l: int, m: int, base_sorted: np.ndarray) -> np.ndarray:
    """Config 4's private edges of layer l (a process-pool task)."""
    return G.take_distinct(G.rmat_draw(n), max(0, m - len(base_sorted)), n, G.rng_for(4, 0, l), exclude=base_sorted)


def config4(scale: float = 1.0, workers: int = 1, progress=None) -> HoMLN:
    """workers > 1 draws the six private edge streams in that many spawned
    processes (each stream has its own seed, so the result is the same);
    progress(str) is called after the base and after each layer."""
    n = max(256, int(round(1_000_000 * scale)))
    m = n * 16 // 2
    base = G.take_distinct(G.rmat_draw(n), int(math.ceil(0.25 * m)), n, G.rng_for(4, 0, 255))
    base_sorted = np.sort(base)
    if progress:
        progress("config 4: base of %d edges drawn" % len(base))
    priv = [None] * 6
    if workers > 1:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor, as_completed
        with ProcessPoolExecutor(max_workers=min(workers, 6), mp_context=mp.get_context("spawn")) as ex:
            futs = {ex.submit(_rmat_private, n, l, m, base_sorted): l for l in range(6)}
            for f in as_completed(futs):
                priv[futs[f]] = f.result()
                if progress:
                    progress("config 4: layer %d drawn" % futs[f])
    else:
        for l in range(6):
            priv[l] = _rmat_private(n, l, m, base_sorted)
            if progress:
                progress("config 4: layer %d drawn" % l)
    return _assemble(4, 0, n, base, priv, "cfg4-rmat-6x%d" % n,
                     {"layers": 6, "family": "R-MAT", "avg_degree": 16, "shared": 0.25})


def config4_sources(g: int, deg: np.ndarray, count: int = 16384) -> np.ndarray:
    """Uniform sample without replacement over vertices of degree >= 1 of
    graph g (layers 0..5, AND = 6), in ascending id order."""
    cand = np.nonzero(deg > 0)[0]
    rng = G.rng_for(4, 0, 512 + g)
    k = min(count, len(cand))
    return np.sort(rng.choice(cand, size=k, replace=False)).astype(np.int32)


def config5(scale: float = 1.0) -> HoMLN:
    n = max(64, int(round(200_000 * scale)))
    rng = G.rng_for(5, 0, 253)
    gammas = [float(rng.uniform(2.2, 2.8)) for _ in range(5)]
    degs = [int(rng.integers(8, 21)) for _ in range(5)]
    ms = [n * d // 2 for d in degs]
    specs = [("stream", G.chung_lu_draw(n, g), m) for g, m in zip(gammas, ms)]
    base_draw = G.chung_lu_draw(n, sum(gammas) / len(gammas))
    return _shared_homln(5, 0, n, base_draw, int(math.ceil(0.30 * min(ms))), specs, "cfg5-chunglu-5x%d" % n,
                         {"layers": 5, "gammas": gammas, "avg_degrees": degs, "shared": 0.30})


def make_config(i: int, scale: float = 1.0):
    return {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}[i](scale=scale)
