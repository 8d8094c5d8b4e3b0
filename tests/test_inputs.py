"""The seeded workload generators: canonical form, sizes, determinism and
the shared-base structure of a HoMLN (every layer holds the base edges)."""
import numpy as np
import pytest

from homln_inputs import configs as C
from homln_inputs import generators as G


def _check_canonical(n, eu, ev):
    assert eu.dtype == np.int32 and ev.dtype == np.int32
    assert np.all(eu < ev) and np.all(eu >= 0) and np.all(ev < n)
    keys = eu.astype(np.int64) * n + ev
    assert np.all(np.diff(keys) > 0)  # sorted, unique


@pytest.mark.parametrize("cfg,scale", [(1, 1.0), (2, 0.05), (4, 0.002), (5, 0.02)])
def test_config_shapes(cfg, scale):
    h = C.make_config(cfg, scale)
    n = h.n
    for eu, ev in h.layers:
        _check_canonical(n, eu, ev)
    if cfg == 1:
        assert h.m == [4000] * 3
    if cfg == 2:
        assert h.m == [n * 5] * 4
    if cfg == 4:
        assert h.m == [n * 8] * 6
    if cfg == 5:
        degs = h.meta["avg_degrees"]
        assert h.m == [n * d // 2 for d in degs]


def test_determinism():
    a = C.config2(0.02)
    b = C.config2(0.02)
    for (u1, v1), (u2, v2) in zip(a.layers, b.layers):
        assert np.array_equal(u1, u2) and np.array_equal(v1, v2)


def test_shared_base_in_every_layer():
    h = C.config2(0.05)
    n = h.n
    sets = [set((u.astype(np.int64) * n + v).tolist()) for u, v in h.layers]
    common = set.intersection(*sets)
    assert len(common) >= int(0.30 * h.m[0])


def test_chung_lu_is_heavy_tailed():
    h = C.config2(0.1)
    eu, ev = h.layers[0]
    deg = np.bincount(np.concatenate([eu, ev]), minlength=h.n)
    assert deg.max() > 20 * deg.mean()


def test_config3_params_range():
    for hh in range(64):
        nl, n, f, kinds = C.config3_params(hh)
        assert 2 <= nl <= 8 and 2000 <= n <= 50000 and 0.2 <= f <= 0.5
        for j, (k, d) in enumerate(kinds):
            assert (k == "er" and 4 <= d <= 16) if j % 2 == 0 else (k == "ba" and 3 <= d <= 8)


def test_config3_small_homln():
    h = C.config3_homln(0, scale=0.05)
    for eu, ev in h.layers:
        _check_canonical(h.n, eu, ev)


def test_rmat_in_range():
    rng = G.rng_for(9, 0, 0)
    u, v = G.rmat_draw(1000)(rng, 5000)
    assert u.max() < 1000 and v.max() < 1000


def test_config4_sources():
    deg = np.array([0, 1, 2, 0, 5, 1, 0, 3])
    s = C.config4_sources(0, deg, count=3)
    assert len(s) == 3 and np.all(deg[s] > 0) and np.all(np.diff(s) > 0)
