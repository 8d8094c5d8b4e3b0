"""The no-allocation entry point hln_closeness_layer_static (for callers
that cannot allocate device memory), called through the C ABI: its outputs
equal those of hln_closeness_layer with a caller workspace (and the
oracle's), on two calls in a row whose second input is smaller, so the
second call runs on scratch the first one left behind.  A graph that needs
more scratch than the static array is refused before anything runs."""
import ctypes

import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from oracle import oracle as O
from tests.gpu_common import csr_np, graph_dev, say, to_dev

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")

HLN_ENOMEM = 2


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def call_static(g, sources, width, out):
    L = P.lib()
    o = P._lib.hln_opts(width, 0, 0, None, None, 0)
    gc = g.c()
    n_src = g.n if sources is None else int(sources.numel())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.hln_closeness_layer_static(ctypes.byref(gc), _p(sources), n_src, ctypes.byref(o), _p(out["S"]),
                                        _p(out["R"]), _p(out["cc"]), _p(out.get("h2")), stream)


def empty_like(ref):
    return {k: (None if v is None else torch.full_like(v, -7)) for k, v in ref.items()}


CASES = [
    # (tag, graph builder, listed source count or None, width)
    ("cfg2-scaled layer 1, all sources, W=512", lambda: csr_np(*_cfg2_layer()), None, 512),
    ("cfg1 AND graph, 300 listed sources, W=64", lambda: _cfg1_and(), 300, 64),
]


def _cfg2_layer():
    h = C.config2(scale=0.2)
    return (h.n, *h.layers[1])


def _cfg1_and():
    h = C.config1()
    return O.compose("and", [csr_np(h.n, *e) for e in h.layers])


def test_static_scratch_matches_workspace_call_twice():
    rng = np.random.default_rng(77)
    sizes = []
    for tag, build, count, width in CASES:
        rp, ci = build()
        n = len(rp) - 1
        sizes.append(n)
        g = graph_dev(P, rp, ci)
        src = None
        if count is not None:
            src = to_dev(np.sort(rng.choice(n, size=count, replace=False)).astype(np.int32))
        say("static scratch:", tag, "n=%d nnz=%d" % (n, len(ci)))
        ref = P.hln_closeness_layer(g, sources=src, width_bits=width, want_h2=src is None)
        got = empty_like(ref)
        st = call_static(g, src, width, got)
        assert st == 0, P.lib().hln_last_error()
        torch.cuda.synchronize()
        P.device_status()
        for key in ("S", "R", "cc", "h2"):
            if ref[key] is None:
                continue
            assert torch.equal(got[key], ref[key]), (tag, key)
        S, R = O.bfs_sums(rp, ci, sources=None if src is None else src.cpu().numpy())
        assert np.array_equal(got["S"].cpu().numpy(), S), tag
        assert np.array_equal(got["R"].cpu().numpy(), R), tag
        assert np.array_equal(got["cc"].cpu().numpy().view(np.int64), O.closeness_wf(n, S, R).view(np.int64)), tag
    assert sizes[1] < sizes[0]          # the second call is the smaller one


def test_static_scratch_refuses_what_does_not_fit():
    h = C.config2(scale=0.5)
    rp, ci = csr_np(h.n, *h.layers[0])
    g = graph_dev(P, rp, ci)
    out = {"S": torch.empty(h.n, dtype=torch.int64, device="cuda"), "R": torch.empty(h.n, dtype=torch.int32, device="cuda"),
           "cc": None, "h2": None}
    need = P.closeness_workspace_size(h.n, len(ci), h.n, 4096)
    assert need > P._lib.HLN_STATIC_SCRATCH_BYTES
    assert call_static(g, None, 4096, out) == HLN_ENOMEM
    assert b"static" in P.lib().hln_last_error()
    torch.cuda.synchronize()
    P.device_status()
