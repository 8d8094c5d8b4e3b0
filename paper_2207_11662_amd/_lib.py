"""ctypes binding of ``libhln.so`` (the C ABI declared in ``include/hln.h``).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch provides device memory (tensors) and the stream
(``torch.cuda.current_stream()``).  If the library has not been built the
first call raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhln.so")

HLN_OK, HLN_EINVAL, HLN_ENOMEM, HLN_EDEVICE, HLN_EUNSUPPORTED = 0, 1, 2, 3, 4
_STATUS = {0: "HLN_OK", 1: "HLN_EINVAL", 2: "HLN_ENOMEM", 3: "HLN_EDEVICE", 4: "HLN_EUNSUPPORTED"}

# every symbol include/hln.h declares (checked by the tests)
EXPORTS = [
    "hln_last_error", "hln_version", "hln_device_cu_count", "hln_device_status",
    "hln_resident_blocks", "hln_closeness_kernel_residency", "hln_last_launch_path", "hln_plan_launch_paths",
    "hln_closeness_layer_static",
    "hln_csr_from_edges_workspace_size", "hln_csr_from_edges", "hln_csr_from_edges_batch_workspace_size",
    "hln_csr_from_edges_batch", "hln_csr_validate",
    "hln_compose_workspace_size", "hln_compose_and", "hln_compose_or", "hln_compose_and_batch_workspace_size",
    "hln_compose_and_batch",
    "hln_closeness_workspace_size", "hln_closeness_layer", "hln_closeness_estimate",
    "hln_compose_cc_topk_workspace_size", "hln_compose_cc_topk",
    "hln_compose_cc_topk_batch_workspace_size", "hln_compose_cc_topk_batch", "hln_compose_cc1_workspace_size", "hln_compose_cc1",
    "hln_plan_create", "hln_plan_destroy", "hln_plan_width", "hln_plan_set_width", "hln_closeness_batch_workspace_size",
    "hln_closeness_batch", "hln_plan_tune", "hln_plan_capture", "hln_plan_replay", "hln_plan_reserve",
    "hln_mlp_param_count", "hln_proposer_features", "hln_mlp_init", "hln_mlp_forward",
    "hln_mlp_train_workspace_size", "hln_mlp_train_step", "hln_topk_workspace_size", "hln_topk", "hln_rank_labels",
]

HLN_RANK_WF, HLN_RANK_CC2, HLN_RANK_NAIVE = 0, 1, 2
HLN_FLAG_PER_VERTEX = 1
HLN_STATIC_SCRATCH_BYTES = 64 * 1024 * 1024   # scratch of hln_closeness_layer_static (include/hln.h)


class HlnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


class hln_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class hln_edge_list(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("eu", ctypes.c_void_p), ("ev", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class hln_topk_problem(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("n", ctypes.c_int32), ("r", ctypes.c_int32), ("k", ctypes.c_int32),
                ("S", ctypes.c_void_p), ("R", ctypes.c_void_p), ("ids", ctypes.c_void_p), ("score", ctypes.c_void_p),
                ("count", ctypes.c_void_p)]


class hln_and_problem(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("layers", ctypes.c_void_p), ("out_row_ptr", ctypes.c_void_p),
                ("out_col_idx", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class hln_opts(ctypes.Structure):
    _fields_ = [("width_bits", ctypes.c_int32), ("direction", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("levels", ctypes.c_void_p), ("trace", ctypes.c_void_p), ("trace_cap", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhln.so is not built (run `python -m paper_2207_11662_amd.build`); "
                          "there is no non-HIP fallback")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    st = ctypes.c_int
    csr_p, opts_p = ctypes.POINTER(hln_csr), ctypes.POINTER(hln_opts)
    sig = {
        "hln_last_error": ([], ctypes.c_char_p),
        "hln_version": ([], i32),
        "hln_device_cu_count": ([], i32),
        "hln_device_status": ([P], st),
        "hln_resident_blocks": ([i32, i32, i32], i32),
        "hln_closeness_kernel_residency": ([i32, i32, i32, P], st),
        "hln_last_launch_path": ([], i32),
        "hln_plan_launch_paths": ([P, P, P], st),
        "hln_csr_from_edges_workspace_size": ([i32, i64], sz),
        "hln_csr_from_edges": ([i32, i64, P, P, P, P, P, sz, P], st),
        "hln_csr_from_edges_batch_workspace_size": ([ctypes.POINTER(hln_edge_list), i32], sz),
        "hln_csr_from_edges_batch": ([ctypes.POINTER(hln_edge_list), i32, P, sz, P], st),
        "hln_csr_validate": ([csr_p, P, P], st),
        "hln_compose_workspace_size": ([csr_p, i32], sz),
        "hln_compose_and": ([csr_p, i32, P, P, i64, P, sz, P], st),
        "hln_compose_or": ([csr_p, i32, P, P, i64, P, sz, P], st),
        "hln_compose_and_batch_workspace_size": ([ctypes.POINTER(hln_and_problem), i32], sz),
        "hln_compose_and_batch": ([ctypes.POINTER(hln_and_problem), i32, P, sz, P], st),
        "hln_closeness_workspace_size": ([i32, i64, i32, opts_p], sz),
        "hln_closeness_layer": ([csr_p, P, i32, opts_p, P, P, P, P, P, sz, P], st),
        "hln_closeness_layer_static": ([csr_p, P, i32, opts_p, P, P, P, P, P], st),
        "hln_closeness_estimate": ([i32, i32, P, i32, P, P, P, P], st),
        "hln_compose_cc_topk_workspace_size": ([i32], sz),
        "hln_compose_cc_topk": ([i32, i32, i32, P, P, i32, P, P, P, P, sz, P], st),
        "hln_compose_cc_topk_batch_workspace_size": ([ctypes.POINTER(hln_topk_problem), i32], sz),
        "hln_compose_cc_topk_batch": ([ctypes.POINTER(hln_topk_problem), i32, P, sz, P], st),
        "hln_compose_cc1_workspace_size": ([i32, i32], sz),
        "hln_compose_cc1": ([P, i32, P, P, i32, i32, P, P, P, P, sz, P], st),
        "hln_plan_create": ([ctypes.POINTER(ctypes.c_void_p)], st),
        "hln_plan_destroy": ([P], None),
        "hln_plan_width": ([P, i32], i32),
        "hln_plan_set_width": ([P, i32, i32], st),
        "hln_closeness_batch_workspace_size": ([P, csr_p, i32], sz),
        "hln_closeness_batch": ([P, csr_p, i32, P, P, P, P, P, P, P, sz, P], st),
        "hln_plan_tune": ([P, csr_p, i32, P, P, P, sz, P], st),
        "hln_plan_capture": ([P, csr_p, i32, P, P, P, P, P, P, P, sz, P], st),
        "hln_plan_replay": ([P, P], st),
        "hln_plan_reserve": ([P, csr_p, i32], st),
        "hln_mlp_param_count": ([], i32),
        "hln_proposer_features": ([i32, i32, P, P, P, P, P, P, P], st),
        "hln_mlp_init": ([P, P, P, ctypes.c_uint64, P], st),
        "hln_mlp_forward": ([P, P, i32, P, P], st),
        "hln_mlp_train_workspace_size": ([i32], sz),
        "hln_mlp_train_step": ([P, P, P, i32, ctypes.c_float, P, P, i32, P, P, sz, P], st),
        "hln_topk_workspace_size": ([i32], sz),
        "hln_topk": ([i32, P, i32, i32, P, P, sz, P], st),
        "hln_rank_labels": ([i32, P, i32, P, P, sz, P], st),
    }
    for name, (args, res) in sig.items():
        if hasattr(L, name):
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
    _lib = L
    return L


def check(status: int):
    if status != HLN_OK:
        msg = lib().hln_last_error()
        raise HlnError(status, msg.decode() if msg else "")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """Caller-owned scratch; the caching allocator returns 512-byte aligned blocks."""
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")
    if t.data_ptr() % 256:
        raise HlnError(HLN_EINVAL, "workspace tensor is not 256-byte aligned")
    return t


class Graph:
    """A CSR graph in device memory (int32 row_ptr[n+1], col_idx[nnz]).

    nnz is the host-side arc count, or an upper bound on it when the graph
    was produced asynchronously (the kernels read the exact count from
    row_ptr[n])."""

    def __init__(self, row_ptr: torch.Tensor, col_idx: torch.Tensor, nnz: int | None = None):
        assert row_ptr.dtype == torch.int32 and col_idx.dtype == torch.int32
        assert row_ptr.is_cuda and col_idx.is_cuda and row_ptr.is_contiguous() and col_idx.is_contiguous()
        self.row_ptr = row_ptr
        self.col_idx = col_idx
        self.n = row_ptr.numel() - 1
        self.nnz = int(col_idx.numel() if nnz is None else nnz)

    def c(self) -> hln_csr:
        return hln_csr(self.n, self.nnz, self.row_ptr.data_ptr(),
                       self.col_idx.data_ptr() if self.col_idx.numel() else None)

    def exact_nnz(self) -> int:
        """Arc count from row_ptr[n] (synchronises)."""
        return int(self.row_ptr[self.n].item())

    def trimmed(self) -> "Graph":
        """The same graph with col_idx cut to the exact arc count (synchronises)."""
        m = self.exact_nnz()
        return Graph(self.row_ptr, self.col_idx[:m], m)


def device_status(stream=None):
    check(lib().hln_device_status(_stream(stream)))


# ---------------------------------------------------------------------------
# a3-a6: exact closeness of one graph
# ---------------------------------------------------------------------------

def closeness_workspace_size(n: int, nnz: int, n_src: int, width_bits: int = 512, direction: int = 0) -> int:
    o = hln_opts(width_bits, direction, 0, None)
    return int(lib().hln_closeness_workspace_size(n, nnz, n_src, ctypes.byref(o)))


def hln_closeness_layer(g: Graph, sources: torch.Tensor | None = None, width_bits: int = 512,
                        direction: int = 0, want_cc: bool = True, want_h2: bool = False,
                        out=None, ws: torch.Tensor | None = None, stream=None, levels: torch.Tensor | None = None,
                        trace: torch.Tensor | None = None, per_vertex: bool = False):
    """Returns dict(S int64, R int32, cc float64 | None, h2 int32 | None).
    `levels` (int32, ceil(n_src / width_bits) entries) receives the BFS levels
    run per source batch; `trace` (int64 [levels, 4], zero-filled) the
    per-level trace described in include/hln.h.  `per_vertex` (listed
    sources only, no cc): S and R per vertex, summed over the sources
    (HLN_FLAG_PER_VERTEX)."""
    dev = g.row_ptr.device
    n_src = g.n if sources is None else int(sources.numel())
    if sources is not None:
        assert sources.dtype == torch.int32 and sources.is_cuda and sources.is_contiguous()
    n_out = g.n if per_vertex else n_src
    if per_vertex:
        want_cc = False
    if out is None:
        out = {"S": torch.empty(max(n_out, 1), dtype=torch.int64, device=dev),
               "R": torch.empty(max(n_out, 1), dtype=torch.int32, device=dev),
               "cc": torch.empty(max(n_out, 1), dtype=torch.float64, device=dev) if want_cc else None,
               "h2": torch.empty(max(n_out, 1), dtype=torch.int32, device=dev) if want_h2 else None}
    o = hln_opts(width_bits, direction, HLN_FLAG_PER_VERTEX if per_vertex else 0,
                 None if levels is None else levels.data_ptr(),
                 None if trace is None else trace.data_ptr(), 0 if trace is None else trace.shape[0])
    need = int(lib().hln_closeness_workspace_size(g.n, g.nnz, n_src, ctypes.byref(o)))
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    gc = g.c()
    check(lib().hln_closeness_layer(ctypes.byref(gc), _ptr(sources), n_src, ctypes.byref(o),
                                    _ptr(out["S"]), _ptr(out["R"]), _ptr(out["cc"]), _ptr(out["h2"]),
                                    _ptr(ws), ws.numel(), _stream(stream)))
    return {k: (v[:n_out] if v is not None else None) for k, v in out.items()}


def hln_closeness_estimate(n: int, n_pop: int, sources: torch.Tensor, S: torch.Tensor, R: torch.Tensor,
                           cc: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Sampling estimate of every vertex's closeness from per-vertex sample
    sums (hln_closeness_layer(..., per_vertex=True) over `sources`)."""
    assert sources.dtype == torch.int32 and sources.is_contiguous()
    assert S.dtype == torch.int64 and R.dtype == torch.int32 and S.numel() >= n and R.numel() >= n
    if cc is None:
        cc = torch.empty(max(n, 1), dtype=torch.float64, device=S.device)
    assert cc.dtype == torch.float64 and cc.numel() >= n
    check(lib().hln_closeness_estimate(n, n_pop, _ptr(sources), int(sources.numel()), _ptr(S), _ptr(R), _ptr(cc),
                                       _stream(stream)))
    return cc[:n]


# ---------------------------------------------------------------------------
# a1: ingest, validation
# ---------------------------------------------------------------------------

def hln_csr_from_edges(n: int, eu: torch.Tensor, ev: torch.Tensor, ws: torch.Tensor | None = None,
                       out=None, stream=None) -> Graph:
    """Normalised symmetric CSR of an arbitrary edge list (device tensors).
    The returned Graph's col_idx has room for 2*m arcs; nnz is that bound."""
    assert eu.dtype == torch.int32 and ev.dtype == torch.int32 and eu.numel() == ev.numel()
    dev = eu.device
    m = int(eu.numel())
    if out is None:
        out = (torch.empty(n + 1, dtype=torch.int32, device=dev), torch.empty(max(2 * m, 1), dtype=torch.int32, device=dev))
    need = int(lib().hln_csr_from_edges_workspace_size(n, m))
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    check(lib().hln_csr_from_edges(n, m, _ptr(eu), _ptr(ev), _ptr(out[0]), _ptr(out[1]), _ptr(ws), ws.numel(),
                                   _stream(stream)))
    return Graph(out[0], out[1][:max(2 * m, 0)] if m else out[1][:0], 2 * m)


def _edge_lists(items, outs):
    arr = (hln_edge_list * max(len(items), 1))()
    for i, ((n, eu, ev), (rp, ci)) in enumerate(zip(items, outs)):
        assert eu.dtype == torch.int32 and ev.dtype == torch.int32 and eu.numel() == ev.numel()
        assert rp.numel() >= n + 1 and ci.numel() >= 2 * eu.numel()
        arr[i] = hln_edge_list(n, int(eu.numel()), _ptr(eu), _ptr(ev), _ptr(rp), _ptr(ci))
    return arr


def csr_from_edges_batch_workspace_size(items) -> int:
    """Workspace bytes of hln_csr_from_edges_batch for (n, eu, ev) lists."""
    arr = (hln_edge_list * max(len(items), 1))()
    for i, (n, eu, _) in enumerate(items):
        arr[i] = hln_edge_list(n, int(eu.numel()), None, None, None, None)
    return int(lib().hln_csr_from_edges_batch_workspace_size(arr, len(items)))


def hln_csr_from_edges_batch(items, ws: torch.Tensor | None = None, outs=None, stream=None) -> list:
    """hln_csr_from_edges of many edge lists in one set of launches.  items:
    (n, eu, ev) per list (int32 device tensors); outs: optional (row_ptr,
    col_idx) per list.  Returns one Graph per list (nnz = the 2*m bound)."""
    if not items:
        return []
    dev = items[0][1].device
    if outs is None:
        outs = [(torch.empty(n + 1, dtype=torch.int32, device=dev), torch.empty(max(2 * eu.numel(), 1), dtype=torch.int32,
                                                                               device=dev)) for n, eu, _ in items]
    arr = _edge_lists(items, outs)
    need = int(lib().hln_csr_from_edges_batch_workspace_size(arr, len(items)))
    if need == 0:           # invalid sizes: the call itself reports them
        check(lib().hln_csr_from_edges_batch(arr, len(items), None, 0, _stream(stream)))
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    check(lib().hln_csr_from_edges_batch(arr, len(items), _ptr(ws), ws.numel(), _stream(stream)))
    res = []
    for (n, eu, _), (rp, ci) in zip(items, outs):
        m = int(eu.numel())
        res.append(Graph(rp, ci[:2 * m] if m else ci[:0], 2 * m))
    return res


def hln_csr_validate(g: Graph, stream=None) -> int:
    """Bit mask of CSR convention violations (0 = valid); synchronises."""
    res = torch.zeros(1, dtype=torch.int32, device=g.row_ptr.device)
    gc = g.c()
    check(lib().hln_csr_validate(ctypes.byref(gc), _ptr(res), _stream(stream)))
    return int(res.item())


# ---------------------------------------------------------------------------
# a2: Boolean aggregation
# ---------------------------------------------------------------------------

def _layers_c(layers):
    arr = (hln_csr * len(layers))(*[g.c() for g in layers])
    return arr


def compose_workspace_size(layers) -> int:
    arr = _layers_c(layers)
    return int(lib().hln_compose_workspace_size(arr, len(layers)))


def _compose(fn, layers, capacity, ws, out, stream):
    dev = layers[0].row_ptr.device
    n = layers[0].n
    arr = _layers_c(layers)
    need = int(lib().hln_compose_workspace_size(arr, len(layers)))
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    if out is None:
        out = (torch.empty(n + 1, dtype=torch.int32, device=dev), torch.empty(max(capacity, 1), dtype=torch.int32, device=dev))
    check(fn(arr, len(layers), _ptr(out[0]), _ptr(out[1]), capacity, _ptr(ws), ws.numel(), _stream(stream)))
    return Graph(out[0], out[1][:capacity], capacity)


def hln_compose_and(layers, ws=None, out=None, stream=None) -> Graph:
    """Edges present in every layer; col_idx sized by the smallest layer."""
    return _compose(lib().hln_compose_and, layers, min(g.nnz for g in layers), ws, out, stream)


def hln_compose_or(layers, ws=None, out=None, stream=None) -> Graph:
    """Edges present in at least one layer; col_idx sized by the sum."""
    return _compose(lib().hln_compose_or, layers, sum(g.nnz for g in layers), ws, out, stream)


class AndBatch:
    """hln_compose_and of many layer sets in one call.  problems: a list of
    layer lists (Graphs of equal n within a list); outs: optional
    (row_ptr, col_idx) per problem, col_idx sized by its smallest layer.
    The host-side table is built once and kept, so run() can be repeated
    or captured; it returns one Graph per problem (nnz = the capacity)."""

    def __init__(self, problems, outs=None, ws=None):
        self.problems = [list(p) for p in problems]
        dev = self.problems[0][0].row_ptr.device if self.problems else torch.device("cuda")
        caps = [min(g.nnz for g in p) for p in self.problems]
        if outs is None:
            outs = [(torch.empty(p[0].n + 1, dtype=torch.int32, device=dev),
                     torch.empty(max(c, 1), dtype=torch.int32, device=dev)) for p, c in zip(self.problems, caps)]
        self.outs, self.caps = outs, caps
        self._keep = [_layers_c(p) for p in self.problems]
        self.arr = (hln_and_problem * max(len(self.problems), 1))()
        for i, (lay, (rp, ci), c) in enumerate(zip(self._keep, outs, caps)):
            self.arr[i] = hln_and_problem(len(self.problems[i]), ctypes.cast(lay, ctypes.c_void_p), _ptr(rp), _ptr(ci), c)
        self.need = int(lib().hln_compose_and_batch_workspace_size(self.arr, len(self.problems)))
        if ws is None or ws.numel() < self.need:
            ws = workspace(self.need, dev) if self.need else None
        self.ws = ws

    def run(self, stream=None):
        wsp, wsn = (None, 0) if self.ws is None else (_ptr(self.ws), self.ws.numel())
        check(lib().hln_compose_and_batch(self.arr, len(self.problems), wsp, wsn, _stream(stream)))
        return [Graph(rp, ci[:c], c) for (rp, ci), c in zip(self.outs, self.caps)]


def hln_compose_and_batch(problems, ws=None, outs=None, stream=None) -> list:
    """AND aggregates of many layer sets in one call (see AndBatch)."""
    if not problems:
        return []
    return AndBatch(problems, outs=outs, ws=ws).run(stream)


# ---------------------------------------------------------------------------
# a7: selection / composition
# ---------------------------------------------------------------------------

def hln_compose_cc_topk(mode: int, n: int, S_list, R_list, k: int, ws=None, out=None, stream=None):
    """Returns (ids, score, count) device tensors; count is a 1-element int32."""
    dev = S_list[0].device
    r = len(S_list)
    Sp = (ctypes.c_void_p * r)(*[t.data_ptr() for t in S_list])
    Rp = (ctypes.c_void_p * r)(*[t.data_ptr() for t in R_list])
    need = int(lib().hln_compose_cc_topk_workspace_size(n))
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    if out is None:
        size = n if k < 0 else max(k, 1)
        out = (torch.empty(max(size, 1), dtype=torch.int32, device=dev),
               torch.empty(max(size, 1), dtype=torch.float64, device=dev),
               torch.empty(1, dtype=torch.int32, device=dev))
    check(lib().hln_compose_cc_topk(mode, n, r, ctypes.cast(Sp, ctypes.c_void_p), ctypes.cast(Rp, ctypes.c_void_p),
                                    k, _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return out


class TopkBatch:
    """The k >= 0 top-k of many problems in one call
    (hln_compose_cc_topk_batch).  problems: (mode, n, S_list, R_list, k)
    each; outs: optional (ids, score, count) per problem.  The host-side
    problem table is built once and kept (so the call can be repeated or
    captured); run() enqueues the batch and returns the outs."""

    def __init__(self, problems, outs=None, ws=None):
        self.problems = list(problems)
        dev = self.problems[0][2][0].device if self.problems else torch.device("cuda")
        if outs is None:
            outs = [(torch.empty(max(k, 1), dtype=torch.int32, device=dev),
                     torch.empty(max(k, 1), dtype=torch.float64, device=dev),
                     torch.empty(1, dtype=torch.int32, device=dev)) for _, _, _, _, k in self.problems]
        self.outs = outs
        self._keep = []
        self.arr = (hln_topk_problem * max(len(self.problems), 1))()
        for i, ((mode, n, S_list, R_list, k), (ids, sc, cnt)) in enumerate(zip(self.problems, outs)):
            Sp = (ctypes.c_void_p * len(S_list))(*[t.data_ptr() for t in S_list])
            Rp = (ctypes.c_void_p * len(R_list))(*[t.data_ptr() for t in R_list])
            self._keep += [Sp, Rp]
            self.arr[i] = hln_topk_problem(mode, n, len(S_list), k, ctypes.cast(Sp, ctypes.c_void_p),
                                           ctypes.cast(Rp, ctypes.c_void_p), _ptr(ids),
                                           None if sc is None else _ptr(sc), _ptr(cnt))
        self.need = int(lib().hln_compose_cc_topk_batch_workspace_size(self.arr, len(self.problems)))
        if ws is None or ws.numel() < self.need:
            ws = workspace(self.need, dev) if self.need else None
        self.ws = ws

    def run(self, stream=None):
        wsp, wsn = (None, 0) if self.ws is None else (_ptr(self.ws), self.ws.numel())
        check(lib().hln_compose_cc_topk_batch(self.arr, len(self.problems), wsp, wsn, _stream(stream)))
        return self.outs


def hln_compose_cc_topk_batch(problems, ws=None, outs=None, stream=None):
    """Top-k of many problems, (mode, n, S_list, R_list, k) each; returns one
    (ids, score, count) per problem."""
    if not problems:
        return []
    return TopkBatch(problems, outs=outs, ws=ws).run(stream)


def hln_compose_cc1(layers, S_list, R_list, tau=(1, 2), ws=None, out=None, stream=None):
    """CC1 nodes of the layers' AND aggregate (Sec. 5.1, readings in
    include/hln.h).  Returns (ids, count, avg) device tensors: ids ascending
    (the first count entries), count a 1-element int32, avg Eq. 3's value."""
    r = len(layers)
    n = layers[0].n
    dev = layers[0].row_ptr.device
    arr = (hln_csr * r)(*[g.c() for g in layers])
    Sp = (ctypes.c_void_p * r)(*[t.data_ptr() for t in S_list])
    Rp = (ctypes.c_void_p * r)(*[t.data_ptr() for t in R_list])
    need = int(lib().hln_compose_cc1_workspace_size(n, r))
    if need == 0:
        raise HlnError(1, "hln_compose_cc1_workspace_size: bad arguments (n=%d, r=%d)" % (n, r))
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    if out is None:
        out = (torch.empty(max(n, 1), dtype=torch.int32, device=dev), torch.empty(1, dtype=torch.int32, device=dev),
               torch.empty(1, dtype=torch.float64, device=dev))
    check(lib().hln_compose_cc1(ctypes.cast(arr, ctypes.c_void_p), r, ctypes.cast(Sp, ctypes.c_void_p),
                                ctypes.cast(Rp, ctypes.c_void_p), int(tau[0]), int(tau[1]), _ptr(out[0]), _ptr(out[1]),
                                _ptr(out[2]), _ptr(ws), ws.numel(), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# a8: batched closeness (persistent LDS tiles, hipGraph capture, autotuner)
# ---------------------------------------------------------------------------

def _ptr_array(tensors):
    if tensors is None:
        return None
    arr = (ctypes.c_void_p * len(tensors))(*[None if t is None else t.data_ptr() for t in tensors])
    return ctypes.cast(arr, ctypes.c_void_p)


class Plan:
    """Owner of an hln_plan (tuned widths, staging, captured graph)."""

    def __init__(self):
        h = ctypes.c_void_p()
        check(lib().hln_plan_create(ctypes.byref(h)))
        self.h = h
        self._keep = None

    def close(self):
        if self.h:
            lib().hln_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def width(self, n: int) -> int:
        return int(lib().hln_plan_width(self.h, n))

    def set_width(self, n: int, width: int):
        """Set the width of n's log2(n) class (0: the untuned default)."""
        check(lib().hln_plan_set_width(self.h, n, width))

    def _args(self, graphs, outs):
        arr = _layers_c(graphs)
        S = _ptr_array([o["S"] for o in outs])
        R = _ptr_array([o["R"] for o in outs])
        cc = _ptr_array([o.get("cc") for o in outs])
        h2 = _ptr_array([o.get("h2") for o in outs]) if any(o.get("h2") is not None for o in outs) else None
        return arr, S, R, cc, h2

    @staticmethod
    def _sources(graphs, sources):
        """(pointer array, n_src array) for per-graph listed sources (None
        entries: all of that graph's vertices), or (None, None)."""
        if sources is None or all(s is None for s in sources):
            return None, None
        assert len(sources) == len(graphs)
        for s in sources:
            if s is not None:
                assert s.dtype == torch.int32 and s.is_cuda and s.is_contiguous()
        ptrs = _ptr_array(sources)
        # -1: all of the graph's vertices; an empty list (whose data pointer
        # may be NULL) is 0 listed sources
        counts = (ctypes.c_int32 * len(graphs))(*[-1 if s is None else int(s.numel()) for s in sources])
        return ptrs, counts

    @staticmethod
    def outputs_listed(graphs, sources):
        """Outputs of a call with listed sources: per listed graph S, R, cc
        indexed by list position; per all-source graph as outputs()."""
        out = []
        for g, s in zip(graphs, sources):
            k = g.n if s is None else int(s.numel())
            dev = g.row_ptr.device
            out.append({"S": torch.empty(max(k, 1), dtype=torch.int64, device=dev),
                        "R": torch.empty(max(k, 1), dtype=torch.int32, device=dev),
                        "cc": torch.empty(max(k, 1), dtype=torch.float64, device=dev), "h2": None})
        return out

    def workspace_size(self, graphs) -> int:
        arr = _layers_c(graphs)
        return int(lib().hln_closeness_batch_workspace_size(self.h, arr, len(graphs)))

    @staticmethod
    def outputs(graphs, want_h2=False):
        out = []
        for g in graphs:
            dev = g.row_ptr.device
            out.append({"S": torch.empty(g.n, dtype=torch.int64, device=dev),
                        "R": torch.empty(g.n, dtype=torch.int32, device=dev),
                        "cc": torch.empty(g.n, dtype=torch.float64, device=dev),
                        "h2": torch.empty(g.n, dtype=torch.int32, device=dev) if want_h2 else None})
        return out

    def run(self, graphs, outs, ws=None, stream=None, sources=None):
        """hln_closeness_batch; sources: None, or one int32 device tensor of
        listed source ids (or None for all vertices) per graph."""
        arr, S, R, cc, h2 = self._args(graphs, outs)
        src, cnt = self._sources(graphs, sources)
        need = self.workspace_size(graphs)
        if ws is None or ws.numel() < need:
            ws = workspace(need, graphs[0].row_ptr.device)
        check(lib().hln_closeness_batch(self.h, arr, len(graphs), src, cnt, S, R, cc, h2, _ptr(ws), ws.numel(),
                                        _stream(stream)))
        return ws

    def tune(self, graphs, outs, ws=None, stream=None):
        arr, S, R, _, _ = self._args(graphs, outs)
        need = self.workspace_size(graphs)
        if ws is None or ws.numel() < need:
            ws = workspace(need, graphs[0].row_ptr.device)
        check(lib().hln_plan_tune(self.h, arr, len(graphs), S, R, _ptr(ws), ws.numel(), _stream(stream)))

    def capture(self, graphs, outs, ws, stream, sources=None):
        arr, S, R, cc, h2 = self._args(graphs, outs)
        src, cnt = self._sources(graphs, sources)
        self._keep = (graphs, outs, ws, sources)       # captured buffers must outlive replays
        check(lib().hln_plan_capture(self.h, arr, len(graphs), src, cnt, S, R, cc, h2, _ptr(ws), ws.numel(),
                                     _stream(stream)))

    def reserve(self, graphs):
        """Staging for a capture made by the caller (e.g. torch.cuda.graph)."""
        arr = _layers_c(graphs)
        check(lib().hln_plan_reserve(self.h, arr, len(graphs)))

    def replay(self, stream=None):
        check(lib().hln_plan_replay(self.h, _stream(stream)))

    def launch_paths(self):
        """(cooperative, ordinary-in-capture) persistent launches of the
        plan's last enqueue."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(lib().hln_plan_launch_paths(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


def closeness_kernel_residency(width_bits: int, block: int, mode: int) -> dict:
    """Registers, LDS, scratch, the runtime's occupancy answer and the
    co-residency bound of one persistent closeness kernel (needs a GPU)."""
    info = (ctypes.c_int32 * 5)()
    check(lib().hln_closeness_kernel_residency(width_bits, block, mode, info))
    return dict(zip(("vgprs", "lds", "scratch", "query", "bound"), list(info)))


def last_launch_path() -> int:
    return int(lib().hln_last_launch_path())


# ---------------------------------------------------------------------------
# a9: learned candidate proposer (features, FP32 MLP, generic top-k)
# ---------------------------------------------------------------------------

def mlp_param_count() -> int:
    return int(lib().hln_mlp_param_count())


def hln_proposer_features(graphs, S_list, R_list, h2s, X=None, stream=None) -> torch.Tensor:
    """12 features per vertex from r layers' CSR and all-source S, R, h2.
    Each Graph's nnz must be its exact arc count (it sets the mean degree)."""
    n = graphs[0].n
    r = len(graphs)
    if X is None:
        X = torch.empty((n, 12), dtype=torch.float32, device=graphs[0].row_ptr.device)
    nnz = (ctypes.c_int64 * r)(*[g.nnz for g in graphs])
    check(lib().hln_proposer_features(n, r, _ptr_array([g.row_ptr for g in graphs]), _ptr_array(S_list),
                                      _ptr_array(R_list), _ptr_array(h2s), ctypes.cast(nnz, ctypes.c_void_p),
                                      _ptr(X), _stream(stream)))
    return X


def hln_mlp_init(params, m=None, v=None, seed: int = 0, stream=None):
    check(lib().hln_mlp_init(_ptr(params), _ptr(m), _ptr(v), seed, _stream(stream)))


def hln_mlp_forward(params, X, y=None, stream=None):
    if y is None:
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    check(lib().hln_mlp_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(y), _stream(stream)))
    return y


def hln_mlp_train_step(params, m, v, step: int, lr: float, X, target, loss=None, ws=None, stream=None):
    n = X.shape[0]
    need = int(lib().hln_mlp_train_workspace_size(n))
    if ws is None or ws.numel() < need:
        ws = workspace(need, X.device)
    check(lib().hln_mlp_train_step(_ptr(params), _ptr(m), _ptr(v), step, lr, _ptr(X), _ptr(target), n, _ptr(loss),
                                   _ptr(ws), ws.numel(), _stream(stream)))
    return ws


HLN_TOPK_SET = 0x100


def hln_topk(score: torch.Tensor, k: int, ids=None, ws=None, stream=None, as_set: bool = False) -> torch.Tensor:
    """Indices of the k largest scores (float64 or float32), descending,
    ties by ascending index; with `as_set` the same indices ascending."""
    n = score.numel()
    dtype = (0 if score.dtype == torch.float64 else 1) | (HLN_TOPK_SET if as_set else 0)
    assert score.dtype in (torch.float64, torch.float32)
    need = int(lib().hln_topk_workspace_size(n))
    if ws is None or ws.numel() < need:
        ws = workspace(need, score.device)
    if ids is None:
        ids = torch.empty(max(k, 1), dtype=torch.int32, device=score.device)
    check(lib().hln_topk(n, _ptr(score), dtype, k, _ptr(ids), _ptr(ws), ws.numel(), _stream(stream)))
    return ids[:k]


def hln_rank_labels(score: torch.Tensor, label=None, ws=None, stream=None) -> torch.Tensor:
    """Log-rank labels: log((n+1)/(g+1)) / log(n+1), g = count of strictly
    larger scores."""
    n = score.numel()
    dtype = 0 if score.dtype == torch.float64 else 1
    need = int(lib().hln_topk_workspace_size(n))
    if ws is None or ws.numel() < need:
        ws = workspace(need, score.device)
    if label is None:
        label = torch.empty(n, dtype=torch.float32, device=score.device)
    check(lib().hln_rank_labels(n, _ptr(score), dtype, _ptr(label), _ptr(ws), ws.numel(), _stream(stream)))
    return label
