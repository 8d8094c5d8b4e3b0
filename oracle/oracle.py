"""Python face of the CPU oracle (``hln_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``.  The product package never imports it,
and it never imports the product package.  It shares no code with the HIP
path; the only thing both sides receive is the seeded input from
``homln_inputs``.

Every function wraps one plain C routine (see the C file for the passage of
the paper each one follows) and works on numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hln_oracle.c")
_LIB = os.path.join(_HERE, "libhln_oracle.so")

_CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-pthread", "-Wall", "-Wextra"]

_default = None


def build(force: bool = False, out: str | None = None, defines=()) -> str:
    """Compile the oracle with gcc into ``oracle/libhln_oracle.so`` (or
    ``out``).  ``defines`` are extra -D flags; the tests use them to plant
    known mistakes in a separate copy and check that the pins catch them."""
    target = out or _LIB
    if force or out or not os.path.exists(target) or os.path.getmtime(target) < os.path.getmtime(_SRC):
        tmp = target + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, *["-D" + d for d in defines], "-o", tmp, _SRC])
        os.replace(tmp, target)
    return target


def _bind(path: str):
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.oracle_csr_from_edges.argtypes = [i32, i64, P, P, P, P]
    L.oracle_csr_from_edges.restype = i64
    L.oracle_bfs_sums.argtypes = [i32, P, P, i32, P, P, P, P, P, P, i32]
    L.oracle_bfs_sums.restype = ctypes.c_int
    L.oracle_closeness_wf.argtypes = [i32, i32, P, P, P]
    L.oracle_closeness_wf.restype = None
    L.oracle_penalised.argtypes = [i32, i32, P, P, P]
    L.oracle_penalised.restype = None
    L.oracle_compose.argtypes = [i32, i32, i32, P, P, P, P, i64]
    L.oracle_compose.restype = i64
    L.oracle_mean_fixed_shape.argtypes = [i32, P]
    L.oracle_mean_fixed_shape.restype = ctypes.c_double
    L.oracle_above_mean.argtypes = [i32, P, P]
    L.oracle_above_mean.restype = i32
    L.oracle_topk_desc.argtypes = [i32, P, i32, P]
    L.oracle_topk_desc.restype = i32
    L.oracle_topk_asc_i64.argtypes = [i32, P, i32, P]
    L.oracle_topk_asc_i64.restype = i32
    L.oracle_cc2_est.argtypes = [i32, i32, P, P, P]
    L.oracle_cc2_est.restype = None
    L.oracle_cc2_score.argtypes = [i32, P, P]
    L.oracle_cc2_score.restype = None
    L.oracle_naive.argtypes = [i32, i32, P, P]
    L.oracle_naive.restype = i32
    L.oracle_naive_topk.argtypes = [i32, i32, P, i32, P]
    L.oracle_naive_topk.restype = i32
    L.oracle_sample_sums.argtypes = [i32, P, P, i32, P, P, P]
    L.oracle_sample_sums.restype = ctypes.c_int
    L.oracle_sample_sums_at.argtypes = [i32, P, P, P, i32, P, P, P]
    L.oracle_sample_sums_at.restype = ctypes.c_int
    L.oracle_sample_estimate.argtypes = [i32, i32, i32, P, P, P, P]
    L.oracle_sample_estimate.restype = None
    L.oracle_cc1.argtypes = [i32, i32, P, P, P, P, i32, i32, P, P]
    L.oracle_cc1.restype = i32
    return L


def _load():
    global _default
    if _default is None:
        _default = _bind(build())
    return _default


class Variant:
    """The oracle's functions bound to another build of the same source
    (used only to plant mistakes in tests).  Attribute access returns the
    module-level function running against that library."""

    def __init__(self, path: str):
        self._L = _bind(path)

    def __getattr__(self, name):
        fn = globals()[name]

        def call(*a, **k):
            global _default
            saved = _load()
            _default = self._L
            try:
                return fn(*a, **k)
            finally:
                _default = saved
        return call


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def threads_default() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# --------------------------------------------------------------------------
# graphs
# --------------------------------------------------------------------------

def csr_from_edges(n: int, eu, ev):
    """Normalised symmetric CSR (rows sorted, no self-loops, no duplicates)."""
    L = _load()
    eu = _c(eu, np.int32)
    ev = _c(ev, np.int32)
    m = len(eu)
    row_ptr = np.zeros(n + 1, np.int32)
    col_idx = np.zeros(max(2 * m, 1), np.int32)
    nnz = L.oracle_csr_from_edges(n, m, _p(eu), _p(ev), _p(row_ptr), _p(col_idx))
    if nnz < 0:
        raise ValueError("oracle_csr_from_edges failed (%d)" % nnz)
    return row_ptr, col_idx[:nnz].copy()


def bfs_sums(row_ptr, col_idx, sources=None, nthreads: int | None = None, extras: bool = False):
    """One plain BFS per source.  Returns (S int64, R int32[, H2, ecc, comp_edges])."""
    L = _load()
    row_ptr = _c(row_ptr, np.int32)
    col_idx = _c(col_idx, np.int32) if len(col_idx) else np.zeros(1, np.int32)
    n = len(row_ptr) - 1
    if sources is None:
        src = None
        k = n
    else:
        src = _c(sources, np.int32)
        k = len(src)
    S = np.zeros(max(k, 1), np.int64)
    R = np.zeros(max(k, 1), np.int32)
    H2 = np.zeros(max(k, 1), np.int32)
    ecc = np.zeros(max(k, 1), np.int32)
    ce = np.zeros(max(k, 1), np.int64)
    rc = L.oracle_bfs_sums(n, _p(row_ptr), _p(col_idx), k, None if src is None else _p(src),
                           _p(S), _p(R), _p(H2), _p(ecc), _p(ce),
                           nthreads or threads_default())
    if rc != 0:
        raise ValueError("oracle_bfs_sums failed (%d)" % rc)
    if extras:
        return S[:k], R[:k], H2[:k], ecc[:k], ce[:k]
    return S[:k], R[:k]


def closeness_wf(n: int, S, R):
    L = _load()
    S = _c(S, np.int64)
    R = _c(R, np.int32)
    cc = np.zeros(max(len(S), 1), np.float64)
    L.oracle_closeness_wf(n, len(S), _p(S), _p(R), _p(cc))
    return cc[:len(S)]


def penalised(n: int, S, R):
    L = _load()
    S = _c(S, np.int64)
    R = _c(R, np.int32)
    P = np.zeros(max(len(S), 1), np.int64)
    L.oracle_penalised(n, len(S), _p(S), _p(R), _p(P))
    return P[:len(S)]


def compose(mode: str, layers):
    """AND / OR aggregation.  layers: list of (row_ptr, col_idx)."""
    L = _load()
    r = len(layers)
    n = len(layers[0][0]) - 1
    rps = [_c(a, np.int32) for a, _ in layers]
    cis = [_c(b, np.int32) if len(b) else np.zeros(1, np.int32) for _, b in layers]
    rp_arr = (ctypes.c_void_p * r)(*[a.ctypes.data for a in rps])
    ci_arr = (ctypes.c_void_p * r)(*[b.ctypes.data for b in cis])
    cap = int(sum(int(a[-1]) for a in rps))
    out_rp = np.zeros(n + 1, np.int32)
    out_ci = np.zeros(max(cap, 1), np.int32)
    nnz = L.oracle_compose(0 if mode == "and" else 1, n, r,
                           ctypes.cast(rp_arr, ctypes.c_void_p), ctypes.cast(ci_arr, ctypes.c_void_p),
                           _p(out_rp), _p(out_ci), cap)
    if nnz < 0:
        raise ValueError("oracle_compose failed (%d)" % nnz)
    return out_rp, out_ci[:nnz].copy()


def mean_fixed_shape(x) -> float:
    L = _load()
    x = _c(x, np.float64)
    return float(L.oracle_mean_fixed_shape(len(x), _p(x)))


def above_mean(x):
    L = _load()
    x = _c(x, np.float64)
    ids = np.zeros(max(len(x), 1), np.int32)
    c = L.oracle_above_mean(len(x), _p(x), _p(ids))
    return ids[:c].copy()


def topk_desc(score, k: int):
    L = _load()
    score = _c(score, np.float64)
    ids = np.zeros(max(k, 1), np.int32)
    c = L.oracle_topk_desc(len(score), _p(score), k, _p(ids))
    if c < 0:
        raise ValueError("oracle_topk_desc failed")
    return ids[:c].copy()


def topk_asc_i64(key, k: int):
    L = _load()
    key = _c(key, np.int64)
    ids = np.zeros(max(k, 1), np.int32)
    c = L.oracle_topk_asc_i64(len(key), _p(key), k, _p(ids))
    if c < 0:
        raise ValueError("oracle_topk_asc_i64 failed")
    return ids[:c].copy()


def cc2_est(n: int, S_list, R_list):
    L = _load()
    r = len(S_list)
    Ss = [_c(s, np.int64) for s in S_list]
    Rs = [_c(x, np.int32) for x in R_list]
    s_arr = (ctypes.c_void_p * r)(*[a.ctypes.data for a in Ss])
    r_arr = (ctypes.c_void_p * r)(*[a.ctypes.data for a in Rs])
    est = np.zeros(max(n, 1), np.int64)
    L.oracle_cc2_est(n, r, ctypes.cast(s_arr, ctypes.c_void_p), ctypes.cast(r_arr, ctypes.c_void_p),
                     _p(est))
    return est[:n]


def cc2_score(n: int, est):
    L = _load()
    est = _c(est, np.int64)
    sc = np.zeros(max(n, 1), np.float64)
    L.oracle_cc2_score(n, _p(est), _p(sc))
    return sc[:n]


def naive(n: int, cc_list):
    L = _load()
    r = len(cc_list)
    ccs = [_c(c, np.float64) for c in cc_list]
    arr = (ctypes.c_void_p * r)(*[a.ctypes.data for a in ccs])
    ids = np.zeros(max(n, 1), np.int32)
    c = L.oracle_naive(n, r, ctypes.cast(arr, ctypes.c_void_p), _p(ids))
    if c < 0:
        raise ValueError("oracle_naive failed")
    return ids[:c].copy()


def naive_topk(n: int, cc_list, k: int):
    """Intersection of the layers' top-k sets (ids ascending)."""
    L = _load()
    r = len(cc_list)
    ccs = [_c(c, np.float64) for c in cc_list]
    arr = (ctypes.c_void_p * r)(*[a.ctypes.data for a in ccs])
    ids = np.zeros(max(n, 1), np.int32)
    c = L.oracle_naive_topk(n, r, ctypes.cast(arr, ctypes.c_void_p), k, _p(ids))
    if c < 0:
        raise ValueError("oracle_naive_topk failed")
    return ids[:c].copy()


def cc1(n: int, layers, S_list, R_list, tau=(1, 2), with_avg: bool = False):
    """CC1 nodes (ids ascending) of the layers' AND graph from the layers'
    CSR (row_ptr, col_idx) and all-source S, R; tau = (num, den) is the
    overlap threshold.  With `with_avg`, also Eq. 3's average."""
    L = _load()
    r = len(layers)
    rps = [_c(rp, np.int32) for rp, _ in layers]
    cis = [_c(ci, np.int32) if len(ci) else np.zeros(1, np.int32) for _, ci in layers]
    Ss = [_c(S, np.int64) for S in S_list]
    Rs = [_c(R, np.int32) for R in R_list]
    arr = lambda xs: ctypes.cast((ctypes.c_void_p * r)(*[a.ctypes.data for a in xs]), ctypes.c_void_p)  # noqa: E731
    ids = np.zeros(max(n, 1), np.int32)
    avg = np.zeros(1, np.float64)
    c = L.oracle_cc1(n, r, arr(rps), arr(cis), arr(Ss), arr(Rs), int(tau[0]), int(tau[1]), _p(ids), _p(avg))
    if c < 0:
        raise ValueError("oracle_cc1 failed (%d)" % c)
    out = ids[:c].copy()
    return (out, float(avg[0])) if with_avg else out


def sample_mask(n: int, sources) -> np.ndarray:
    m = np.zeros(max(n, 1), np.uint8)
    m[np.asarray(sources, np.int64)] = 1
    return m[:n]


def sample_sums(row_ptr, col_idx, sources):
    """Per vertex: (SQ, RQ) = sum of distances from, and count of, the listed
    sources that reach it (one BFS per source)."""
    L = _load()
    row_ptr = _c(row_ptr, np.int32)
    col_idx = _c(col_idx, np.int32) if len(col_idx) else np.zeros(1, np.int32)
    n = len(row_ptr) - 1
    src = _c(sources, np.int32)
    SQ = np.zeros(max(n, 1), np.int64)
    RQ = np.zeros(max(n, 1), np.int32)
    if L.oracle_sample_sums(n, _p(row_ptr), _p(col_idx), len(src), _p(src), _p(SQ), _p(RQ)) != 0:
        raise ValueError("oracle_sample_sums failed")
    return SQ[:n], RQ[:n]


def sample_sums_at(row_ptr, col_idx, sources, verts):
    """(SQ, RQ) of the listed vertices only, one BFS from each vertex."""
    L = _load()
    row_ptr = _c(row_ptr, np.int32)
    col_idx = _c(col_idx, np.int32) if len(col_idx) else np.zeros(1, np.int32)
    n = len(row_ptr) - 1
    mask = sample_mask(n, sources)
    vv = _c(verts, np.int32)
    SQ = np.zeros(max(len(vv), 1), np.int64)
    RQ = np.zeros(max(len(vv), 1), np.int32)
    if L.oracle_sample_sums_at(n, _p(row_ptr), _p(col_idx), _p(mask), len(vv), _p(vv), _p(SQ), _p(RQ)) != 0:
        raise ValueError("oracle_sample_sums_at failed")
    return SQ[:len(vv)], RQ[:len(vv)]


def sample_estimate(n: int, n_pop: int, sources, SQ, RQ):
    """Estimated closeness of every vertex from sample sums (WF form)."""
    L = _load()
    mask = sample_mask(n, sources)
    SQ = _c(SQ, np.int64)
    RQ = _c(RQ, np.int32)
    cc = np.zeros(max(n, 1), np.float64)
    L.oracle_sample_estimate(n, n_pop, len(sources), _p(mask), _p(SQ), _p(RQ), _p(cc))
    return cc[:n]


# --------------------------------------------------------------------------
# whole-graph conveniences used by the tests and the benchmark
# --------------------------------------------------------------------------

def closeness_all(row_ptr, col_idx, nthreads: int | None = None):
    """(S, R, cc) for every vertex of one graph."""
    n = len(row_ptr) - 1
    S, R = bfs_sums(row_ptr, col_idx, None, nthreads)
    return S, R, closeness_wf(n, S, R)


def topk_count(n: int, pnum: int, pden: int) -> int:
    """K = ceil(p*n) in integer arithmetic for p = pnum/pden."""
    return (n * pnum + pden - 1) // pden
