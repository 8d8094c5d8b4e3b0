"""The C-ABI library loads, exports every symbol include/hln.h declares, and
rejects bad arguments on the host before touching the device (these run
without a GPU: device pointers are never dereferenced on the host)."""
import ctypes
import os
import re

import pytest

P = pytest.importorskip("paper_2207_11662_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(0x100000)       # stands for a device pointer; never read on the host
HLN_EINVAL, HLN_ENOMEM, HLN_EUNSUPPORTED = 1, 2, 4


def header_symbols():
    with open(os.path.join(ROOT, "include", "hln.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(hln_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    declared = header_symbols()
    assert declared, "no declarations parsed"
    missing = [s for s in declared if not hasattr(L, s)]
    assert not missing, missing
    assert sorted(P.EXPORTS) == declared


def test_version_and_error_string():
    L = P.lib()
    assert L.hln_version() >= 0x000100
    assert isinstance(L.hln_last_error(), bytes)


def _csr(n=10, nnz=20):
    return P._lib.hln_csr(n, nnz, 0x100000, 0x200000)


def test_closeness_argument_checks():
    L = P.lib()
    o = P._lib.hln_opts(512, 0, 0, None)
    g = _csr()
    call = lambda **kw: L.hln_closeness_layer(kw.get("g", ctypes.byref(g)), kw.get("src", None), kw.get("n_src", 10),
                                              kw.get("opts", ctypes.byref(o)), kw.get("S", FAKE), kw.get("R", FAKE),
                                              None, None, kw.get("ws", FAKE), kw.get("wsb", 1 << 30), None)
    assert call(g=None) == HLN_EINVAL
    assert call(S=None) == HLN_EINVAL
    assert call(n_src=9) == HLN_EINVAL                      # all-source mode needs n_src == n
    bad = P._lib.hln_opts(100, 0, 0, None)
    assert call(opts=ctypes.byref(bad)) == HLN_EINVAL
    assert b"width_bits" in L.hln_last_error()
    bad = P._lib.hln_opts(512, 7, 0, None)
    assert call(opts=ctypes.byref(bad)) == HLN_EINVAL
    assert call(ws=None) == HLN_EINVAL
    assert call(ws=ctypes.c_void_p(0x100001)) == HLN_EINVAL    # misaligned workspace
    g0 = _csr(0, 0)
    assert call(g=ctypes.byref(g0)) == HLN_EINVAL
    # a bitset of n * W / 8 bytes must stay below 2^31 (32-bit buffer offsets)
    big = _csr(1 << 22, 20)
    w4096 = P._lib.hln_opts(4096, 0, 0, None)
    assert call(g=ctypes.byref(big), n_src=1 << 22, opts=ctypes.byref(w4096)) == HLN_EUNSUPPORTED
    assert b"2^31" in L.hln_last_error()


def test_ingest_argument_checks():
    L = P.lib()
    assert L.hln_csr_from_edges(0, 1, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == HLN_EINVAL
    assert L.hln_csr_from_edges(5, -1, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == HLN_EINVAL
    assert L.hln_csr_from_edges(5, 3, None, FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == HLN_EINVAL
    need = L.hln_csr_from_edges_workspace_size(5, 3)
    assert need > 0
    assert L.hln_csr_from_edges(5, 3, FAKE, FAKE, FAKE, FAKE, FAKE, need - 1, None) == HLN_ENOMEM


def test_compose_argument_checks():
    L = P.lib()
    a, b = _csr(10, 20), _csr(10, 30)
    arr = (P._lib.hln_csr * 2)(a, b)
    ws = L.hln_compose_workspace_size(arr, 2)
    assert ws > 0
    assert L.hln_compose_and(arr, 0, FAKE, FAKE, 20, FAKE, ws, None) == HLN_EINVAL       # r = 0
    assert L.hln_compose_and(arr, 65, FAKE, FAKE, 20, FAKE, ws, None) == HLN_EINVAL      # r > 64
    assert L.hln_compose_and(arr, 2, FAKE, FAKE, 19, FAKE, ws, None) == HLN_ENOMEM       # capacity < min nnz
    assert L.hln_compose_or(arr, 2, FAKE, FAKE, 49, FAKE, ws, None) == HLN_ENOMEM        # capacity < sum nnz
    assert L.hln_compose_or(arr, 2, FAKE, FAKE, 50, FAKE, ws - 1, None) == HLN_ENOMEM
    c = _csr(11, 20)
    arr2 = (P._lib.hln_csr * 2)(a, c)
    assert L.hln_compose_and(arr2, 2, FAKE, FAKE, 20, FAKE, ws, None) == HLN_EINVAL      # n mismatch
    assert L.hln_compose_workspace_size(arr2, 2) == 0


def test_select_argument_checks():
    L = P.lib()
    S = (ctypes.c_void_p * 2)(0x100000, 0x100000)
    R = (ctypes.c_void_p * 2)(0x200000, 0x200000)
    ws = L.hln_compose_cc_topk_workspace_size(100)
    args = lambda mode, r, k, wsb=ws: L.hln_compose_cc_topk(mode, 100, r, ctypes.cast(S, ctypes.c_void_p),
                                                           ctypes.cast(R, ctypes.c_void_p), k, FAKE, FAKE, FAKE,
                                                           FAKE, wsb, None)
    assert args(9, 1, 5) == HLN_EINVAL                    # bad mode
    assert args(0, 2, 5) == HLN_EINVAL                    # WF ranks one graph
    assert args(0, 1, 101) == HLN_EINVAL                  # k > n
    assert args(0, 1, -2) == HLN_EINVAL
    assert args(2, 2, 101) == HLN_EINVAL                  # naive top-k: k > n
    assert args(1, 2, 5, ws - 1) == HLN_ENOMEM


def test_batched_ingest_argument_checks():
    L = P.lib()
    EL = P._lib.hln_edge_list
    ok = EL(5, 3, FAKE, FAKE, FAKE, FAKE)
    arr = (EL * 2)(ok, EL(7, 0, None, None, FAKE, None))
    need = L.hln_csr_from_edges_batch_workspace_size(arr, 2)
    assert need > 0
    assert L.hln_csr_from_edges_batch(arr, 2, FAKE, need - 1, None) == HLN_ENOMEM
    assert L.hln_csr_from_edges_batch(arr, 2, ctypes.c_void_p(0x100001), need, None) == HLN_EINVAL   # misaligned
    assert L.hln_csr_from_edges_batch(arr, -1, FAKE, need, None) == HLN_EINVAL
    assert L.hln_csr_from_edges_batch(None, 2, FAKE, need, None) == HLN_EINVAL
    assert L.hln_csr_from_edges_batch(None, 0, None, 0, None) == 0                                   # nothing to do
    for bad in [EL(0, 3, FAKE, FAKE, FAKE, FAKE), EL(5, -1, FAKE, FAKE, FAKE, FAKE),
                EL(5, (1 << 30) + 1, FAKE, FAKE, FAKE, FAKE), EL(5, 3, None, FAKE, FAKE, FAKE),
                EL(5, 3, FAKE, FAKE, None, FAKE)]:
        b = (EL * 2)(ok, bad)
        assert L.hln_csr_from_edges_batch(b, 2, FAKE, 1 << 40, None) == HLN_EINVAL
    # the size query reads only n and m
    assert L.hln_csr_from_edges_batch_workspace_size((EL * 1)(EL(5, 3, None, None, None, None)), 1) == \
        L.hln_csr_from_edges_batch_workspace_size((EL * 1)(ok), 1)
    assert L.hln_csr_from_edges_batch_workspace_size((EL * 1)(EL(0, 3, None, None, None, None)), 1) == 0
    # totals above 2^31 - 1 arcs: split the batch
    big = (EL * 3)(*[EL(10, 1 << 30, FAKE, FAKE, FAKE, FAKE)] * 3)
    assert L.hln_csr_from_edges_batch(big, 3, FAKE, 1 << 40, None) == HLN_EUNSUPPORTED


def test_batched_topk_argument_checks():
    L = P.lib()
    TP = P._lib.hln_topk_problem
    S = (ctypes.c_void_p * 2)(0x100000, 0x100000)
    R = (ctypes.c_void_p * 2)(0x200000, 0x200000)
    sp, rp = ctypes.cast(S, ctypes.c_void_p), ctypes.cast(R, ctypes.c_void_p)
    ok = TP(1, 100, 2, 10, sp, rp, FAKE, FAKE, FAKE)
    arr = (TP * 1)(ok)
    need = L.hln_compose_cc_topk_batch_workspace_size(arr, 1)
    assert need > 0
    assert L.hln_compose_cc_topk_batch(arr, 1, FAKE, need - 1, None) == HLN_ENOMEM
    assert L.hln_compose_cc_topk_batch(None, 0, None, 0, None) == 0
    for bad in [TP(2, 100, 2, 10, sp, rp, FAKE, FAKE, FAKE),      # naive is not a top-k mode
                TP(0, 100, 2, 10, sp, rp, FAKE, FAKE, FAKE),      # WF ranks one graph
                TP(1, 100, 2, 101, sp, rp, FAKE, FAKE, FAKE),     # k > n
                TP(1, 100, 65, 10, sp, rp, FAKE, FAKE, FAKE),     # r > 64
                TP(1, 0, 2, 0, sp, rp, FAKE, FAKE, FAKE),         # n = 0
                TP(1, 100, 2, 10, sp, rp, None, FAKE, FAKE),      # ids NULL
                TP(1, 100, 2, 10, None, rp, FAKE, FAKE, FAKE)]:   # S NULL
        b = (TP * 2)(ok, bad)
        assert L.hln_compose_cc_topk_batch(b, 2, FAKE, 1 << 40, None) == HLN_EINVAL


def test_plan_set_width_host():
    plan = P.Plan()
    for n, w in [(3000, 8), (3000, 16), (3000, 32), (3000, 64), (70000, 512), (70000, 2048)]:
        plan.set_width(n, w)
    assert plan.width(70000) == 2048
    for bad in [(3000, 128), (3000, 4), (3000, 8192), (0, 64)]:
        with pytest.raises(P.HlnError):
            plan.set_width(*bad)
    plan.set_width(70000, 0)
    assert plan.width(70000) == 4096


def test_batched_and_argument_checks():
    L = P.lib()
    AP = P._lib.hln_and_problem
    a, b = _csr(10, 20), _csr(10, 30)
    lay = (P._lib.hln_csr * 2)(a, b)
    lp = ctypes.cast(lay, ctypes.c_void_p)
    ok = AP(2, lp, FAKE, FAKE, 20)
    need = L.hln_compose_and_batch_workspace_size((AP * 1)(ok), 1)
    assert need > 0
    assert L.hln_compose_and_batch((AP * 1)(ok), 1, FAKE, need - 1, None) == HLN_ENOMEM
    assert L.hln_compose_and_batch((AP * 1)(AP(2, lp, FAKE, FAKE, 19)), 1, FAKE, 1 << 40, None) == HLN_ENOMEM
    c = _csr(11, 20)
    lay2 = (P._lib.hln_csr * 2)(a, c)
    for bad in [AP(0, lp, FAKE, FAKE, 20), AP(65, lp, FAKE, FAKE, 20), AP(2, None, FAKE, FAKE, 20),
                AP(2, lp, None, FAKE, 20), AP(2, ctypes.cast(lay2, ctypes.c_void_p), FAKE, FAKE, 20)]:
        assert L.hln_compose_and_batch((AP * 2)(ok, bad), 2, FAKE, 1 << 40, None) == HLN_EINVAL
    assert b"problem 1" in L.hln_last_error()
    assert L.hln_compose_and_batch(None, 0, None, 0, None) == 0
    assert L.hln_compose_and_batch(None, -1, None, 0, None) == HLN_EINVAL


def _resource_report():
    """The compiler's resource-usage remarks for hln_msbfs.hip (written by
    the build next to the objects; compiled here if missing)."""
    from paper_2207_11662_amd import build as B
    if not os.path.exists(B.RESOURCE_REPORT):
        os.makedirs(B.BUILD, exist_ok=True)
        B._compile(os.path.join(B.CSRC, "hln_msbfs.hip"))
    with open(B.RESOURCE_REPORT) as f:
        return f.read()


def closeness_kernels_from_report():
    """{(kind, NW, BLOCK, PS): {'VGPRs', 'LDS', 'occ'}} for k_closeness and
    k_closeness_multi, from the compiler's remarks."""
    out, cur = {}, None
    for line in _resource_report().splitlines():
        m = re.search(r"Function Name: \S*?(k_closeness(?:_multi)?)ILi(\d+)ELi(\d+)(?:ELb([01]))?E", line)
        if m:
            cur = (m.group(1), int(m.group(2)), int(m.group(3)), int(m.group(4) or 0))
            out[cur] = {}
            continue
        if "Function Name" in line:
            cur = None
            continue
        m = re.search(r"remark:\s+(VGPRs|AGPRs|LDS Size \[bytes/block\]|Occupancy \[waves/SIMD\]): (\d+)", line)
        if m and cur:
            key = {"VGPRs": "VGPRs", "AGPRs": "AGPRs", "LDS Size [bytes/block]": "LDS",
                   "Occupancy [waves/SIMD]": "occ"}[m.group(1)]
            out[cur][key] = int(m.group(2))
    return out


def test_residency_bound_matches_the_compiler():
    """The co-residency bound the persistent launches are held to
    (hln_resident_blocks: VGPRs and LDS against CDNA4's register file and
    LDS) equals, for every closeness kernel the library builds, the blocks
    per compute unit that the compiler's own occupancy figure allows
    (waves per SIMD / wave slots a block takes per SIMD).  The 256-thread
    kernels use 115-190 VGPRs: at most 4 waves per SIMD, so at most 4
    blocks per compute unit, not the 7 an occupancy answer once claimed."""
    L = P.lib()
    ks = closeness_kernels_from_report()
    assert len(ks) >= 42, len(ks)
    for (kind, nw, block, ps), r in sorted(ks.items()):
        assert r.get("AGPRs", 0) == 0
        slots = ((block + 63) // 64 + 3) // 4
        want = r["occ"] // slots
        got = L.hln_resident_blocks(r["VGPRs"], r["LDS"], block)
        assert got == want, (kind, nw, block, ps, r, got)
        assert got >= 1, (kind, nw, block, ps)
    # the 1024-thread kernels the library launches by default: one block per CU
    assert all(L.hln_resident_blocks(r["VGPRs"], r["LDS"], b) == 1 for (k, nw, b, ps), r in ks.items() if b == 1024)
    assert all(L.hln_resident_blocks(r["VGPRs"], r["LDS"], b) <= 4 for (k, nw, b, ps), r in ks.items() if b == 256)


def test_resident_blocks_arithmetic():
    L = P.lib()
    assert L.hln_resident_blocks(64, 0, 256) == 8          # 8 waves per SIMD, one slot each
    assert L.hln_resident_blocks(72, 0, 256) == 7
    assert L.hln_resident_blocks(128, 0, 1024) == 1        # 4 waves per SIMD, a block takes 4
    assert L.hln_resident_blocks(129, 0, 1024) == 0        # 136 VGPRs: 3 waves per SIMD
    assert L.hln_resident_blocks(137, 0, 256) == 3
    assert L.hln_resident_blocks(24, 40 * 1024, 64) == 4   # LDS-bound
    assert L.hln_resident_blocks(24, 0, 64) == 8
    assert L.hln_resident_blocks(-1, 0, 64) == 0
    assert L.hln_resident_blocks(64, 0, 2048) == 0


def test_static_entry_point_host_checks():
    """hln_closeness_layer_static (no workspace, for callers that cannot
    allocate) checks its arguments on the host like hln_closeness_layer; its
    scratch size is the header's constant."""
    L = P.lib()
    assert L.hln_closeness_layer_static(None, None, 0, None, FAKE, FAKE, None, None, None) == HLN_EINVAL
    g = _csr()
    bad = P._lib.hln_opts(100, 0, 0, None)
    assert L.hln_closeness_layer_static(ctypes.byref(g), None, 10, ctypes.byref(bad), FAKE, FAKE, None, None,
                                        None) == HLN_EINVAL
    g0 = _csr(0, 0)
    ok = P._lib.hln_opts(512, 0, 0, None)
    assert L.hln_closeness_layer_static(ctypes.byref(g0), None, 0, ctypes.byref(ok), FAKE, FAKE, None, None,
                                        None) == HLN_EINVAL
    with open(os.path.join(ROOT, "include", "hln.h")) as f:
        m = re.search(r"#define HLN_STATIC_SCRATCH_BYTES \((\d+)u \* (\d+)u \* (\d+)u\)", f.read())
    assert m and int(m.group(1)) * int(m.group(2)) * int(m.group(3)) == P._lib.HLN_STATIC_SCRATCH_BYTES
