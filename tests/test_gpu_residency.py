"""Co-residency of the persistent closeness kernels on the device: the
registers and LDS the runtime reports for each kernel are the compiler's,
the bound a launch is held to is the compiler's occupancy in blocks, and
the launch path (cooperative, or an ordinary node inside a stream capture)
is recorded for single-graph calls and for plans."""
import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from oracle import oracle as O
from tests.gpu_common import csr_np, graph_dev, say
from tests.test_abi_host import closeness_kernels_from_report

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")


def test_runtime_attributes_match_the_compiler():
    ks = closeness_kernels_from_report()
    rows = []
    for (kind, nw, block, ps), r in sorted(ks.items()):
        mode = 2 + ps if kind == "k_closeness_multi" else ps
        info = P.closeness_kernel_residency(64 * nw, block, mode)
        slots = ((block + 63) // 64 + 3) // 4
        rows.append((kind, nw * 64, block, ps, r["VGPRs"], r["LDS"], r["occ"], info))
        assert info["vgprs"] == r["VGPRs"], (kind, nw, block, ps, info, r)
        assert info["lds"] == r["LDS"], (kind, nw, block, ps, info, r)
        assert info["bound"] == min(info["query"], r["occ"] // slots), (kind, nw, block, ps, info, r)
        assert info["bound"] >= 1
    for row in rows:
        say("%s W=%d block=%d ps=%d: compiler V=%d LDS=%d occ=%d; runtime %s" % row)


def test_launch_paths_recorded():
    """A single-graph call outside a capture goes out cooperatively; inside
    torch.cuda.graph capture the path taken is recorded (and the replay
    matches the oracle).  A plan reports its persistent launches."""
    h = C.config2(scale=0.03)
    rp, ci = csr_np(h.n, *h.layers[0])
    g = graph_dev(P, rp, ci)
    out = P.hln_closeness_layer(g, width_bits=4096)
    torch.cuda.synchronize()
    P.device_status()
    assert P.last_launch_path() == 1
    S, R = O.bfs_sums(rp, ci)
    cap_out = {"S": torch.empty_like(out["S"]), "R": torch.empty_like(out["R"]), "cc": torch.empty_like(out["cc"]),
               "h2": None}
    ws = P.workspace(P.closeness_workspace_size(h.n, len(ci), h.n, 4096))
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg):
        P.hln_closeness_layer(g, width_bits=4096, out=cap_out, ws=ws)
    path = P.last_launch_path()
    say("single-graph call inside stream capture went out as path", path)
    assert path in (1, 2)
    for rep in range(2):
        cap_out["S"].zero_()
        cg.replay()
        torch.cuda.synchronize()
        P.device_status()
        assert np.array_equal(cap_out["S"].cpu().numpy(), S), rep
        assert np.array_equal(cap_out["R"].cpu().numpy(), R), rep
    plan = P.Plan()
    plan.set_width(h.n, 4096)
    outs = P.Plan.outputs([g])
    plan.run([g], outs)
    torch.cuda.synchronize()
    P.device_status()
    assert plan.launch_paths() == (1, 0)
    plan.reserve([g])
    pg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(pg):
        plan.run([g], outs)
    coop, ordinary = plan.launch_paths()
    say("plan inside stream capture: cooperative %d, ordinary %d" % (coop, ordinary))
    assert coop + ordinary == 1
    outs[0]["S"].zero_()
    pg.replay()
    torch.cuda.synchronize()
    P.device_status()
    assert np.array_equal(outs[0]["S"].cpu().numpy(), S)
