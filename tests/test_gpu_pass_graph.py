"""One whole pass of Algorithm 1 through the stage calls, with every count
left on the device (kNN -> union edges -> edge costs -> greedy pairs ->
merge), captured into a HIP graph and replayed: every replay (with eager
work and synchronisation between replays) gives the eager pass's output
bit for bit, and the eager pass equals the host-count stage calls."""
import numpy as np
import pytest

import oracle as O
from paper_2603_16103_amd.synth import gen_scene
from tests.test_gpu_parity import log

pytestmark = pytest.mark.gpu


def _pass(ng, s, k, d_crn, dP, ws):
    nbr = ng.knn(s.mu, k, ws=ws["knn"])
    ei, ej, dm = ng.edges_dev(nbr, ws=ws["edges"])
    cost = ng.edge_cost_dev(s, ei, ej, dm, d_crn, ws=ws["cost"])
    partner, dnp = ng.select_dev(ei, ej, cost, dm, s.n, dP, ws=ws["select"])
    out, dn = ng.merge_dev(s, partner, ws=ws["merge"])
    return out, dn, dnp


def _bytes(out, n):
    return [x[:n].cpu().numpy().view(np.uint32)
            for x in (out.mu, out.scale, out.quat, out.alpha, out.sh)] + [out.origin[:n].cpu().numpy()]


@pytest.mark.parametrize("n,k", [(20_000, 16), (3000, 8)])
def test_pass_captured_and_replayed(gpu_lib, n, k):
    import torch
    ng = gpu_lib
    lib = ng.load()
    sc = gen_scene(n, 31)
    g = ng.GaussianTensors.from_scene(sc)
    s = ng.activate(g)
    s.origin = torch.arange(n, dtype=torch.int32, device="cuda")
    crn = O.crn_block(5, 0, 1)
    d_crn = torch.from_numpy(crn).cuda()
    dP = torch.full((1,), n // 3, dtype=torch.int64, device="cuda")
    ws = {"knn": ng._workspace(lib.nanogs_knn_workspace_bytes(n, k)),
          "edges": ng._workspace(lib.nanogs_edges_workspace_bytes(n, k)),
          "cost": ng._workspace(lib.nanogs_edge_cost_workspace_bytes(n, n * k)),
          "select": ng._workspace(lib.nanogs_select_workspace_bytes(n, n * k)),
          "merge": ng._workspace(lib.nanogs_merge_workspace_bytes(n))}
    # eager, device counts
    out_e, dn_e, dnp_e = _pass(ng, s, k, d_crn, dP, ws)
    torch.cuda.synchronize()
    n_e = int(dn_e.item())
    ref = _bytes(out_e, n_e)
    # eager, host counts (the plain stage calls)
    nbr = ng.knn(s.mu, k)
    ei, ej = ng.edges(nbr)
    cost = ng.edge_cost(s, ei, ej, crn)
    partner, npairs = ng.select(ei, ej, cost, n, n // 3)
    out_h = ng.merge(s, partner)
    assert out_h.n == n_e == n - npairs == n - int(dnp_e.item())
    for a, b in zip(_bytes(out_h, n_e), ref):
        assert np.array_equal(a, b)
    # captured once, replayed
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            out_g, dn_g, dnp_g = _pass(ng, s, k, d_crn, dP, ws)
    torch.cuda.synchronize()
    for r in range(4):
        out_g.mu.fill_(float("nan"))
        dn_g.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        assert int(dn_g.item()) == n_e, r
        for a, b in zip(_bytes(out_g, n_e), ref):
            assert np.array_equal(a, b), r
        _ = ng.edge_cost_dev(s, *ng.edges_dev(ng.knn(s.mu, k))[:3], d_crn)  # eager work between
        torch.cuda.synchronize()
    # timing of the pass: eager launches against one replay
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(5):
        _pass(ng, s, k, d_crn, dP, ws)
    ev[1].record()
    ev[2].record()
    for _ in range(5):
        graph.replay()
    ev[3].record()
    torch.cuda.synchronize()
    log(f"pass at n={n}: eager {ev[0].elapsed_time(ev[1]) / 5:.3f} ms, "
        f"graph replay {ev[2].elapsed_time(ev[3]) / 5:.3f} ms")
