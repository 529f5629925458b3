"""Device-count stage calls (nanogs_edge_cost_dev, nanogs_select_dev): same
results as the host-count calls, with the edge count and the pair budget
read on the device; the chain cost -> select captured into a graph and
replayed (eager work and synchronisation between replays) gives the eager
result on every replay."""
import numpy as np
import pytest

import oracle as O
from paper_2603_16103_amd.synth import gen_scene
from tests.test_gpu_parity import _activated32, _splats, _t, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup(gpu_lib):
    import torch
    ng = gpu_lib
    sc = gen_scene(12_000, 5)
    act = _activated32(sc)
    nbr = ng.knn(_t(act[0]), 16)
    n, k = nbr.shape
    # capacity-sized edge arrays and the device count, as nanogs_edges leaves them
    ei = torch.empty(n * k, dtype=torch.int32, device="cuda")
    ej = torch.empty(n * k, dtype=torch.int32, device="cuda")
    dm = torch.zeros(1, dtype=torch.int64, device="cuda")
    lib = ng.load()
    nb = lib.nanogs_edges_workspace_bytes(n, k)
    ws = ng._workspace(nb)
    ng._check(lib.nanogs_edges(ng._ptr(nbr), n, k, ng._ptr(ei), ng._ptr(ej), ng._ptr(dm),
                               ng._ptr(ws), nb, ng._stream()))
    torch.cuda.synchronize()
    m = int(dm.item())
    return ng, act, ei, ej, dm, m


@pytest.mark.parametrize("prec", [0, 1])
def test_edge_cost_dev_equals_host_count(setup, prec):
    import torch
    ng, act, ei, ej, dm, m = setup
    crn = O.crn_block(4, 1, 2)
    d_crn = torch.from_numpy(crn).cuda()
    s = _splats(ng, *act)
    got = ng.edge_cost_dev(s, ei, ej, dm, d_crn, ng.options(precision=prec))
    ref = ng.edge_cost(s, ei[:m], ej[:m], crn, ng.options(precision=prec))
    assert np.array_equal(got[:m].cpu().numpy().view(np.uint32), ref.cpu().numpy().view(np.uint32))
    # a smaller device count
    half = torch.full((1,), m // 2, dtype=torch.int64, device="cuda")
    out = ng.edge_cost_dev(s, ei, ej, half, d_crn, ng.options(precision=prec))
    assert np.array_equal(out[:m // 2].cpu().numpy().view(np.uint32),
                          ref[:m // 2].cpu().numpy().view(np.uint32))


def test_select_dev_equals_host_count(setup):
    import torch
    ng, act, ei, ej, dm, m = setup
    n = act[0].shape[0]
    cost = ng.edge_cost(_splats(ng, *act), ei[:m], ej[:m], O.crn_block(0, 0, 1))
    cost_cap = torch.full((ei.shape[0],), float("nan"), device="cuda")
    cost_cap[:m] = cost
    for P in (n, 2000, 1, 0):
        ref_p, ref_n = ng.select(ei[:m], ej[:m], cost, n, P)
        dP = torch.full((1,), P, dtype=torch.int64, device="cuda")
        got_p, got_n = ng.select_dev(ei, ej, cost_cap, dm, n, dP)
        log("P", P, "pairs", ref_n)
        assert int(got_n.item()) == ref_n
        assert np.array_equal(got_p.cpu().numpy(), ref_p.cpu().numpy())


def test_cost_select_chain_in_a_graph(setup):
    import torch
    ng, act, ei, ej, dm, m = setup
    n = act[0].shape[0]
    s = _splats(ng, *act)
    d_crn = torch.from_numpy(O.crn_block(9, 0, 1)).cuda()
    dP = torch.full((1,), n // 3, dtype=torch.int64, device="cuda")
    lib = ng.load()
    # eager run (also sets up the library's pinned host buffer outside capture)
    cost_e = ng.edge_cost_dev(s, ei, ej, dm, d_crn)
    part_e, np_e = ng.select_dev(ei, ej, cost_e, dm, n, dP)
    torch.cuda.synchronize()
    ws_c = ng._workspace(lib.nanogs_edge_cost_workspace_bytes(n, ei.shape[0]))
    ws_s = ng._workspace(lib.nanogs_select_workspace_bytes(n, ei.shape[0]))
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            cost_g = ng.edge_cost_dev(s, ei, ej, dm, d_crn, ws=ws_c)
            part_g, np_g = ng.select_dev(ei, ej, cost_g, dm, n, dP, ws=ws_s)
    torch.cuda.synchronize()
    ref_c = cost_e[:m].cpu().numpy().view(np.uint32)
    ref_p = part_e.cpu().numpy()
    for r in range(4):
        cost_g.fill_(float("nan"))
        part_g.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cost_g[:m].cpu().numpy().view(np.uint32), ref_c), r
        assert np.array_equal(part_g.cpu().numpy(), ref_p), r
        assert int(np_g.item()) == int(np_e.item()), r
        # eager work between replays
        _ = ng.edge_cost_dev(s, ei, ej, dm, d_crn)
        torch.cuda.synchronize()
