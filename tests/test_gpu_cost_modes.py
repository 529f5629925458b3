"""The geometric-term variants (options.cost_mode) against the oracle's:
component-stratified Monte Carlo and the closed-form KL bound, stage by stage
(teacher-forced, 20,000 splats; flat and needle splats) and end to end.

Bars as for the default estimator: costs within 1e-4 |C| + 1e-5 (FP32 path)
or 1e-6 |C| + 1e-7 (FP64 path); neither variant draws a component, so no
edge can flip."""
import numpy as np
import pytest

import oracle as O
from paper_2603_16103_amd.synth import gen_scene
from tests.test_gpu_parity import _activated32, _splats, _state64, _t, log

pytestmark = pytest.mark.gpu

MODES = [(O.COST_MC_STRAT, "strat"), (O.COST_BOUND, "bound")]


@pytest.fixture(scope="module")
def c1():
    sc = gen_scene(20_000, 1)
    act = _activated32(sc)
    ei, ej = O.union_edges(O.knn(act[0], 16))
    return sc, act, _state64(*act), ei, ej


def _check(got, ref, rel, ab):
    err = np.abs(got.astype(np.float64) - ref)
    bad = err > rel * np.abs(ref) + ab
    log("max abs", float(np.max(err)), "outside", int(np.sum(bad)), "of", bad.size)
    assert not np.any(bad), (np.sum(bad), err[bad][:5], ref[bad][:5])


@pytest.mark.parametrize("mode,name", MODES)
@pytest.mark.parametrize("S,seed", [(1, 0), (4, 9)])
def test_cost_mode_parity(gpu_lib, c1, mode, name, S, seed):
    if mode == O.COST_BOUND and S > 1:
        pytest.skip("the bound draws nothing")
    sc, act, st, ei, ej = c1
    crn = O.crn_block(seed, 1, S)
    log("cost mode", name, "S", S, "edges", ei.size)
    ref = O.edge_costs(st, ei, ej, crn, mode=mode)[0]
    got = gpu_lib.edge_cost(_splats(gpu_lib, *act), _t(ei), _t(ej), crn,
                            gpu_lib.options(cost_mode=mode)).cpu().numpy()
    _check(got, ref, 1e-4, 1e-5)
    got64 = gpu_lib.edge_cost(_splats(gpu_lib, *act), _t(ei), _t(ej), crn,
                              gpu_lib.options(cost_mode=mode,
                                              precision=gpu_lib.PREC_FP64)).cpu().numpy()
    _check(got64, ref, 1e-6, 1e-7)


@pytest.mark.parametrize("mode,name", MODES)
def test_cost_mode_stress_scales(gpu_lib, mode, name):
    sc = gen_scene(20_000, 3, n_planes=64, n_spheres=0, stress=True)
    act = _activated32(sc)
    st = _state64(*act)
    ei, ej = O.union_edges(O.knn(act[0], 24))
    crn = O.crn_block(3, 0, 2)
    log("stress", name, "edges", ei.size)
    ref = O.edge_costs(st, ei, ej, crn, mode=mode)[0]
    got = gpu_lib.edge_cost(_splats(gpu_lib, *act), _t(ei), _t(ej), crn,
                            gpu_lib.options(cost_mode=mode)).cpu().numpy()
    _check(got, ref, 1e-4, 1e-5)


def test_bound_is_above_the_estimate_mean(gpu_lib, c1):
    """Joint convexity: the bound's geometric term is at least the mixture's
    divergence, which the stratified estimate approaches at large S."""
    sc, act, st, ei, ej = c1
    sel = np.arange(0, ei.size, 37)
    a, b = ei[sel], ej[sel]
    S = 16
    lo = np.zeros(sel.size)
    for r in range(8):
        crn = O.crn_block(100 + r, 0, S)
        lo += gpu_lib.edge_cost(_splats(gpu_lib, *act), _t(a), _t(b), crn,
                                gpu_lib.options(cost_mode=O.COST_MC_STRAT, S=S,
                                                app_dims=0)).cpu().numpy()
    lo /= 8
    crn = O.crn_block(0, 0, 1)
    hi = gpu_lib.edge_cost(_splats(gpu_lib, *act), _t(a), _t(b), crn,
                           gpu_lib.options(cost_mode=O.COST_BOUND, app_dims=0)).cpu().numpy()
    # 128 draws per edge: allow the estimate's own noise above the bound
    frac_above = float(np.mean(hi >= lo - 0.05 * np.abs(lo) - 1e-4))
    log("bound >= estimate on", frac_above, "of", sel.size)
    assert frac_above >= 0.99


@pytest.mark.parametrize("mode,name", MODES)
def test_cost_mode_end_to_end(gpu_lib, mode, name):
    import torch
    from tests.e2e_compare import pair_identity
    sc = gen_scene(20_000, 4)
    g = gpu_lib.GaussianTensors.from_scene(sc)
    trace = torch.full((sc.n, 2), -1, dtype=torch.int32, device="cuda")
    opts = gpu_lib.options(seed=2, cost_mode=mode, d_trace=trace)
    log("simplify 20k -> 6k", name)
    res, stats = gpu_lib.simplify(g, 6000, k=16, opts=opts, return_stats=True)
    ref_trace = []
    ref = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, 6000, 16, seed=2,
                     trace=ref_trace, cost_mode=mode)
    assert res.n == ref.n == 6000
    ppr = stats["pairs_per_round"][:stats["rounds"]]
    frac, per = pair_identity(ppr, trace.cpu().numpy(), ref_trace)
    log("identical pairs", frac, per)
    assert frac >= 0.99


def test_bad_cost_mode_is_rejected(gpu_lib, c1):
    sc, act, st, ei, ej = c1
    with pytest.raises(gpu_lib.NanoGSError):
        gpu_lib.edge_cost(_splats(gpu_lib, *act), _t(ei[:10]), _t(ej[:10]),
                          O.crn_block(0, 0, 1), gpu_lib.options(cost_mode=3))
