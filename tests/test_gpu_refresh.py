"""Local neighbourhood refresh (options.refresh) and the per-pass pair cap
(options.pass_frac) against the oracle's modes, end to end: the same merges
pass by pass (>= 99% identical provenance pairs), the same final count and
the same number of rows queried per pass."""
import numpy as np
import pytest

import oracle as O
from paper_2603_16103_amd.synth import gen_scene
from tests.test_gpu_parity import log

pytestmark = pytest.mark.gpu


def _run(ng, sc, target, k, **kw):
    import torch
    g = ng.GaussianTensors.from_scene(sc)
    trace = torch.full((sc.n, 2), -1, dtype=torch.int32, device="cuda")
    opts = ng.options(seed=3, d_trace=trace, **kw)
    res, stats = ng.simplify(g, target, k=k, opts=opts, return_stats=True)
    return res, stats, trace.cpu().numpy()


@pytest.mark.parametrize("refresh,frac", [("local", 0.1), ("full", 0.1), ("local", 0.0)])
def test_refresh_and_pass_cap_end_to_end(gpu_lib, refresh, frac):
    from tests.e2e_compare import pair_identity
    ng = gpu_lib
    sc = gen_scene(20_000, 6)
    target, k = 9000, 16
    mode = ng.REFRESH_LOCAL if refresh == "local" else ng.REFRESH_FULL
    log("refresh", refresh, "pass_frac", frac)
    res, stats, trace = _run(ng, sc, target, k, refresh=mode, pass_frac=frac)
    ref_trace, ref_q = [], []
    ref = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, target, k, seed=3,
                     trace=ref_trace, refresh=refresh, pass_frac=frac, requeried=ref_q)
    assert res.n == ref.n == target
    ppr = stats["pairs_per_round"][:stats["rounds"]]
    assert len(ppr) == len(ref_trace)
    frac_id, per = pair_identity(ppr, trace, ref_trace)
    got_q = stats["requery_per_round"][:stats["rounds"]]
    log("identical pairs", frac_id, "queried", got_q, ref_q)
    assert frac_id >= 0.99
    if frac_id == 1.0:
        assert got_q == ref_q
    else:
        assert all(abs(a - b) <= 0.02 * b for a, b in zip(got_q, ref_q))
    if refresh == "local" and frac > 0:
        assert all(q < n for q, n in zip(got_q[1:], stats["n_per_round"][1:]))
    if refresh == "full":
        assert got_q == stats["n_per_round"][:stats["rounds"]]


def test_refresh_options_checked(gpu_lib):
    ng = gpu_lib
    sc = gen_scene(2000, 7)
    g = ng.GaussianTensors.from_scene(sc)
    for kw in (dict(refresh=2), dict(pass_frac=-0.1), dict(pass_frac=1.5),
               dict(pass_frac=float("nan"))):
        with pytest.raises(ng.NanoGSError):
            ng.simplify(g, 500, k=8, opts=ng.options(**kw))
    with pytest.raises(ng.NanoGSError):
        ng.Batch(max_rows=4000, max_k=16, max_jobs=2,
                 opts=ng.options(refresh=ng.REFRESH_LOCAL))
