"""Opacity pre-filter on the GPU against the oracle: the kept set of the
stage entry point bit-exact on the same float32 opacities (odd and even
counts, thresholds below and above the median, ties at the threshold), and
the whole loop with the filter against the oracle's loop."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2603_16103_amd.synth import gen_scene

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _act32(sc):
    st = O.activate(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh)
    f32 = np.float32
    return (st.mu.astype(f32), st.s.astype(f32), st.q.astype(f32), st.alpha.astype(f32),
            st.f.astype(f32))


@pytest.mark.parametrize("n", [20001, 20000, 7])
@pytest.mark.parametrize("tau", [0.0, 0.005, 0.3, 0.9])
def test_prune_stage_bit_exact(gpu_lib, n, tau):
    ng = gpu_lib
    sc = gen_scene(n, 60 + n % 5)
    mu, s, q, al, f = _act32(sc)
    if n == 20000:
        al[::3] = al[n // 2]  # many opacities equal to one near the median
    st = O.State(mu.astype(np.float64), s.astype(np.float64), q.astype(np.float64),
                 al.astype(np.float64), f.astype(np.float64), np.arange(n))
    ref = O.opacity_prune(st, float(np.float32(tau)))
    org = np.arange(n, dtype=np.int32)
    out = ng.prune(ng.SplatTensors(_t(mu), _t(s), _t(q), _t(al), _t(f), _t(org)), tau)
    got = out.origin.cpu().numpy()
    log("prune", n, tau, "kept", got.size, "of", n)
    np.testing.assert_array_equal(got, ref.origin)
    np.testing.assert_array_equal(out.alpha.cpu().numpy(), al[ref.origin])
    np.testing.assert_array_equal(out.sh.cpu().numpy(), f[ref.origin])


def test_simplify_with_prefilter(gpu_lib):
    import torch
    from tests.e2e_compare import pair_identity
    ng = gpu_lib
    sc = gen_scene(20000, 66)
    tau, target = 0.4, 4000
    trace = torch.full((sc.n, 2), -1, dtype=torch.int32, device="cuda")
    origin = torch.full((sc.n,), -1, dtype=torch.int32, device="cuda")
    res, stats = ng.simplify(ng.GaussianTensors.from_scene(sc), target, k=16,
                             opts=ng.options(tau=tau, d_trace=trace, d_origin=origin),
                             return_stats=True)
    ref_trace = []
    ref = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, target, 16, tau=tau,
                     trace=ref_trace)
    st0 = O.activate(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh)
    kept_ref = O.opacity_prune(st0, tau).n
    log("kept", stats["n_kept"], "oracle", kept_ref)
    assert stats["n_kept"] == kept_ref
    assert res.n == ref.n == target
    org = origin.cpu().numpy()[:res.n]
    assert len(np.unique(org)) == res.n
    frac, per = pair_identity(stats["pairs_per_round"][:stats["rounds"]], trace.cpu().numpy(),
                              ref_trace)
    log("identical merges", frac, per)
    assert frac >= 0.99
