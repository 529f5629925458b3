"""HIP path vs the FP64 oracle, stage by stage and end to end, on seeded
synthetic scenes (20,000 splats and smaller edge cases).

Each stage is teacher-forced: both sides get the same float32 state.  Bars:
kNN lists, edges and pair selection bit-exact; edge costs within
1e-4 |C| + 1e-5; merged parameters within 1e-5 relative.  Both sides take
the component choice u < pi with pi = w_i / W in double, so a draw can only
pick different components where u lies within double rounding of pi; such
edges would be counted and printed as flips (none are expected).
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2603_16103_amd.synth import gen_scene

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def _activated32(scene):
    """Oracle activation rounded to float32 (the teacher-forced state)."""
    st = O.activate(scene.pos, scene.log_scale, scene.rot, scene.opacity, scene.sh)
    f32 = np.float32
    return (st.mu.astype(f32), st.s.astype(f32), st.q.astype(f32), st.alpha.astype(f32),
            st.f.astype(f32))


def _state64(mu, s, q, al, f):
    """Float32 state widened to float64; the quaternion is renormalised (the
    activated form carries unit quaternions; both sides normalise)."""
    q = q.astype(np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    return O.State(mu.astype(np.float64), s.astype(np.float64), q,
                   al.astype(np.float64), f.astype(np.float64), np.arange(mu.shape[0]))


def _splats(ng, mu, s, q, al, f, origin=None):
    import torch
    return ng.SplatTensors(_t(mu), _t(s), _t(q), _t(al), _t(f),
                           _t(origin, torch.int32) if origin is not None else None)


@pytest.fixture(scope="module")
def c1():
    sc = gen_scene(20_000, 1)
    return sc, _activated32(sc)


# --------------------------------------------------------------------------
# kNN
# --------------------------------------------------------------------------
def test_knn_bit_exact_20k(gpu_lib, c1):
    sc, (mu, *_ ) = c1
    log("knn 20k k=16")
    got = gpu_lib.knn(_t(mu), 16).cpu().numpy()
    ref = O.knn(mu, 16)
    np.testing.assert_array_equal(got, ref)
    log("knn 20k k=24/k=5")
    for k in (24, 5):
        np.testing.assert_array_equal(gpu_lib.knn(_t(mu), k).cpu().numpy(), O.knn(mu, k))


def test_knn_translated_scene(gpu_lib, c1):
    """The 20k scene moved by +1e4 on every axis: the coordinates' float
    rounding is far larger than at the origin, the lists stay exact."""
    sc, (mu, *_ ) = c1
    X = (mu.astype(np.float64) + 1e4).astype(np.float32)
    for k in (16, 5):
        log("translated knn k", k)
        np.testing.assert_array_equal(gpu_lib.knn(_t(X), k).cpu().numpy(), O.knn(X, k))


def test_knn_lattice_ties_and_duplicates(gpu_lib):
    g = np.stack(np.meshgrid(*(np.arange(12),) * 3, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(0)
    perm = rng.permutation(len(g))
    X = g[perm].astype(np.float32)
    for k in (6, 16, 32):
        log("lattice k", k)
        np.testing.assert_array_equal(gpu_lib.knn(_t(X), k).cpu().numpy(), O.knn(X, k))
    # duplicated centres: equal distances, ties by index
    D = np.repeat(rng.normal(size=(300, 3)).astype(np.float32), 4, axis=0)
    np.testing.assert_array_equal(gpu_lib.knn(_t(D), 16).cpu().numpy(), O.knn(D, 16))


@pytest.mark.parametrize("n", [1, 2, 3, 17, 33, 100])
def test_knn_small_n(gpu_lib, n):
    X = np.random.default_rng(n).normal(size=(n, 3)).astype(np.float32)
    np.testing.assert_array_equal(gpu_lib.knn(_t(X), 16).cpu().numpy(), O.knn(X, 16))


# --------------------------------------------------------------------------
# union edges
# --------------------------------------------------------------------------
def test_edges_bit_exact(gpu_lib, c1):
    """The union edges in lexicographic (i, j) order, element by element."""
    sc, (mu, *_ ) = c1
    nbr = O.knn(mu, 16)
    ei, ej = gpu_lib.edges(_t(nbr))
    ri, rj = O.union_edges(nbr)
    np.testing.assert_array_equal(ei.cpu().numpy(), ri)
    np.testing.assert_array_equal(ej.cpu().numpy(), rj)


@pytest.mark.parametrize("n,k", [(1, 16), (2, 1), (7, 32), (5000, 3)])
def test_edges_small_and_padded(gpu_lib, n, k):
    """Rows padded with -1 (k_eff < k), tiny sets, a ragged count."""
    rng = np.random.default_rng(n + k)
    mu = rng.normal(size=(n, 3)).astype(np.float32)
    keff = min(k, n - 1)
    nbr = np.full((n, k), -1, np.int32)
    if keff > 0:
        nbr[:, :keff] = O.knn(mu, keff)
    ei, ej = gpu_lib.edges(_t(nbr))
    ri, rj = O.union_edges(nbr)
    np.testing.assert_array_equal(ei.cpu().numpy(), ri)
    np.testing.assert_array_equal(ej.cpu().numpy(), rj)


# --------------------------------------------------------------------------
# edge cost
# --------------------------------------------------------------------------
def _cost_compare(gpu_cost, ref_cost, u_draws, pa_ref, tol_rel=1e-4, tol_abs=1e-5):
    """Returns (edges outside the bar, max relative error); fails on any edge
    outside the bar unless some draw's u lies within double rounding of pi
    (a flip of the component choice, counted and printed)."""
    err = np.abs(gpu_cost.astype(np.float64) - ref_cost)
    bad = err > tol_rel * np.abs(ref_cost) + tol_abs
    near = np.zeros_like(bad)
    for u in u_draws:
        near |= np.abs(pa_ref - float(u)) < 1e-12
    log("component-choice flips:", int(np.sum(bad & near)), "of", bad.size, "edges")
    assert not np.any(bad & ~near), (np.sum(bad & ~near), err[bad & ~near][:5])
    return int(np.sum(bad)), float(np.max(err / (np.abs(ref_cost) + 1e-12)))


def _pa(st, ei, ej):
    wa = O.mass(st.s[ei], st.alpha[ei])
    wb = O.mass(st.s[ej], st.alpha[ej])
    return wa / (wa + wb)


@pytest.mark.parametrize("S,app_dims,seed", [(1, 48, 0), (4, 48, 7), (1, 3, 3)])
def test_edge_cost_parity(gpu_lib, c1, S, app_dims, seed):
    sc, act = c1
    st = _state64(*act)
    nbr = O.knn(act[0], 16)
    ei, ej = O.union_edges(nbr)
    crn = O.crn_block(seed, 0, S)
    log("cost", S, app_dims, "edges", ei.size)
    ref = O.edge_costs(st, ei, ej, crn, app_dims)[0]
    opts = gpu_lib.options(app_dims=app_dims)
    got = gpu_lib.edge_cost(_splats(gpu_lib, *act), _t(ei), _t(ej), crn, opts).cpu().numpy()
    flips, rel = _cost_compare(got, ref, crn[:, 0], _pa(st, ei, ej))
    log("flips", flips, "max rel", rel)
    assert flips == 0


def test_edge_cost_fp64_mode_is_tighter(gpu_lib, c1):
    sc, act = c1
    st = _state64(*act)
    ei, ej = O.union_edges(O.knn(act[0], 16))
    crn = O.crn_block(11, 2, 2)
    ref = O.edge_costs(st, ei, ej, crn)[0]
    got = gpu_lib.edge_cost(_splats(gpu_lib, *act), _t(ei), _t(ej), crn,
                            gpu_lib.options(precision=gpu_lib.PREC_FP64)).cpu().numpy()
    err = np.abs(got.astype(np.float64) - ref)
    # float64 arithmetic; only the float32 rounding of the stored cost remains
    assert np.all(err <= 1e-6 * np.abs(ref) + 1e-7), np.max(err)


def test_edge_cost_stress_scales(gpu_lib):
    """Flat and needle splats (one or two log-scales near -7)."""
    sc = gen_scene(20_000, 3, n_planes=64, n_spheres=0, stress=True)
    act = _activated32(sc)
    st = _state64(*act)
    ei, ej = O.union_edges(O.knn(act[0], 24))
    crn = O.crn_block(3, 0, 1)
    ref = O.edge_costs(st, ei, ej, crn)[0]
    got = gpu_lib.edge_cost(_splats(gpu_lib, *act), _t(ei), _t(ej), crn).cpu().numpy()
    flips, rel = _cost_compare(got, ref, crn[:, 0], _pa(st, ei, ej))
    log("stress flips", flips, "max rel", rel)
    assert flips == 0


# --------------------------------------------------------------------------
# selection
# --------------------------------------------------------------------------
def _partner_from_pairs(n, pairs):
    p = np.full(n, -1, np.int32)
    for a, b in pairs:
        p[a], p[b] = b, a
    return p


def test_select_bit_exact(gpu_lib, c1):
    sc, act = c1
    st = _state64(*act)
    n = st.n
    ei, ej = O.union_edges(O.knn(act[0], 16))
    cost = gpu_lib.edge_cost(_splats(gpu_lib, *act), _t(ei), _t(ej), O.crn_block(0, 0, 1))
    c32 = cost.cpu().numpy()
    for P in (n, 9000, 1000, 1, 0):
        log("select P", P)
        partner, npairs = gpu_lib.select(_t(ei), _t(ej), cost, n, P)
        ref = O.greedy_pairs(ei, ej, c32.astype(np.float64), n, P)
        assert npairs == len(ref)
        np.testing.assert_array_equal(partner.cpu().numpy(), _partner_from_pairs(n, ref))


def test_select_ties_nan_and_signed_zero(gpu_lib):
    rng = np.random.default_rng(4)
    n = 3000
    X = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    ei, ej = O.union_edges(O.knn(X, 8))
    cost = rng.integers(0, 5, ei.size).astype(np.float32)  # heavy ties
    cost[rng.random(ei.size) < 0.02] = np.nan
    cost[rng.random(ei.size) < 0.01] = np.inf
    z = cost == 0
    cost[z & (rng.random(ei.size) < 0.5)] = -0.0
    # shuffle the edge order and orientation: the result must not depend on it
    perm = rng.permutation(ei.size)
    flip = rng.random(ei.size) < 0.5
    a = np.where(flip, ej, ei)[perm]
    b = np.where(flip, ei, ej)[perm]
    c = cost[perm]
    for P in (n, 700, 5):
        partner, npairs = gpu_lib.select(_t(a), _t(b), _t(c), n, P)
        ref = O.greedy_pairs(ei, ej, cost.astype(np.float64), n, P)
        assert npairs == len(ref)
        np.testing.assert_array_equal(partner.cpu().numpy(), _partner_from_pairs(n, ref))


def test_select_empty(gpu_lib):
    import torch
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    partner, npairs = gpu_lib.select(e, e, e.float(), 10, 5)
    assert npairs == 0 and np.all(partner.cpu().numpy() == -1)


# --------------------------------------------------------------------------
# merge
# --------------------------------------------------------------------------
def _sigma(s, q):
    return O.covariance(s.astype(np.float64), q.astype(np.float64))


def test_merge_parity(gpu_lib, c1):
    sc, act = c1
    st = _state64(*act)
    n = st.n
    ei, ej = O.union_edges(O.knn(act[0], 16))
    cost = O.edge_costs(st, ei, ej, O.crn_block(0, 0, 1))[0]
    pairs = O.greedy_pairs(ei, ej, cost, n, n)
    ref = O.merge_pairs(st, pairs)
    origin = np.arange(n, dtype=np.int32)
    out = gpu_lib.merge(_splats(gpu_lib, *act, origin=origin),
                        _t(_partner_from_pairs(n, pairs)))
    assert out.n == ref.n
    np.testing.assert_array_equal(out.origin.cpu().numpy(), ref.origin)
    mu = out.mu.cpu().numpy().astype(np.float64)
    s = out.scale.cpu().numpy()
    q = out.quat.cpu().numpy()
    al = out.alpha.cpu().numpy().astype(np.float64)
    f = out.sh.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(mu - ref.mu) / np.maximum(np.abs(ref.mu).max(1, keepdims=True), 1)) < 1e-5 * 1.01
    Sg, Sr = _sigma(s, q), O.covariance(ref.s, ref.q)
    fro = np.linalg.norm(Sg - Sr, axis=(1, 2)) / np.linalg.norm(Sr, axis=(1, 2))
    assert fro.max() < 1e-5, fro.max()
    srt = np.sort(s.astype(np.float64), 1)
    assert np.max(np.abs(srt - np.sort(ref.s, 1)) / np.sort(ref.s, 1)) < 1e-5
    assert np.max(np.abs(al - ref.alpha)) < 1e-5
    df = np.linalg.norm(f - ref.f, axis=1) / np.maximum(np.linalg.norm(ref.f, axis=1), 1e-3)
    assert df.max() < 1e-5
    merged = np.isin(np.arange(out.n), np.nonzero(np.isin(ref.origin, pairs.min(1)))[0])
    assert np.all(q[merged, 0] >= 0)


def test_merge_no_pairs_is_identity(gpu_lib, c1):
    sc, act = c1
    n = 500
    sub = [a[:n] for a in act]
    out = gpu_lib.merge(_splats(gpu_lib, *sub), _t(np.full(n, -1, np.int32)))
    assert out.n == n
    np.testing.assert_array_equal(out.mu.cpu().numpy(), sub[0])
    np.testing.assert_array_equal(out.sh.cpu().numpy(), sub[4])


# --------------------------------------------------------------------------
# whole loop
# --------------------------------------------------------------------------
def _run_simplify(gpu_lib, sc, target, k, seed=0, S=1):
    import torch
    g = gpu_lib.GaussianTensors.from_scene(sc)
    trace = torch.full((sc.n, 2), -1, dtype=torch.int32, device="cuda")
    origin = torch.full((sc.n,), -1, dtype=torch.int32, device="cuda")
    opts = gpu_lib.options(seed=seed, S=S, d_trace=trace, d_origin=origin)
    res, stats = gpu_lib.simplify(g, target, k=k, opts=opts, return_stats=True)
    return res, stats, trace.cpu().numpy(), origin.cpu().numpy()[:res.n]


def test_simplify_end_to_end_20k(gpu_lib, c1):
    from tests.e2e_compare import E2E_BARS, compare_clusters, gpu_merges, pair_identity
    sc, _ = c1
    log("simplify 20k -> 10k")
    res, stats, trace, origin = _run_simplify(gpu_lib, sc, 10_000, 16)
    ref_trace = []
    ref = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, 10_000, 16,
                     trace=ref_trace)
    log("stats", stats["n_per_round"], stats["pairs_per_round"], stats["fallback_per_round"])
    assert res.n == ref.n == 10_000
    ppr = stats["pairs_per_round"][:stats["rounds"]]
    frac, per = pair_identity(ppr, trace, ref_trace)
    log("identical pairs", frac, per)
    assert frac >= 0.99
    err = compare_clusters(sc.n, res.numpy(), origin, gpu_merges(ppr, trace), ref, ref_trace)
    log("cluster errors", err)
    assert err["identical_clusters"] >= 0.98
    for f, bar in E2E_BARS.items():
        assert err[f + "_max"] < bar, (f, err)


def test_simplify_output_order_and_passthrough(gpu_lib):
    sc = gen_scene(3000, 21)
    g = gpu_lib.GaussianTensors.from_scene(sc)
    res = gpu_lib.simplify(g, 5000, k=16)  # target >= n: activation round trip only
    assert res.n == sc.n
    pos, ls, rot, op, sh = res.numpy()
    np.testing.assert_array_equal(pos, sc.pos)
    np.testing.assert_array_equal(sh, sc.sh)
    np.testing.assert_allclose(ls, sc.log_scale, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(op, sc.opacity, rtol=1e-4, atol=1e-5)


@pytest.mark.parametrize("n,target,k", [(1, 1, 16), (2, 1, 16), (5, 1, 16), (40, 3, 32),
                                        (1000, 10, 1)])
def test_simplify_small_cases(gpu_lib, n, target, k):
    sc = gen_scene(n, 30 + n)
    res, stats, trace, origin = _run_simplify(gpu_lib, sc, target, k)
    ref = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, target, k)
    assert res.n == ref.n == target
    assert not stats["early_exit"]
    assert sorted(origin.tolist()) == sorted(ref.origin.tolist())


def test_simplify_rejects_non_finite(gpu_lib):
    sc = gen_scene(200, 40)
    sc.sh[7, 5] = np.nan
    g = gpu_lib.GaussianTensors.from_scene(sc)
    with pytest.raises(gpu_lib.NanoGSError) as ei:
        gpu_lib.simplify(g, 100, k=16)
    assert ei.value.status == 3
    sc = gen_scene(200, 40)
    sc.pos[3, 1] = np.inf
    with pytest.raises(gpu_lib.NanoGSError):
        gpu_lib.simplify(gpu_lib.GaussianTensors.from_scene(sc), 100, k=16)
