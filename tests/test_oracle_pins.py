"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
generator vectors, closed forms, invariants, special cases with a 1-D
quadrature answer, an independent library sampler, brute force.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate, stats
from scipy.spatial import cKDTree

import oracle as O
from paper_2603_16103_amd.synth import gen_scene


def _state(mu, s, q, alpha, f=None):
    mu = np.asarray(mu, float)
    n = mu.shape[0]
    f = np.zeros((n, 48)) if f is None else np.asarray(f, float)
    return O.State(mu, np.asarray(s, float), np.asarray(q, float),
                   np.asarray(alpha, float), f, np.arange(n))


def _rand_quat(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


# --------------------------------------------------------------------------
# Common random numbers: published SplitMix64 vectors, Box-Muller moments
# --------------------------------------------------------------------------
def test_splitmix64_published_vectors():
    # first output for state 0, and the first five outputs for seed 1234567
    assert O.splitmix64(0) == 0xE220A8397B1DCDAF
    x, got = 1234567, []
    for _ in range(5):
        got.append(O.splitmix64(x))
        x = (x + 0x9E3779B97F4A7C15) % (1 << 64)
    assert got == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_crn_distribution():
    blk = np.concatenate([O.crn_block(7, r, 512) for r in range(8)])
    u, z = blk[:, 0].astype(float), blk[:, 1:].astype(float)
    assert np.all((u >= 0) & (u <= 1))
    assert abs(u.mean() - 0.5) < 0.02
    assert np.all(np.abs(z.mean(0)) < 0.06)
    assert np.all(np.abs(z.var(0) - 1.0) < 0.08)
    # different rounds and seeds give different draws
    assert not np.array_equal(O.crn_block(7, 0, 4), O.crn_block(7, 1, 4))
    assert not np.array_equal(O.crn_block(7, 0, 4), O.crn_block(8, 0, 4))
    # Kolmogorov-Smirnov against the standard normal and uniform
    assert stats.kstest(z[:, 0], "norm").pvalue > 1e-3
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_crn_golden_fixture():
    """The stored known-answer block is what the generator writes."""
    from tests.golden.make_golden import load_crn_golden
    for (seed, r, S), vals in load_crn_golden().items():
        np.testing.assert_array_equal(O.crn_block(seed, r, S), vals)


# --------------------------------------------------------------------------
# Boundary: stored <-> activated
# --------------------------------------------------------------------------
def test_activation_round_trip():
    sc = gen_scene(500, 11)
    st = O.activate(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh)
    assert np.allclose(np.linalg.norm(st.q, axis=1), 1.0, atol=1e-14)
    assert np.all((st.alpha > 0) & (st.alpha < 1))
    pos, ls, rot, op, sh = O.deactivate(st)
    np.testing.assert_array_equal(pos, sc.pos)
    np.testing.assert_allclose(ls, sc.log_scale, rtol=1e-6)
    np.testing.assert_allclose(op, sc.opacity, rtol=1e-5, atol=1e-6)
    r = sc.rot.astype(float)
    r = r / np.linalg.norm(r, axis=1, keepdims=True)
    r *= np.where(r[:, :1] < 0, -1, 1)
    np.testing.assert_allclose(rot, r, atol=1e-6)
    np.testing.assert_array_equal(sh, sc.sh)


def test_activation_special_values():
    st = O.activate(np.zeros((2, 3)), np.zeros((2, 3)), np.zeros((2, 4)),
                    np.array([0.0, 100.0]), np.zeros((2, 48)))
    np.testing.assert_array_equal(st.q, [[1, 0, 0, 0], [1, 0, 0, 0]])
    assert st.alpha[0] == 0.5 and st.alpha[1] == 1.0
    st.alpha[:] = [0.0, 1.0]
    _, _, _, op, _ = O.deactivate(st)
    assert np.all(np.isfinite(op))
    assert op[0] < -16 and op[1] > 16


# --------------------------------------------------------------------------
# kNN: integer-lattice closed form, KD-tree library, k_eff edge cases
# --------------------------------------------------------------------------
def _lattice(m):
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m),
                             indexing="ij"), -1).reshape(-1, 3)
    return g.astype(np.float32)


def test_knn_lattice_closed_form():
    m = 6
    X = _lattice(m)  # index = (x*m + y)*m + z
    # interior point (2,2,2): 6 neighbours at distance 1, then 12 at sqrt2,
    # then 8 at sqrt3; equal distances are ordered by index
    q = (2 * m + 2) * m + 2
    def idx(dx, dy, dz):
        return ((2 + dx) * m + 2 + dy) * m + 2 + dz
    shells = {}
    for dx, dy, dz in itertools.product((-1, 0, 1), repeat=3):
        d2 = dx * dx + dy * dy + dz * dz
        if d2:
            shells.setdefault(d2, []).append(idx(dx, dy, dz))
    expect = sorted(shells[1]) + sorted(shells[2]) + sorted(shells[3])
    for k in (1, 6, 10, 18, 24):
        for method in ("brute", "tree"):
            got = O.knn(X, k, queries=[q], method=method)[0]
            assert list(got) == expect[:k], (k, method)


def test_knn_brute_equals_tree_and_kdtree():
    sc = gen_scene(3000, 5)
    X = sc.pos
    for k in (1, 8, 16):
        a = O.knn(X, k, method="brute")
        b = O.knn(X, k, method="tree")
        np.testing.assert_array_equal(a, b)
    # distances agree with the library KD-tree (set of k distances)
    tree = cKDTree(X.astype(np.float64))
    d, _ = tree.query(X.astype(np.float64), k=17)
    Xd = X.astype(np.float64)
    dd = np.sqrt(np.sum((Xd[a] - Xd[:, None]) ** 2, axis=-1))
    np.testing.assert_allclose(dd, d[:, 1:], rtol=1e-12, atol=1e-15)
    # lattices are full of exact ties
    L = _lattice(7)
    np.testing.assert_array_equal(O.knn(L, 16, method="brute"),
                                  O.knn(L, 16, method="tree"))


def test_knn_small_n_and_duplicates():
    X = np.zeros((5, 3), np.float32)  # all coincident: order by index
    got = O.knn(X, 16)
    assert got.shape == (5, 16)
    for i in range(5):
        assert list(got[i, :4]) == [j for j in range(5) if j != i]
        assert np.all(got[i, 4:] == -1)
    assert np.all(O.knn(np.zeros((1, 3), np.float32), 4) == -1)


# --------------------------------------------------------------------------
# Union edges: count identity
# --------------------------------------------------------------------------
def test_union_edges_count_identity():
    sc = gen_scene(2000, 9)
    nbr = O.knn(sc.pos, 16)
    ei, ej = O.union_edges(nbr)
    assert np.all(ei < ej)
    key = ei.astype(np.int64) * 2001 + ej
    assert np.all(np.diff(key) > 0)  # sorted, unique
    n, k = nbr.shape
    directed = {(i, int(j)) for i in range(n) for j in nbr[i]}
    mutual = sum(1 for (i, j) in directed if i < j and (j, i) in directed)
    assert ei.size == n * k - mutual
    es = set(zip(ei.tolist(), ej.tolist()))
    assert all((min(i, j), max(i, j)) in es for (i, j) in directed)


# --------------------------------------------------------------------------
# Covariance and its factorisation
# --------------------------------------------------------------------------
def test_quaternion_round_trip():
    rng = np.random.default_rng(0)
    q = _rand_quat(rng, 200)
    q *= np.where(q[:, :1] < 0, -1, 1)
    R = O.rotation_matrix(q)
    np.testing.assert_allclose(R @ np.swapaxes(R, 1, 2), np.eye(3)[None].repeat(200, 0),
                               atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)
    np.testing.assert_allclose(O.quat_from_rotation(R), q, atol=1e-13)
    # rotating e_x by 90 degrees about z gives e_y
    h = math.sqrt(0.5)
    Rz = O.rotation_matrix(np.array([h, 0, 0, h]))
    np.testing.assert_allclose(Rz @ [1, 0, 0], [0, 1, 0], atol=1e-15)


def test_cov_factor_round_trip_and_invariants():
    rng = np.random.default_rng(1)
    s = np.exp(rng.normal(-4, 1.0, (300, 3)))
    q = _rand_quat(rng, 300)
    Sig = O.covariance(s, q)
    s2, q2 = O.scale_rot_from_cov(Sig)
    np.testing.assert_allclose(O.covariance(s2, q2), Sig, rtol=0,
                               atol=1e-12 * np.abs(Sig).max())
    assert np.all(np.diff(s2, axis=1) <= 0)  # decreasing
    assert np.all(q2[:, 0] >= 0)
    # characteristic-polynomial invariants: trace, principal minors, det
    l = s2 ** 2
    np.testing.assert_allclose(l.sum(1), np.trace(Sig, axis1=1, axis2=2), rtol=1e-12)
    np.testing.assert_allclose(l.prod(1), np.prod(s ** 2, 1), rtol=1e-9)
    m2 = (Sig[:, 0, 0] * Sig[:, 1, 1] - Sig[:, 0, 1] ** 2 + Sig[:, 0, 0] * Sig[:, 2, 2]
          - Sig[:, 0, 2] ** 2 + Sig[:, 1, 1] * Sig[:, 2, 2] - Sig[:, 1, 2] ** 2)
    np.testing.assert_allclose(l[:, 0] * l[:, 1] + l[:, 0] * l[:, 2] + l[:, 1] * l[:, 2],
                               m2, rtol=1e-9)
    # sorted scales are the input scales
    np.testing.assert_allclose(s2, np.sort(s, 1)[:, ::-1], rtol=1e-9)


def test_mass_is_integral_of_density():
    """w = (2 pi)^{3/2} alpha prod s equals the integral of
    alpha exp(-x^T Sigma^-1 x / 2) (Eq. unnormalized_splats)."""
    s = np.array([0.7, 0.4, 0.2])
    q = np.array([0.9, 0.2, -0.3, 0.25])
    q /= np.linalg.norm(q)
    alpha = 0.37
    Sinv = np.linalg.inv(O.covariance(s, q))
    h = 0.035
    g = np.arange(-4.0, 4.0 + h / 2, h)
    X, Y = np.meshgrid(g, g, indexing="ij")
    tot = 0.0
    for zz in g:
        P = np.stack([X, Y, np.full_like(X, zz)], -1)
        m = np.einsum("...i,ij,...j->...", P, Sinv, P)
        tot += alpha * np.exp(-0.5 * m).sum()
    tot *= h ** 3
    assert abs(tot - O.mass(s, alpha)) < 1e-6 * O.mass(s, alpha) + 1e-9


# --------------------------------------------------------------------------
# MPMM: moment preservation and closed-form special cases
# --------------------------------------------------------------------------
def _rand_pairs(rng, m):
    mu_a = rng.normal(0, 1, (m, 3))
    mu_b = mu_a + rng.normal(0, 0.1, (m, 3))
    s_a = np.exp(rng.normal(-3, 0.5, (m, 3)))
    s_b = np.exp(rng.normal(-3, 0.5, (m, 3)))
    return (mu_a, s_a, _rand_quat(rng, m), rng.uniform(0.01, 1, m), rng.normal(size=(m, 48)),
            mu_b, s_b, _rand_quat(rng, m), rng.uniform(0.01, 1, m), rng.normal(size=(m, 48)))


def test_mpmm_preserves_mass_weighted_moments():
    rng = np.random.default_rng(2)
    A = _rand_pairs(rng, 200)
    mu_a, s_a, q_a, al_a, f_a, mu_b, s_b, q_b, al_b, f_b = A
    mum, Sm, am, fm = O.mpmm(*A)
    # mixture of the unnormalised densities: total mass, first and second
    # moments computed from each component's own moments
    wa = (2 * np.pi) ** 1.5 * al_a * np.prod(s_a, 1)
    wb = (2 * np.pi) ** 1.5 * al_b * np.prod(s_b, 1)
    Sa, Sb = O.covariance(s_a, q_a), O.covariance(s_b, q_b)
    M1 = wa[:, None] * mu_a + wb[:, None] * mu_b
    M2 = (wa[:, None, None] * (Sa + mu_a[:, :, None] * mu_a[:, None, :])
          + wb[:, None, None] * (Sb + mu_b[:, :, None] * mu_b[:, None, :]))
    W = wa + wb
    np.testing.assert_allclose(W[:, None] * mum, M1, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(W[:, None, None] * (Sm + mum[:, :, None] * mum[:, None, :]),
                               M2, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(W[:, None] * fm, wa[:, None] * f_a + wb[:, None] * f_b,
                               rtol=1e-12, atol=1e-12)
    assert np.all(am >= np.maximum(al_a, al_b) - 1e-15) and np.all(am <= 1)
    # symmetric in the pair
    B = A[5:] + A[:5]
    for x, y in zip(O.mpmm(*A), O.mpmm(*B)):
        np.testing.assert_allclose(x, y, rtol=1e-14, atol=1e-15)


def test_mpmm_identical_copy_and_zero_opacity():
    rng = np.random.default_rng(3)
    A = _rand_pairs(rng, 50)
    same = A[:5] + A[:5]
    mum, Sm, am, fm = O.mpmm(*same)
    np.testing.assert_allclose(mum, A[0], rtol=1e-14)
    np.testing.assert_allclose(Sm, O.covariance(A[1], A[2]), rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(fm, A[4], rtol=1e-14)
    np.testing.assert_allclose(am, 2 * A[3] - A[3] ** 2, rtol=1e-14)
    zero_b = A[:5] + (A[5], A[6], A[7], np.zeros(50), A[9])
    mum, Sm, am, fm = O.mpmm(*zero_b)
    np.testing.assert_allclose(mum, A[0], rtol=1e-15)
    np.testing.assert_allclose(Sm, O.covariance(A[1], A[2]), rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(am, A[3], rtol=1e-14)


def test_mpmm_equivariance():
    rng = np.random.default_rng(4)
    A = list(_rand_pairs(rng, 30))
    mum, Sm, _, _ = O.mpmm(*A)
    h = math.sqrt(0.5)
    r = np.array([h, 0, h, 0])  # 90 degrees about y
    Rm = O.rotation_matrix(r)
    t = np.array([3.0, -1.0, 2.0])
    B = list(A)
    for i in (0, 5):
        B[i] = A[i] @ Rm.T + t
    for i in (2, 7):  # q' = r * q (Hamilton product)
        w1, x1, y1, z1 = r
        w2, x2, y2, z2 = A[i].T
        B[i] = np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                         w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                         w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)
    mum2, Sm2, _, _ = O.mpmm(*B)
    np.testing.assert_allclose(mum2, mum @ Rm.T + t, atol=1e-12)
    np.testing.assert_allclose(Sm2, Rm @ Sm @ Rm.T, atol=1e-14)


# --------------------------------------------------------------------------
# D_geo: zero cases, 1-D reduction, entropy identity, convexity bound,
# invariance
# --------------------------------------------------------------------------
def _iid_crn(rng, S):
    blk = np.empty((S, 4), np.float32)
    blk[:, 0] = rng.random(S)
    blk[:, 1:] = rng.normal(size=(S, 3))
    return blk


def test_dgeo_zero_for_identical_pair_and_zero_weight():
    rng = np.random.default_rng(5)
    n = 40
    mu = rng.normal(size=(n, 3))
    s = np.exp(rng.normal(-4, 0.5, (n, 3)))
    q = _rand_quat(rng, n)
    al = rng.uniform(0.05, 1, n)
    st = _state(np.concatenate([mu, mu]), np.concatenate([s, s]),
                np.concatenate([q, q]), np.concatenate([al, al]))
    ei, ej = np.arange(n), np.arange(n) + n
    for seed in range(3):
        c, dgeo, dapp = O.edge_costs(st, ei, ej, O.crn_block(seed, 0, 3))
        assert np.max(np.abs(dgeo)) < 1e-12 and np.all(dapp == 0)
    st2 = _state(np.concatenate([mu, mu + 0.05]), np.concatenate([s, s * 1.5]),
                 np.concatenate([q, _rand_quat(rng, n)]),
                 np.concatenate([np.zeros(n), al]))
    _, dgeo, _ = O.edge_costs(st2, ei, ej, O.crn_block(1, 0, 2))
    assert np.max(np.abs(dgeo)) < 1e-12


def _kl_1d(pi, delta):
    """KL(pi N(0,1) + (1-pi) N(delta,1) || N(m, v)) with (m, v) the
    matched moments, by quadrature of the mixture entropy."""
    v = 1.0 + pi * (1 - pi) * delta ** 2
    def p(t):
        return (pi * stats.norm.pdf(t) + (1 - pi) * stats.norm.pdf(t - delta))
    def integrand(t):
        pt = p(t)
        return -pt * math.log(pt) if pt > 0 else 0.0
    H = integrate.quad(integrand, -12, delta + 12, limit=200, epsabs=1e-12)[0]
    return 0.5 * math.log(2 * math.pi * math.e * v) - H


def test_dgeo_equal_covariance_reduces_to_1d():
    """Equal covariances: in the whitened frame the pair differs along one
    axis only, so KL(p~ || q_m) is a 1-D quantity (quadrature)."""
    rng = np.random.default_rng(6)
    s = np.array([0.05, 0.02, 0.01])
    q = _rand_quat(rng, 1)[0]
    Sig = O.covariance(s, q)
    L = np.linalg.cholesky(Sig)
    for pi, delta in ((0.3, 3.32), (0.5, 1.0), (0.8, 5.0)):
        d = L @ np.array([delta, 0.0, 0.0])
        # masses set by opacity only (equal scales)
        al_a, al_b = pi, 1 - pi
        st = _state([[0, 0, 0], d], [s, s], [q, q], [al_a, al_b])
        crn = _iid_crn(rng, 1 << 17)
        _, dgeo, _ = O.edge_costs(st, [0], [1], crn)
        kl = _kl_1d(pi, delta)
        # standard error of the mean of the per-sample terms
        assert abs(dgeo[0] - kl) < 0.012 + 0.01 * kl, (pi, delta, dgeo[0], kl)


def test_dgeo_entropy_identity_and_convexity_bound():
    """E[estimator] = H(q_m) - H(p~) with H(p~) from an independent library
    sampler/density, and 0 <= KL <= pi KL(N_a||q_m) + (1-pi) KL(N_b||q_m)
    (joint convexity, closed form of Appendix A)."""
    rng = np.random.default_rng(7)
    mu_a, mu_b = np.zeros(3), np.array([0.05, -0.02, 0.03])
    s_a, s_b = np.array([0.04, 0.02, 0.008]), np.array([0.03, 0.03, 0.01])
    q_a, q_b = _rand_quat(rng, 2)
    al_a, al_b = 0.6, 0.4
    st = _state([mu_a, mu_b], [s_a, s_b], [q_a, q_b], [al_a, al_b])
    _, dgeo, _ = O.edge_costs(st, [0], [1], _iid_crn(rng, 1 << 17))
    Sa, Sb = O.covariance(s_a, q_a), O.covariance(s_b, q_b)
    wa = al_a * np.prod(s_a)
    wb = al_b * np.prod(s_b)
    pi = wa / (wa + wb)
    mum = pi * mu_a + (1 - pi) * mu_b
    d = mu_a - mu_b
    Sm = pi * Sa + (1 - pi) * Sb + pi * (1 - pi) * np.outer(d, d)
    na = stats.multivariate_normal(mu_a, Sa)
    nb = stats.multivariate_normal(mu_b, Sb)
    M = 400_000
    ka = rng.random(M) < pi
    xs = np.where(ka[:, None], na.rvs(M, random_state=rng), nb.rvs(M, random_state=rng))
    lp = np.logaddexp(np.log(pi) + na.logpdf(xs), np.log(1 - pi) + nb.logpdf(xs))
    H_mix = -lp.mean()
    H_m = 0.5 * math.log((2 * math.pi * math.e) ** 3 * np.linalg.det(Sm))
    kl = H_m - H_mix
    assert abs(dgeo[0] - kl) < 0.015 + 0.02 * abs(kl), (dgeo[0], kl)

    def kl_gauss(m0, S0, m1, S1):
        S1i = np.linalg.inv(S1)
        dm = m1 - m0
        return 0.5 * (np.trace(S1i @ S0) + dm @ S1i @ dm - 3
                      + math.log(np.linalg.det(S1) / np.linalg.det(S0)))
    bound = pi * kl_gauss(mu_a, Sa, mum, Sm) + (1 - pi) * kl_gauss(mu_b, Sb, mum, Sm)
    assert -0.01 < dgeo[0] < bound + 0.01


def test_dgeo_isotropic_s1_closed_form():
    """S = 1, two unit isotropic splats, equal mass, u picks the first: the
    estimator is a scalar expression of z (derived by hand: merged
    covariance I + delta^2/4 e1 e1^T)."""
    delta = 1.7
    st = _state([[0, 0, 0], [delta, 0, 0]], np.ones((2, 3)), [[1, 0, 0, 0]] * 2, [0.5, 0.5])
    for z in ([0.3, -0.4, 1.1], [-1.2, 0.0, 0.5]):
        crn = np.array([[0.25] + z], np.float32)
        zz = crn[0, 1:].astype(float)
        ln_a = -0.5 * zz @ zz
        ln_b = -0.5 * ((zz[0] - delta) ** 2 + zz[1] ** 2 + zz[2] ** 2)
        v = 1 + delta ** 2 / 4
        ln_m = -0.5 * ((zz[0] - delta / 2) ** 2 / v + zz[1] ** 2 + zz[2] ** 2) - 0.5 * math.log(v)
        g = math.log(0.5 * math.exp(ln_a) + 0.5 * math.exp(ln_b)) - ln_m
        _, dgeo, _ = O.edge_costs(st, [0], [1], crn)
        assert abs(dgeo[0] - g) < 1e-13


def test_dgeo_translation_scale_invariance_fixed_draws():
    rng = np.random.default_rng(8)
    n = 30
    mu = rng.normal(size=(2 * n, 3))
    s = np.exp(rng.normal(-3, 0.5, (2 * n, 3)))
    q = _rand_quat(rng, 2 * n)
    al = rng.uniform(0.05, 1, 2 * n)
    ei, ej = np.arange(n), np.arange(n) + n
    crn = O.crn_block(3, 2, 4)
    base = O.edge_costs(_state(mu, s, q, al), ei, ej, crn)[1]
    c = 2.5
    moved = O.edge_costs(_state(c * mu + [1.0, -2.0, 0.5], c * s, q, al), ei, ej, crn)[1]
    np.testing.assert_allclose(moved, base, rtol=1e-9, atol=1e-11)


def test_dapp_closed_form():
    rng = np.random.default_rng(9)
    f = rng.normal(size=(2, 48))
    st = _state(np.zeros((2, 3)), np.ones((2, 3)) * 0.1, [[1, 0, 0, 0]] * 2, [0.5, 0.5], f)
    c, dgeo, dapp = O.edge_costs(st, [0], [1], O.crn_block(0, 0, 1))
    assert abs(dapp[0] - np.sum((f[0] - f[1]) ** 2)) < 1e-12
    _, _, dapp3 = O.edge_costs(st, [0], [1], O.crn_block(0, 0, 1), app_dims=3)
    assert abs(dapp3[0] - np.sum((f[0, :3] - f[1, :3]) ** 2)) < 1e-13
    assert abs(c[0] - dgeo[0] - dapp[0]) < 1e-12


# --------------------------------------------------------------------------
# Greedy disjoint pairs: characterisation, exhaustive tiny graphs
# --------------------------------------------------------------------------
def _is_greedy(ei, ej, cost, M):
    """A set M is the greedy matching under key (cost, i, j) iff it is a
    matching and every other edge touches an M-edge with a smaller key."""
    key = {(int(i), int(j)): (float(c), int(i), int(j)) for i, j, c in zip(ei, ej, cost)
           if np.isfinite(c)}
    Ms = {tuple(map(int, p)) for p in M}
    ends = [v for p in Ms for v in p]
    if len(ends) != len(set(ends)):
        return False
    owner = {}
    for p in Ms:
        owner[p[0]] = owner[p[1]] = key[p]
    for e, ke in key.items():
        if e in Ms:
            continue
        blockers = [owner[v] for v in e if v in owner]
        if not blockers or min(blockers) > ke:
            return False
    return True


def test_greedy_exhaustive_small_graphs():
    rng = np.random.default_rng(10)
    for trial in range(400):
        n = int(rng.integers(2, 7))
        all_e = [(i, j) for i in range(n) for j in range(i + 1, n)]
        m = int(rng.integers(1, min(len(all_e), 8) + 1))
        es = [all_e[t] for t in rng.choice(len(all_e), m, replace=False)]
        ei = np.array([e[0] for e in es])
        ej = np.array([e[1] for e in es])
        cost = rng.integers(0, 3, m).astype(float)  # many ties
        if trial % 5 == 0:
            cost[rng.integers(0, m)] = np.nan
        if trial % 7 == 0:
            cost[cost == 0] = -0.0
        full = O.greedy_pairs(ei, ej, cost, n, n)
        assert _is_greedy(ei, ej, cost, full)
        # brute force over every subset: exactly one is greedy
        cnt = 0
        for r in range(len(es) + 1):
            for sub in itertools.combinations(range(m), r):
                if any(not np.isfinite(cost[t]) for t in sub):
                    continue
                if _is_greedy(ei, ej, cost, [(ei[t], ej[t]) for t in sub]):
                    cnt += 1
                    assert {(int(ei[t]), int(ej[t])) for t in sub} == \
                        {tuple(map(int, p)) for p in full}
        assert cnt == 1
        # a budget keeps the smallest keys of the full matching
        for P in range(0, len(full) + 1):
            sub = O.greedy_pairs(ei, ej, cost, n, P)
            assert [tuple(p) for p in sub] == [tuple(p) for p in full[:P]]


def _ld_matching(ei, ej, cost, n):
    """Locally-dominant matching: repeatedly match edges that are the
    minimum (by key) at both endpoints among live edges."""
    live = [(float(c), int(i), int(j)) for i, j, c in zip(ei, ej, cost) if np.isfinite(c)]
    matched = set()
    M = []
    while live:
        best = {}
        for k in live:
            for v in k[1:]:
                if v not in best or k < best[v]:
                    best[v] = k
        new = [k for k in live if best[k[1]] == k and best[k[2]] == k]
        for k in new:
            M.append(k)
            matched.update(k[1:])
        live = [k for k in live if k[1] not in matched and k[2] not in matched]
    return sorted(M)


def test_greedy_equals_locally_dominant_matching():
    sc = gen_scene(3000, 12)
    st = O.activate(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh)
    nbr = O.knn(st.mu, 16)
    ei, ej = O.union_edges(nbr)
    cost = O.edge_costs(st, ei, ej, O.crn_block(0, 0, 1))[0]
    full = O.greedy_pairs(ei, ej, cost, st.n, st.n)
    ld = _ld_matching(ei, ej, cost, st.n)
    assert sorted((int(a), int(b)) for a, b in full) == sorted((k[1], k[2]) for k in ld)
    assert _is_greedy(ei, ej, cost, full)
    # greedy covers most vertices on these scenes
    assert 2 * len(full) > 0.9 * st.n


# --------------------------------------------------------------------------
# The loop
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,ratio,k", [(2000, 0.1, 16), (1500, 0.5, 8), (300, 0.01, 24)])
def test_simplify_loop_invariants(n, ratio, k):
    sc = gen_scene(n, 13)
    tgt = max(int(math.ceil(ratio * n)), 1)
    trace = []
    st = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, tgt, k, trace=trace)
    assert st.n == tgt
    assert len(trace) >= math.ceil(math.log2(n / tgt))
    N = n
    for pairs in trace:
        assert len(pairs) <= min(N - tgt, N // 2)
        assert len(np.unique(pairs)) == 2 * len(pairs)
        N -= len(pairs)
    assert N == tgt
    # every input splat ends in exactly one output cluster
    assert len(np.unique(st.origin)) == tgt
    assert np.all((st.alpha >= 0) & (st.alpha <= 1))


def test_simplify_degenerate_sizes():
    sc = gen_scene(2, 14)
    st = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, 1, 16)
    assert st.n == 1
    st = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, 5, 16)
    assert st.n == 2  # target >= n: nothing to do


def test_opacity_prune():
    st = _state(np.zeros((5, 3)), np.ones((5, 3)), [[1, 0, 0, 0]] * 5,
                [0.001, 0.002, 0.5, 0.9, 0.003])
    out = O.opacity_prune(st, 0.002)  # tau below the median
    np.testing.assert_array_equal(out.origin, [1, 2, 3, 4])
    out = O.opacity_prune(st, 0.9)  # median 0.003 < tau
    np.testing.assert_array_equal(out.origin, [2, 3, 4])
    st.alpha = np.array([0.1, 0.2, 0.3, 0.4])
    st.mu, st.s, st.q, st.f, st.origin = (x[:4] for x in (st.mu, st.s, st.q, st.f, st.origin))
    out = O.opacity_prune(st, 1.0)  # even N: median 0.25
    np.testing.assert_array_equal(out.origin, [2, 3])


def test_merge_pairs_slots_order_and_provenance():
    """Hand-worked MergePairs case (Algorithm 1; the merged splat's slot is a
    reading): six isotropic splats on the x axis, s = 0.1, pairs given as
    (4, 1) and (5, 2).  The merged splats take slots 1 and 2 (the lower
    index of each pair), splat 3 keeps its place after them, provenance is
    the smaller origin."""
    n = 6
    mu = np.zeros((n, 3))
    mu[:, 0] = np.arange(n)
    s = np.full((n, 3), 0.1)
    q = np.tile([1.0, 0, 0, 0], (n, 1))
    alpha = np.array([0.5, 0.5, 0.2, 0.5, 0.5, 0.8])
    f = np.zeros((n, 48))
    f[:, 0] = np.arange(n)
    st = O.State(mu, s, q, alpha, f, np.array([10, 7, 3, 8, 2, 9]))
    out = O.merge_pairs(st, np.array([[4, 1], [5, 2]]))
    assert out.n == 4
    # equal masses (1, 4): pi = 1/2; masses 0.2 : 0.8 (2, 5): pi = 1/5
    np.testing.assert_allclose(out.mu[:, 0], [0.0, 2.5, 0.2 * 2 + 0.8 * 5, 3.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(out.mu[:, 1:], 0.0, atol=0)
    np.testing.assert_allclose(out.f[:, 0], [0.0, 2.5, 4.4, 3.0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(out.alpha, [0.5, 0.75, 1 - 0.8 * 0.2, 0.5], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(out.origin, [10, 2, 3, 8])
    # Sigma_m = 0.01 I + pi (1 - pi) d d^T with d = (-3, 0, 0)
    Sm = O.covariance(out.s, out.q)
    for row, dxx in ((1, 0.25 * 9), (2, 0.16 * 9)):
        np.testing.assert_allclose(Sm[row], np.diag([0.01 + dxx, 0.01, 0.01]), rtol=0, atol=1e-13)
        np.testing.assert_allclose(out.s[row], [math.sqrt(0.01 + dxx), 0.1, 0.1], rtol=1e-12)
    # untouched splats are copied bit for bit
    np.testing.assert_array_equal(out.s[[0, 3]], s[[0, 3]])
    np.testing.assert_array_equal(out.q[[0, 3]], q[[0, 3]])


def test_simplify_with_prefilter_is_prune_then_loop():
    """Algorithm 1 order: the target is fixed first, the opacity filter runs
    before the loop, and the loop then sees only the survivors."""
    sc = gen_scene(1200, 15)
    tau = 0.3
    st0 = O.activate(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh)
    kept = O.opacity_prune(st0, tau).origin
    med = float(np.median(st0.alpha))
    assert np.array_equal(kept, np.nonzero(st0.alpha >= min(tau, med))[0])
    a = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, 200, 16, tau=tau)
    b = O.simplify(sc.pos[kept], sc.log_scale[kept], sc.rot[kept], sc.opacity[kept],
                   sc.sh[kept], 200, 16)
    assert a.n == b.n == 200
    np.testing.assert_array_equal(a.origin, kept[b.origin])
    np.testing.assert_array_equal(a.mu, b.mu)


def test_merge_parents_hand_case_and_hierarchy():
    """Parents of the hand-worked MergePairs case, and the hierarchy of a
    small loop: every level's parents map it onto the next level, each
    merged splat has exactly the two children the pass merged."""
    par = O.merge_parents(6, np.array([[4, 1], [5, 2]]))
    np.testing.assert_array_equal(par, [0, 1, 2, 3, 1, 2])
    sc = gen_scene(800, 16)
    lod, trace = [], []
    st = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, 100, 16, lod=lod,
                    trace=trace)
    sizes = [lv.n for lv, _ in lod] + [st.n]
    assert sizes[0] == 800 and sizes[-1] == 100
    for r, (lv, par) in enumerate(lod):
        assert par.shape == (lv.n,) and par.min() == 0 and par.max() == sizes[r + 1] - 1
        cnt = np.bincount(par, minlength=sizes[r + 1])
        assert set(cnt.tolist()) <= {1, 2}
        two = np.nonzero(cnt == 2)[0]
        got = sorted(tuple(sorted(lv.origin[par == p].tolist())) for p in two)
        assert got == sorted(map(tuple, trace[r].tolist()))


def test_cost_stratified_unbiased_symmetric_and_zero():
    """Component-stratified estimator: its mean is the KL (1-D quadrature on
    equal covariances, many draws), it is exactly symmetric in the pair, and
    it is exactly zero for an identical pair (p~ = q_m at every point)."""
    rng = np.random.default_rng(11)
    s = np.array([0.05, 0.02, 0.01])
    q = _rand_quat(rng, 1)[0]
    L = np.linalg.cholesky(O.covariance(s, q))
    for pi, delta in ((0.3, 3.32), (0.5, 1.0), (0.8, 5.0)):
        d = L @ np.array([delta, 0.0, 0.0])
        st = _state([[0, 0, 0], d], [s, s], [q, q], [pi, 1 - pi])
        crn = _iid_crn(rng, 1 << 16)
        _, dg, _ = O.edge_costs(st, [0], [1], crn, mode=O.COST_MC_STRAT)
        _, dg2, _ = O.edge_costs(st, [1], [0], crn, mode=O.COST_MC_STRAT)
        kl = _kl_1d(pi, delta)
        assert abs(dg[0] - kl) < 0.006 + 0.01 * kl, (pi, delta, dg[0], kl)
        assert dg[0] == dg2[0]
    st = _state([[0, 0, 0], [0, 0, 0]], [s, s], [q, q], [0.4, 0.7])
    _, dg, _ = O.edge_costs(st, [0], [1], _iid_crn(rng, 64), mode=O.COST_MC_STRAT)
    assert abs(dg[0]) < 1e-12


def test_cost_bound_hand_closed_form_and_bound():
    """Closed-form bound on equal isotropic covariances sigma^2 I, centres
    delta apart along x (merged covariance sigma^2 I + c delta^2 e1 e1^T,
    c = pi (1 - pi)), derived by hand; it is >= the true KL (1-D quadrature)
    and zero for an identical pair or a massless partner."""
    sig = 0.03
    for pi, delta in ((0.3, 0.05), (0.5, 0.02), (0.8, 0.09)):
        st = _state([[0, 0, 0], [delta, 0, 0]], np.full((2, 3), sig), [[1, 0, 0, 0]] * 2,
                    [pi, 1 - pi])
        _, dg, _ = O.edge_costs(st, [0], [1], np.zeros((1, 4), np.float32), mode=O.COST_BOUND)
        v = sig ** 2 + pi * (1 - pi) * delta ** 2

        def kl_to_m(w_other):
            return 0.5 * (sig ** 2 / v + 2 + w_other ** 2 * delta ** 2 / v - 3
                          + math.log(v / sig ** 2))
        hand = pi * kl_to_m(1 - pi) + (1 - pi) * kl_to_m(pi)
        assert abs(dg[0] - hand) < 1e-12 * max(1.0, hand), (dg[0], hand)
        assert dg[0] >= _kl_1d(pi, delta / sig) - 1e-9
    st = _state([[0.1, 0.2, 0.3]] * 2, [[0.01, 0.02, 0.03]] * 2, [[0.5, 0.5, 0.5, 0.5]] * 2,
                [0.3, 0.9])
    _, dg, _ = O.edge_costs(st, [0], [1], np.zeros((1, 4), np.float32), mode=O.COST_BOUND)
    assert abs(dg[0]) < 1e-12
    st = _state([[0, 0, 0], [0.05, 0, 0]], [[0.01, 0.02, 0.03]] * 2, [[1, 0, 0, 0]] * 2,
                [0.5, 0.0])
    _, dg, _ = O.edge_costs(st, [0], [1], np.zeros((1, 4), np.float32), mode=O.COST_BOUND)
    assert abs(dg[0]) < 1e-12


def _brute_knn(c, k, rows, among=None):
    """The definition: sort every other allowed row by (d^2, index)."""
    c = np.asarray(c, dtype=np.float64)
    among = np.arange(c.shape[0]) if among is None else np.asarray(among)
    out = []
    for i in rows:
        cand = [j for j in among if j != i]
        d = [((c[i, 0] - c[j, 0]) ** 2 + (c[i, 1] - c[j, 1]) ** 2) + (c[i, 2] - c[j, 2]) ** 2
             for j in cand]
        order = sorted(range(len(cand)), key=lambda t: (d[t], cand[t]))
        out.append([cand[t] for t in order[:k]])
    return np.array(out, dtype=np.int64).reshape(len(rows), k)


def test_local_refresh_dirty_rows_exact_clean_rows_unchanged_neighbourhood():
    """Dirty rows (formed by a merge, or with a merged splat in their last
    list) get the exact kNN of the new set; every other row's list equals
    the exact kNN among the rows no merge touched (its old neighbours did not
    move and nothing else among those rows came closer)."""
    rng = np.random.default_rng(5)
    n, k = 240, 6
    sc = gen_scene(n, 17, n_planes=2, n_spheres=1)
    st = O.activate(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh)
    prev = O.knn(st.mu, k)
    # a few disjoint pairs among mutual neighbours
    pairs, used = [], set()
    for i in rng.permutation(n):
        j = int(prev[i, 0])
        if i not in used and j not in used and i < j:
            pairs.append((i, j))
            used |= {i, j}
        if len(pairs) == 12:
            break
    pairs = np.array(pairs)
    parent = O.merge_parents(n, pairs)
    new = O.merge_pairs(st, pairs)
    nbr, dirty = O.local_refresh(new.mu, k, prev, parent)
    merged_new = {int(parent[a]) for a, _ in pairs}
    merged_old = set(pairs.ravel().tolist())
    # dirty set by its definition, old list by old list
    want = set(merged_new)
    for o in range(n):
        if o not in merged_old and any(int(e) in merged_old for e in prev[o]):
            want.add(int(parent[o]))
    assert set(np.nonzero(dirty)[0].tolist()) == want
    rows = sorted(want)
    np.testing.assert_array_equal(nbr[rows], _brute_knn(new.mu, k, rows))
    untouched = [v for v in range(new.n) if v not in merged_new]
    clean = [v for v in range(new.n) if v not in want]
    assert clean
    np.testing.assert_array_equal(nbr[clean], _brute_knn(new.mu, k, clean, among=untouched))


def test_local_refresh_misses_a_closer_merged_splat():
    """Hand case: A's only neighbour B (at distance 2) did not merge, so A
    keeps it, although the merge of C and D (each 2.1 away) formed a splat
    1.48 away that a full rebuild finds."""
    mu_old = np.array([[0, 0, 0], [2, 0, 0], [-2.1, 0, 0], [0, 2.1, 0]], float)  # A B C D
    prev = _brute_knn(mu_old, 1, range(4))
    assert prev[0, 0] == 1
    parent = O.merge_parents(4, np.array([[2, 3]]))  # C, D -> new index 2
    mu_new = np.array([[0, 0, 0], [2, 0, 0], [-1.05, 1.05, 0]], float)
    nbr, dirty = O.local_refresh(mu_new, 1, prev, parent)
    assert dirty.tolist() == [False, False, True]  # B's neighbour A did not merge either
    assert nbr[0, 0] == 1                      # kept
    assert O.knn(mu_new, 1)[0, 0] == 2         # full rebuild
    np.testing.assert_array_equal(nbr[2], _brute_knn(mu_new, 1, [2])[0])


def test_pass_budget_hand_values():
    assert O.pass_budget(100, 10) == 90
    assert O.pass_budget(100, 10, 0.1) == 10
    assert O.pass_budget(100, 10, 0.001) == 1
    assert O.pass_budget(100, 10, 0.95) == 90
    assert O.pass_budget(1000, 999, 0.25) == 1


def test_simplify_local_refresh_progressive():
    """With a per-pass cap the loop takes several passes; the local refresh
    queries every row in the first pass and fewer later, and reaches the
    target exactly."""
    sc = gen_scene(3000, 23)
    q_local, q_full = [], []
    a = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, 1500, 8, refresh="local",
                   pass_frac=0.05, requeried=q_local)
    b = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, 1500, 8, refresh="full",
                   pass_frac=0.05, requeried=q_full)
    assert a.n == b.n == 1500
    assert len(q_local) == len(q_full) >= 10
    assert q_local[0] == q_full[0] == 3000
    assert all(ql < qf for ql, qf in zip(q_local[1:], q_full[1:]))
    # the first pass is identical
    assert np.sum(q_full) > 1.5 * np.sum(q_local)
