"""Plain FP64 reference of the NanoGS simplification loop.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Slow on purpose:
every step is the paper's definition written out with numpy in float64,
with no blocking, fusion or reordering beyond what the definition states.

Paper: Xiong et al., "NanoGS: Training-Free Gaussian Splat Simplification"
(arXiv 2603.16103).  Section / equation / algorithm references below are to
that paper.  Readings of passages the paper leaves open are marked READING
and listed in the design notes of the repository.

Parity status per function (what pins each one is in the CPU test suite):
  crn_block         pinned (published SplitMix64 vectors, Box-Muller moments)
  activate          pinned (round trip, closed forms)
  knn               pinned (integer-lattice closed form, KD-tree library)
  union_edges       pinned (edge-count identity)
  edge_costs        pinned (zero cases, 1-D reduction, entropy identity,
                    convexity bound, affine invariance)
  greedy_pairs      pinned (exhaustive small cases, locally-dominant match)
  mpmm/merge_pairs  pinned (moment preservation, identical-copy closed form)
  scale_rot_from_cov pinned (round trip, orthonormality)
  simplify          pinned (loop invariants: exact final count, round bound)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Common random numbers (Appendix A: one shared set of draws per pass)
# ---------------------------------------------------------------------------
_MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(x: int) -> int:
    """First output of Steele-Lea-Flood SplitMix64 seeded with ``x``.

    READING: the paper shares common random numbers across candidate pairs
    (Appendix A) but names no generator; we key them with this published
    64-bit mixer."""
    z = (x + _GAMMA) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def _uniform(seed: int, round_idx: int, s: int, c: int) -> float:
    h = splitmix64(splitmix64(splitmix64(seed & _MASK64) ^ (round_idx & _MASK64))
                   ^ ((8 * s + c) & _MASK64))
    return (h >> 11) * (2.0 ** -53)


def crn_block(seed: int, round_idx: int, S: int) -> np.ndarray:
    """The S shared draws (u, z0, z1, z2) of one pass, float32 [S, 4].

    u ~ U[0,1) picks the mixture component; z ~ N(0, I3) by Box-Muller on
    (1-U) so the logarithm stays finite.  Computed in float64, stored as
    float32: both implementations consume these exact float32 values."""
    out = np.empty((S, 4), dtype=np.float32)
    two_pi = 2.0 * math.pi
    for s in range(S):
        u = _uniform(seed, round_idx, s, 0)
        u1 = _uniform(seed, round_idx, s, 1)
        u2 = _uniform(seed, round_idx, s, 2)
        u3 = _uniform(seed, round_idx, s, 3)
        u4 = _uniform(seed, round_idx, s, 4)
        r1 = math.sqrt(-2.0 * math.log(1.0 - u1))
        r2 = math.sqrt(-2.0 * math.log(1.0 - u3))
        out[s, 0] = u
        out[s, 1] = r1 * math.cos(two_pi * u2)
        out[s, 2] = r1 * math.sin(two_pi * u2)
        out[s, 3] = r2 * math.cos(two_pi * u4)
    return out


# ---------------------------------------------------------------------------
# Splat parameterisation (standard 3DGS form kept by the method, Sec. 1/4)
# ---------------------------------------------------------------------------
@dataclass
class State:
    """Activated splats in float64: centre mu, std-dev scales s, unit
    quaternion q = (w, x, y, z), opacity alpha, appearance f, provenance."""

    mu: np.ndarray
    s: np.ndarray
    q: np.ndarray
    alpha: np.ndarray
    f: np.ndarray
    origin: np.ndarray = field(default=None)

    @property
    def n(self) -> int:
        return int(self.mu.shape[0])


def activate(pos, log_scale, rot, opacity, sh) -> State:
    """Stored 3DGS form -> activated form (READING: the boundary carries the
    stored form; s = exp(log-scale), alpha = sigmoid(logit), q normalised,
    zero quaternion -> identity)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    s = np.exp(np.asarray(log_scale, dtype=np.float64))
    o = np.asarray(opacity, dtype=np.float64)
    alpha = 1.0 / (1.0 + np.exp(-o))
    r = np.asarray(rot, dtype=np.float64)
    nr = np.linalg.norm(r, axis=1, keepdims=True)
    q = np.where(nr > 0, r / np.where(nr > 0, nr, 1.0), np.array([1.0, 0, 0, 0]))
    f = np.asarray(sh, dtype=np.float64)
    return State(pos.copy(), s, q, alpha, f.copy(), np.arange(n, dtype=np.int64))


def rotation_matrix(q: np.ndarray) -> np.ndarray:
    """R(q) for unit q = (w, x, y, z): the rotation used by 3DGS."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def covariance(s: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Sigma = R diag(s^2) R^T (READING: s are standard deviations, which
    is what makes the mass of Eq. (unnormalized splats) the integral of the
    splat's density)."""
    R = rotation_matrix(q)
    return R @ (np.asarray(s)[..., :, None] ** 2 * np.swapaxes(R, -1, -2))


def mass(s: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """w = (2 pi)^{3/2} alpha prod_k s_k  (Eq. vm_weights)."""
    return (2.0 * math.pi) ** 1.5 * alpha * np.prod(s, axis=-1)


# ---------------------------------------------------------------------------
# Stage 1: sparse merge graph (Sec. 3.1; Algorithm 1 KNN + union edges)
# ---------------------------------------------------------------------------
def _rank_exact(X, q, cand, keff):
    """The keff best candidates of query q under the key (d2, j)."""
    cand = cand[cand != q]
    d = X[cand] - X[q]
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    order = np.lexsort((cand, d2))
    return cand[order[:keff]]


def knn(centres: np.ndarray, k: int, queries=None, chunk: int = 256,
        method: str = "auto", workers: int = 1) -> np.ndarray:
    """Directed k nearest neighbours of each query among all centres.

    Key = (d2, j) with d2 = ((dx*dx + dy*dy) + dz*dz) in float64 of the
    centres (READING: ties go to the lower index; the point itself is
    excluded; k_eff = min(max(1,k), N-1) as in Algorithm 1).  Rows are
    padded with -1 up to k columns.

    method "brute" is the definition itself (all N distances per query).
    method "tree" only changes which points are ranked.  A KD-tree library
    query fetches each query's k_eff + 9 nearest points (itself included);
    those are ranked with the key.  Every point not fetched lies at least
    the last fetched library distance away, so the ranking is complete when
    the k_eff-th key is clearly below that distance.  Rows where it is not
    (many equal distances) gather every point within the (k_eff+1)-th
    library distance times (1 + 1e-9) and rank those instead.  Both methods
    return the same lists.  "auto" uses the tree above 4096 points.
    ``workers``: threads of the library query."""
    X = np.asarray(centres, dtype=np.float64)
    n = X.shape[0]
    keff = min(max(1, k), n - 1)
    qs = np.arange(n) if queries is None else np.asarray(queries, dtype=np.int64)
    out = np.full((qs.size, k), -1, dtype=np.int32)
    if keff <= 0:
        return out
    if method == "auto":
        method = "tree" if n > 4096 else "brute"
    if method == "tree":
        from scipy.spatial import cKDTree
        tree = cKDTree(X)
        kq = min(keff + 9, n)
        redo = []
        for c0 in range(0, qs.size, 1 << 17):
            qq = qs[c0:c0 + (1 << 17)]
            dist, idx = tree.query(X[qq], k=kq, workers=workers)
            dist = dist.reshape(qq.size, kq)
            idx = idx.reshape(qq.size, kq)
            d = X[idx] - X[qq][:, None, :]
            d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
            d2 = np.where(idx == qq[:, None], np.inf, d2)
            # key (d2, j): order by j, then stably by d2
            o = np.argsort(idx, axis=1, kind="stable")
            idx = np.take_along_axis(idx, o, 1)
            d2 = np.take_along_axis(d2, o, 1)
            o = np.argsort(d2, axis=1, kind="stable")
            idx = np.take_along_axis(idx, o, 1)
            kth = np.take_along_axis(d2, o, 1)[:, keff - 1]
            out[c0:c0 + qq.size, :keff] = idx[:, :keff]
            ok = np.full(qq.size, kq == n) | (kth * (1.0 + 1e-9) < dist[:, -1] ** 2 * (1.0 - 1e-9))
            redo.extend((c0 + np.nonzero(~ok)[0]).tolist())
        if redo:
            rows = np.asarray(redo, dtype=np.int64)
            dk, _ = tree.query(X[qs[rows]], k=keff + 1)
            dk = np.atleast_2d(dk)[:, -1] if keff + 1 > 1 else np.atleast_1d(dk)
            balls = tree.query_ball_point(X[qs[rows]], dk * (1.0 + 1e-9) + 1e-300)
            for t, r in enumerate(rows):
                out[r, :keff] = _rank_exact(X, qs[r], np.asarray(balls[t], dtype=np.int64), keff)
        return out
    for c0 in range(0, qs.size, chunk):
        qq = qs[c0:c0 + chunk]
        dx = X[qq, None, 0] - X[None, :, 0]
        dy = X[qq, None, 1] - X[None, :, 1]
        dz = X[qq, None, 2] - X[None, :, 2]
        d2 = (dx * dx + dy * dy) + dz * dz
        d2[np.arange(qq.size), qq] = np.inf
        kth = np.partition(d2, keff - 1, axis=1)[:, keff - 1]
        for r in range(qq.size):
            cand = np.nonzero(d2[r] <= kth[r])[0]
            order = np.lexsort((cand, d2[r, cand]))
            out[c0 + r, :keff] = cand[order[:keff]]
    return out


def union_edges(nbr: np.ndarray):
    """Unique undirected edges {i, j}, i < j, from the directed lists
    (Algorithm 1 UndirectedUnionEdges), in lexicographic (i, j) order."""
    nbr = np.asarray(nbr)
    n, k = nbr.shape
    i = np.repeat(np.arange(n, dtype=np.int64), k)
    j = nbr.reshape(-1).astype(np.int64)
    ok = j >= 0
    a = np.minimum(i[ok], j[ok])
    b = np.maximum(i[ok], j[ok])
    key = np.unique(a * (n + 1) + b)
    return (key // (n + 1)).astype(np.int32), (key % (n + 1)).astype(np.int32)


# ---------------------------------------------------------------------------
# Stage 2: merge cost (Eq. cost, Eq. Dgeo, Eq. norm_mixture, Eq. Dmerge,
# Appendix A Monte Carlo estimator, appearance term)
# ---------------------------------------------------------------------------
def _log_gauss_chol(x, mu, L):
    """log N(x; mu, L L^T) without the -(3/2) log(2 pi) constant, which
    cancels between the mixture term and the merged term:
    -1/2 |L^-1 (x - mu)|^2 - log det L, with L^-1 applied by forward
    substitution (L lower triangular)."""
    y = x - mu
    v0 = y[..., 0] / L[..., 0, 0]
    v1 = (y[..., 1] - L[..., 1, 0] * v0) / L[..., 1, 1]
    v2 = (y[..., 2] - L[..., 2, 0] * v0 - L[..., 2, 1] * v1) / L[..., 2, 2]
    logdet = np.log(L[..., 0, 0]) + np.log(L[..., 1, 1]) + np.log(L[..., 2, 2])
    return -0.5 * (v0 * v0 + v1 * v1 + v2 * v2) - logdet


COST_MC = 0     # Monte Carlo estimate of Appendix A (Eq. mc_kl_estimator)
COST_MC_STRAT = 1  # both components sampled with every draw (stratified)
COST_BOUND = 2  # closed-form bound pi KL(N_i||q_m) + (1-pi) KL(N_j||q_m)


def edge_costs(st: State, ei, ej, crn: np.ndarray, app_dims: int = 48,
               chunk: int = 1 << 18, workers: int = 1, mode: int = COST_MC):
    """C(i,j) = D_geo + D_app for every edge (i < j).

    D_geo = KL(p~_ij || q_m) estimated with the S shared draws (Appendix A):
    pi = w_i / (w_i + w_j) in float64 (Eq. norm_mixture, READING: pi belongs
    to the lower index); a draw (u, z) picks component i when u < pi, and
    x = mu_c + chol(Sigma_c) z (READING: Cholesky factor, so the sample does
    not depend on how (s, q) factor Sigma); then
    g = log(pi N_i(x) + (1-pi) N_j(x)) - log q_m(x), averaged over the S
    draws, with q_m = N(mu_m, Sigma_m) the moment-matched Gaussian
    (Eq. vm_cov).  D_app = ||f_i - f_j||^2 over the first ``app_dims`` SH
    coefficients.  Returns (cost, d_geo, d_app) in float64.

    ``mode`` picks the geometric term (READING: the paper defines D_geo and
    estimates it by Monte Carlo; the two other modes are cost variants built
    on the same definition):
      COST_MC     the estimate above;
      COST_MC_STRAT the same expectation without the component draw: each
                  draw z is used in both components, x_i = mu_i + L_i z
                  weighted pi and x_j = mu_j + L_j z weighted 1 - pi, so
                  D = mean_s [pi g(x_i) + (1-pi) g(x_j)] with g = log p~ -
                  log q_m; exactly symmetric in (i, j) and exactly zero for
                  an identical pair;
      COST_BOUND  joint convexity of KL in its first argument bounds the
                  mixture's divergence by pi KL(N_i || q_m) + (1-pi)
                  KL(N_j || q_m), each term the closed form of Appendix A
                  for single Gaussians; no draws.

    The covariance of a splat and its Cholesky factor are formed once per
    splat; the edges are evaluated in chunks (the cost of an edge depends on
    that edge alone).  ``workers`` is accepted for symmetry with knn and does
    not change anything."""
    a = np.asarray(ei, dtype=np.int64)
    b = np.asarray(ej, dtype=np.int64)
    if a.size == 0:
        z = np.zeros(0)
        return z, z, z
    used = np.unique(np.concatenate([a, b]))
    Sig = np.zeros((st.n, 3, 3))
    Sig[used] = covariance(st.s[used], st.q[used])
    L = np.zeros((st.n, 3, 3))
    L[used] = np.linalg.cholesky(Sig[used])
    w = np.zeros(st.n)
    w[used] = mass(st.s[used], st.alpha[used])
    parts = [_edge_costs_block(st, Sig, L, w, a[c0:c0 + chunk], b[c0:c0 + chunk], crn, app_dims,
                               mode)
             for c0 in range(0, a.size, chunk)]
    return tuple(np.concatenate([p[t] for p in parts]) for t in range(3))


def gauss_kl(mu_a, Sa, mu_b, Sb):
    """KL(N(mu_a, Sa) || N(mu_b, Sb)) in closed form (Appendix A, d = 3)."""
    d = 3
    diff = mu_b - mu_a
    sol = np.linalg.solve(Sb, np.concatenate([Sa, diff[..., None]], axis=-1))
    tr = np.trace(sol[..., :d], axis1=-2, axis2=-1)
    maha = np.sum(diff * sol[..., d], axis=-1)
    ld = np.linalg.slogdet(Sb)[1] - np.linalg.slogdet(Sa)[1]
    return 0.5 * (tr + maha - d + ld)


def _edge_costs_block(st: State, Sig, L, w, a, b, crn, app_dims, mode=COST_MC):
    """Costs of the edges (a[e], b[e]); Sig, L, w: per-splat covariance,
    its lower Cholesky factor and mass (Eq. vm_weights)."""
    Sa, Sb = Sig[a], Sig[b]
    wa, wb = w[a], w[b]
    W = wa + wb
    with np.errstate(divide="ignore", invalid="ignore"):
        pa = np.where(W > 0, wa / np.where(W > 0, W, 1.0), 0.5)
        pb = np.where(W > 0, wb / np.where(W > 0, W, 1.0), 0.5)
    mua, mub = st.mu[a], st.mu[b]
    mum = pa[:, None] * mua + pb[:, None] * mub
    da = mua - mum
    db = mub - mum
    Sm = (pa[:, None, None] * (Sa + da[:, :, None] * da[:, None, :])
          + pb[:, None, None] * (Sb + db[:, :, None] * db[:, None, :]))
    La, Lb = L[a], L[b]
    df = st.f[a, :app_dims] - st.f[b, :app_dims]
    dapp = np.sum(df * df, axis=1)
    if mode == COST_BOUND:
        with np.errstate(invalid="ignore"):
            dgeo = (np.where(pa > 0, pa * gauss_kl(mua, Sa, mum, Sm), 0.0)
                    + np.where(pb > 0, pb * gauss_kl(mub, Sb, mum, Sm), 0.0))
        return dgeo + dapp, dgeo, dapp
    Lm = np.linalg.cholesky(Sm)
    crn = np.asarray(crn, dtype=np.float32)
    S = crn.shape[0]
    with np.errstate(divide="ignore"):
        lpa = np.log(pa)
        lpb = np.log(pb)
    if mode == COST_MC_STRAT:
        z = crn[:, 1:4].astype(np.float64)

        def g(x):
            return (np.logaddexp(lpa[None] + _log_gauss_chol(x, mua[None], La[None]),
                                 lpb[None] + _log_gauss_chol(x, mub[None], Lb[None]))
                    - _log_gauss_chol(x, mum[None], Lm[None]))

        xa = mua[None] + np.einsum("eij,sj->sei", La, z)
        xb = mub[None] + np.einsum("eij,sj->sei", Lb, z)
        with np.errstate(invalid="ignore"):
            strat = (np.where(pa > 0, pa * g(xa), 0.0) + np.where(pb > 0, pb * g(xb), 0.0))
        dgeo = np.mean(strat, axis=0)
        return dgeo + dapp, dgeo, dapp
    u = crn[:, 0].astype(np.float64)[:, None]
    z = crn[:, 1:4].astype(np.float64)
    take_a = u < pa[None, :]  # pi = w_i / W in float64 (Eq. norm_mixture)
    xa = mua[None] + np.einsum("eij,sj->sei", La, z)
    xb = mub[None] + np.einsum("eij,sj->sei", Lb, z)
    x = np.where(take_a[..., None], xa, xb)
    lna = _log_gauss_chol(x, mua[None], La[None])
    lnb = _log_gauss_chol(x, mub[None], Lb[None])
    lnm = _log_gauss_chol(x, mum[None], Lm[None])
    g_sum = np.sum(np.logaddexp(lpa[None] + lna, lpb[None] + lnb) - lnm, axis=0)
    dgeo = g_sum / S
    return dgeo + dapp, dgeo, dapp


# ---------------------------------------------------------------------------
# Stage 3: greedy disjoint pairs (Sec. 3.4; Algorithm 1 GreedyDisjointPairs)
# ---------------------------------------------------------------------------
def greedy_pairs(ei, ej, cost, n: int, P: int):
    """Sort edges by increasing cost and scan, taking an edge whenever both
    endpoints are still free, until P pairs are taken.

    READING: order key (cost, i, j); -0 and +0 compare equal; edges with a
    non-finite cost are never taken.  Returns an int array [M, 2] in the
    order the scan took them."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    c = np.asarray(cost, dtype=np.float64)
    ok = np.isfinite(c)
    idx = np.nonzero(ok)[0]
    order = idx[np.lexsort((ej[idx], ei[idx], c[idx]))]
    used = bytearray(n)
    out = []
    if P <= 0:
        return np.zeros((0, 2), dtype=np.int64)
    for i, j in zip(ei[order].tolist(), ej[order].tolist()):
        if not used[i] and not used[j]:
            used[i] = used[j] = 1
            out.append((i, j))
            if len(out) >= P:
                break
    return np.array(out, dtype=np.int64).reshape(-1, 2)


# ---------------------------------------------------------------------------
# Stage 4: mass-preserved moment matching (Sec. 3.3) and the new splat set
# ---------------------------------------------------------------------------
def mpmm(mu_a, s_a, q_a, al_a, f_a, mu_b, s_b, q_b, al_b, f_b):
    """MPMM of pairs: masses (Eq. vm_weights), mass-weighted mean and
    feature, mass-matched covariance (Eq. vm_cov), opacity by the over rule
    (Eq. vm_alpha).  READING: W = 0 gives equal weights.  Returns
    (mu_m, Sigma_m, alpha_m, f_m)."""
    wa = mass(s_a, al_a)
    wb = mass(s_b, al_b)
    W = wa + wb
    with np.errstate(divide="ignore", invalid="ignore"):
        pa = np.where(W > 0, wa / np.where(W > 0, W, 1.0), 0.5)
        pb = np.where(W > 0, wb / np.where(W > 0, W, 1.0), 0.5)
    mum = pa[:, None] * mu_a + pb[:, None] * mu_b
    fm = pa[:, None] * f_a + pb[:, None] * f_b
    Sa = covariance(s_a, q_a)
    Sb = covariance(s_b, q_b)
    da = mu_a - mum
    db = mu_b - mum
    Sm = (pa[:, None, None] * (Sa + da[:, :, None] * da[:, None, :])
          + pb[:, None, None] * (Sb + db[:, :, None] * db[:, None, :]))
    am = 1.0 - (1.0 - al_a) * (1.0 - al_b)
    return mum, Sm, am, fm


def quat_from_rotation(R: np.ndarray) -> np.ndarray:
    """Unit quaternion (w, x, y, z), w >= 0, of rotation matrices, by
    Shepperd's method (branch on the largest of trace and diagonal)."""
    R = np.asarray(R, dtype=np.float64)
    t = R[..., 0, 0] + R[..., 1, 1] + R[..., 2, 2]
    cand = np.stack([t, R[..., 0, 0], R[..., 1, 1], R[..., 2, 2]], axis=-1)
    br = np.argmax(cand, axis=-1)[..., None]
    m = lambda i, j: R[..., i, j]  # noqa: E731
    with np.errstate(divide="ignore", invalid="ignore"):
        # branch 0: w largest
        w0 = 0.5 * np.sqrt(np.maximum(1.0 + t, 0.0))
        q0 = np.stack([w0, (m(2, 1) - m(1, 2)) / (4 * w0), (m(0, 2) - m(2, 0)) / (4 * w0),
                       (m(1, 0) - m(0, 1)) / (4 * w0)], -1)
        # branch 1: x largest
        x1 = 0.5 * np.sqrt(np.maximum(1.0 + m(0, 0) - m(1, 1) - m(2, 2), 0.0))
        q1 = np.stack([(m(2, 1) - m(1, 2)) / (4 * x1), x1, (m(0, 1) + m(1, 0)) / (4 * x1),
                       (m(0, 2) + m(2, 0)) / (4 * x1)], -1)
        # branch 2: y largest
        y2 = 0.5 * np.sqrt(np.maximum(1.0 - m(0, 0) + m(1, 1) - m(2, 2), 0.0))
        q2 = np.stack([(m(0, 2) - m(2, 0)) / (4 * y2), (m(0, 1) + m(1, 0)) / (4 * y2), y2,
                       (m(1, 2) + m(2, 1)) / (4 * y2)], -1)
        # branch 3: z largest
        z3 = 0.5 * np.sqrt(np.maximum(1.0 - m(0, 0) - m(1, 1) + m(2, 2), 0.0))
        q3 = np.stack([(m(1, 0) - m(0, 1)) / (4 * z3), (m(0, 2) + m(2, 0)) / (4 * z3),
                       (m(1, 2) + m(2, 1)) / (4 * z3), z3], -1)
    q = np.where(br == 0, q0, np.where(br == 1, q1, np.where(br == 2, q2, q3)))
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    q *= np.where(q[..., :1] < 0, -1.0, 1.0)
    return q


def scale_rot_from_cov(Sig: np.ndarray):
    """Covariance -> (s, q) in the 3DGS parameterisation.

    READING (the paper keeps the representation but does not say how the
    merged covariance is factored): eigenvalues in decreasing order,
    floored at 1e-12 of the largest, s = sqrt(lambda); the largest-magnitude
    component of the first two eigenvectors is made positive and the third
    is their cross product, so R has determinant +1; q from R with w >= 0."""
    Sig = np.asarray(Sig, dtype=np.float64)
    lam, V = np.linalg.eigh(Sig)
    lam = lam[..., ::-1]
    V = V[..., :, ::-1]
    top = np.maximum(lam[..., :1], 0.0)
    lam = np.maximum(lam, 1e-12 * top)
    e1 = V[..., :, 0].copy()
    e2 = V[..., :, 1].copy()
    for e in (e1, e2):
        piv = np.argmax(np.abs(e), axis=-1)
        sgn = np.where(np.take_along_axis(e, piv[..., None], -1) < 0, -1.0, 1.0)
        e *= sgn
    e3 = np.cross(e1, e2)
    R = np.stack([e1, e2, e3], axis=-1)
    return np.sqrt(lam), quat_from_rotation(R)


def merge_pairs(st: State, pairs: np.ndarray) -> State:
    """MergePairs of Algorithm 1.  READING: the merged splat takes the slot
    of the lower index, the higher index is removed and the survivors keep
    their relative order; provenance is the smaller origin."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    a = np.minimum(pairs[:, 0], pairs[:, 1])
    b = np.maximum(pairs[:, 0], pairs[:, 1])
    mum, Sm, am, fm = mpmm(st.mu[a], st.s[a], st.q[a], st.alpha[a], st.f[a],
                           st.mu[b], st.s[b], st.q[b], st.alpha[b], st.f[b])
    sm, qm = scale_rot_from_cov(Sm) if a.size else (np.zeros((0, 3)), np.zeros((0, 4)))
    mu, s, q = st.mu.copy(), st.s.copy(), st.q.copy()
    alpha, f, origin = st.alpha.copy(), st.f.copy(), st.origin.copy()
    mu[a], s[a], q[a], alpha[a], f[a] = mum, sm, qm, am, fm
    origin[a] = np.minimum(origin[a], origin[b])
    keep = np.ones(st.n, dtype=bool)
    keep[b] = False
    return State(mu[keep], s[keep], q[keep], alpha[keep], f[keep], origin[keep])


def merge_parents(n: int, pairs: np.ndarray) -> np.ndarray:
    """Index in the next set of every splat, under the MergePairs reading:
    the lower index keeps its place among the survivors (relative order
    kept), the higher index goes to the same merged splat."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    a = np.minimum(pairs[:, 0], pairs[:, 1])
    b = np.maximum(pairs[:, 0], pairs[:, 1])
    keep = np.ones(n, dtype=bool)
    keep[b] = False
    parent = np.cumsum(keep) - 1
    parent[b] = parent[a]
    return parent


def local_refresh(centres: np.ndarray, keff: int, prev_nbr: np.ndarray, parent: np.ndarray,
                  workers: int = 1):
    """Local neighbourhood refresh (Sec. 3.4): re-query the kNN only around
    the splats a pass formed.  READING: a splat of the new set is dirty when
    it was formed by a merge, or when its list of the previous pass named a
    splat that took part in a merge; a dirty splat gets its exact kNN over
    the whole new set, every other splat keeps its previous list with the
    indices carried to the new set (``parent``: new index of each old one,
    as merge_parents gives it).  Returns (nbr [n, keff], dirty mask)."""
    centres = np.asarray(centres)
    n_new = centres.shape[0]
    parent = np.asarray(parent, dtype=np.int64)
    cnt = np.bincount(parent, minlength=n_new)
    merged = cnt == 2
    # the old index of every splat that survived unmerged
    old_of = np.full(n_new, -1, dtype=np.int64)
    surv = ~merged[parent]
    old_of[parent[surv]] = np.nonzero(surv)[0]
    nbr = np.empty((n_new, keff), dtype=np.int64)
    dirty = merged.copy()
    kept = np.nonzero(~merged)[0]
    carried = parent[np.asarray(prev_nbr, dtype=np.int64)[old_of[kept]]]
    touched = merged[carried].any(axis=1)
    dirty[kept[touched]] = True
    nbr[kept[~touched]] = carried[~touched]
    rows = np.nonzero(dirty)[0]
    if rows.size:
        nbr[rows] = knn(centres, keff, queries=rows, workers=workers)
    return nbr, dirty


def pass_budget(n: int, target_n: int, pass_frac: float = 0.0) -> int:
    """P = N - N_tgt (Algorithm 1).  With pass_frac > 0 (progressive
    collapses, Sec. 3.4) a pass takes at most max(1, floor(f N)) pairs, f
    being pass_frac rounded to float32 (the option's storage type)."""
    P = n - target_n
    if pass_frac > 0.0:
        P = min(P, max(1, int(np.floor(float(np.float32(pass_frac)) * n))))
    return P


# ---------------------------------------------------------------------------
# Opacity pre-filter (Algorithm 1, before the loop)
# ---------------------------------------------------------------------------
def opacity_prune(st: State, tau: float) -> State:
    """tau' = min(tau, median(alpha)); keep splats with alpha >= tau'
    (READING: numpy's median, the mean of the two middle values for even
    N)."""
    if st.n == 0:
        return st
    t = min(tau, float(np.median(st.alpha)))
    keep = st.alpha >= t
    return State(st.mu[keep], st.s[keep], st.q[keep], st.alpha[keep], st.f[keep],
                 st.origin[keep])


# ---------------------------------------------------------------------------
# The loop (Algorithm 1) and the output form
# ---------------------------------------------------------------------------
def simplify(pos, log_scale, rot, opacity, sh, target_n: int, k: int,
             seed: int = 0, S: int = 1, app_dims: int = 48, trace=None,
             max_rounds: int = 1 << 30, workers: int = 1, tau=None, lod=None,
             cost_mode: int = COST_MC, refresh: str = "full", pass_frac: float = 0.0,
             requeried=None):
    """Algorithm 1: the opacity pre-filter when ``tau`` is given (the target
    count is the caller's, fixed before the filter), then while N > N_tgt, rebuild
    the kNN graph, take the union edges, cost them, pick at most
    P = N - N_tgt greedy disjoint pairs, stop if none, merge.  The shared
    draws of pass r are ``crn_block(seed, r, S)``.  Returns the final State
    (alpha clipped to [0, 1]).  When ``trace`` is a list, each pass appends
    the provenance pairs (origin_i, origin_j) it merged.  When ``lod`` is a
    list, each pass appends (the set at its start, merge_parents of its
    pairs): the coarse-to-fine hierarchy (Sec. 3.4).  ``refresh``: "full"
    rebuilds the kNN graph every pass (the paper's setting), "local" keeps
    the lists of the splats no merge touched (local_refresh) from the second
    pass on; ``requeried`` (list) receives the rows queried per pass.
    ``pass_frac``: per-pass pair cap (pass_budget).  ``workers``: threads
    for the per-query and per-edge steps (results do not change)."""
    st = activate(pos, log_scale, rot, opacity, sh)
    if tau is not None:
        st = opacity_prune(st, tau)
    target_n = max(int(target_n), 1)
    r = 0
    prev = None  # (lists, parent map) of the previous pass
    while st.n > target_n and r < max_rounds:
        n = st.n
        keff = min(max(1, k), n - 1)
        if refresh == "local" and prev is not None and prev[0].shape[1] == keff:
            nbr, dirty = local_refresh(st.mu, keff, prev[0], prev[1], workers=workers)
            nq = int(dirty.sum())
        else:
            nbr = knn(st.mu, keff, workers=workers)
            nq = n
        if requeried is not None:
            requeried.append(nq)
        ei, ej = union_edges(nbr)
        cost = edge_costs(st, ei, ej, crn_block(seed, r, S), app_dims, mode=cost_mode)[0]
        P = pass_budget(n, target_n, pass_frac)
        pairs = greedy_pairs(ei, ej, cost, n, P)
        if pairs.shape[0] == 0:
            break
        if trace is not None:
            trace.append(np.sort(st.origin[pairs], axis=1))
        if lod is not None:
            lod.append((State(st.mu.copy(), st.s.copy(), st.q.copy(), st.alpha.copy(),
                              st.f.copy(), st.origin.copy()), merge_parents(n, pairs)))
        prev = (nbr, merge_parents(n, pairs))
        st = merge_pairs(st, pairs)
        r += 1
    st.alpha = np.clip(st.alpha, 0.0, 1.0)
    return st


def deactivate(st: State):
    """Activated -> stored 3DGS form: log-scale, opacity logit (READING:
    alpha clamped to [2^-24, 1 - 2^-24] so the logit is finite in float32),
    unit quaternion with w >= 0, SH unchanged.  Returns float32 arrays
    (pos, log_scale, rot, opacity, sh)."""
    eps = 2.0 ** -24
    al = np.clip(st.alpha, eps, 1.0 - eps)
    q = st.q / np.linalg.norm(st.q, axis=1, keepdims=True)
    q = q * np.where(q[:, :1] < 0, -1.0, 1.0)
    f32 = np.float32
    return (st.mu.astype(f32), np.log(st.s).astype(f32), q.astype(f32),
            np.log(al / (1.0 - al)).astype(f32), st.f.astype(f32))
