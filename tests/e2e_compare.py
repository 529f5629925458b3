"""End-to-end comparison of a GPU simplification with the FP64 oracle's.

Raw indices shift after the first merge that differs, so merges are matched
by provenance: a merge is the pair (smaller origin, larger origin) of the two
clusters it joins, and a final cluster is identified by its full membership
(the input splats it absorbed), rebuilt from the merges.  Clusters whose
membership is identical on both sides are compared field by field in the
standard 3DGS form: centre, covariance (from scale and rotation), opacity and
SH coefficients.
"""
import numpy as np

import oracle as O

# Bars on the clusters of identical membership.  Centres, opacities and SH
# are compared at the teacher-forced bar.  The covariance is not: the GPU
# keeps the standard float32 parameterisation between passes, so a centre
# carries a rounding of up to half an ulp of |mu| (3e-7 at |mu| = 10), and a
# later merge's dispersion term d d^T inherits it relative to |d| (about
# 0.05 between neighbours): about 1e-5 of Sigma after a few passes.  Scales
# then carry it into the masses, so into the weights of f.  Those two are
# held to 2e-4.
E2E_BARS = {"mu": 1e-5, "alpha": 1e-5, "sigma": 2e-4, "f": 2e-4}


def pair_identity(pairs_per_round, gpu_trace, ref_trace):
    """Fraction of the oracle's merges (summed over passes) that the GPU made
    in the same pass, and the per-pass fractions."""
    off = same = total = 0
    per = []
    for r, cnt in enumerate(pairs_per_round):
        got = {tuple(x) for x in gpu_trace[off:off + cnt].tolist()}
        off += cnt
        exp = {tuple(x) for x in ref_trace[r].tolist()} if r < len(ref_trace) else set()
        same += len(got & exp)
        total += len(exp)
        per.append(len(got & exp) / max(len(exp), 1))
    return same / max(total, 1), per


def _roots(n, merges):
    """Root (smallest member) of every input splat after the merges, each
    given as (smaller origin, larger origin) of the two clusters joined."""
    parent = np.arange(n, dtype=np.int64)
    for m in merges:
        m = np.asarray(m, dtype=np.int64).reshape(-1, 2)
        parent[m[:, 1]] = m[:, 0]
    while True:
        nxt = parent[parent]
        if np.array_equal(nxt, parent):
            return parent
        parent = nxt


def _signature(n, roots):
    """(root -> member count, member-hash sum) of every cluster."""
    x = np.arange(n, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        x = x ^ (x >> np.uint64(31))
    order = np.argsort(roots, kind="stable")
    r = roots[order]
    starts = np.r_[0, np.nonzero(np.diff(r))[0] + 1]
    cnt = np.diff(np.r_[starts, r.size])
    with np.errstate(over="ignore"):
        hs = np.add.reduceat(x[order], starts)
    return {int(k): (int(c), int(h)) for k, c, h in zip(r[starts], cnt, hs)}


def compare_clusters(n, gpu_out, gpu_origin, gpu_merges, ref, ref_merges):
    """Field errors on the clusters with identical membership.

    gpu_out: stored-form arrays (pos, log_scale, rot, opacity, sh) of the GPU
    result, gpu_origin its provenance per row; ref: the oracle's final State.
    Returns a dict of the identical fraction and max / p99 errors."""
    gs = _signature(n, _roots(n, gpu_merges))
    rs = _signature(n, _roots(n, ref_merges))
    g_row = {int(o): i for i, o in enumerate(np.asarray(gpu_origin).tolist())}
    r_row = {int(o): i for i, o in enumerate(np.asarray(ref.origin).tolist())}
    same = [o for o in r_row if o in g_row and gs.get(o) == rs.get(o)]
    gi = np.array([g_row[o] for o in same], dtype=np.int64)
    ri = np.array([r_row[o] for o in same], dtype=np.int64)
    pos, ls, rot, op, sh = (np.asarray(a, dtype=np.float64) for a in gpu_out)
    out = {"identical_clusters": len(same) / max(len(r_row), 1), "clusters": len(r_row)}
    if len(same) == 0:
        return out
    mu_r = ref.mu[ri]
    e_mu = np.abs(pos[gi] - mu_r).max(1) / np.maximum(np.abs(mu_r).max(1), 1.0)
    s_g = np.exp(ls[gi])
    q_g = rot[gi] / np.linalg.norm(rot[gi], axis=1, keepdims=True)
    Sg = O.covariance(s_g, q_g)
    Sr = O.covariance(ref.s[ri], ref.q[ri])
    e_sig = np.linalg.norm(Sg - Sr, axis=(1, 2)) / np.linalg.norm(Sr, axis=(1, 2))
    a_g = 1.0 / (1.0 + np.exp(-op[gi]))
    e_al = np.abs(a_g - ref.alpha[ri])
    f_r = ref.f[ri]
    e_f = np.linalg.norm(sh[gi] - f_r, axis=1) / np.maximum(np.linalg.norm(f_r, axis=1), 1e-3)
    for name, e in (("mu", e_mu), ("sigma", e_sig), ("alpha", e_al), ("f", e_f)):
        out[name + "_max"] = float(e.max())
        out[name + "_p99"] = float(np.percentile(e, 99))
    return out


def gpu_merges(pairs_per_round, gpu_trace):
    """The GPU trace split into passes."""
    out, off = [], 0
    for cnt in pairs_per_round:
        out.append(gpu_trace[off:off + cnt])
        off += cnt
    return out


def compare_by_origin(gpu_out, gpu_origin, ref):
    """Final outputs matched by provenance (no merge trace needed): for every
    oracle output splat whose origin also names a GPU output splat, the
    per-field errors of that pair.  Returns the fraction of oracle splats
    matched and the fraction of matched pairs within E2E_BARS on every
    field."""
    pos, ls, rot, op, sh = (np.asarray(a, dtype=np.float64) for a in gpu_out)
    g_row = {int(o): i for i, o in enumerate(np.asarray(gpu_origin).tolist())}
    ri = np.array([i for i, o in enumerate(ref.origin.tolist()) if int(o) in g_row], np.int64)
    gi = np.array([g_row[int(ref.origin[i])] for i in ri], np.int64)
    out = {"matched": ri.size / max(ref.n, 1)}
    if ri.size == 0:
        out["within"] = 0.0
        return out
    mu_r = ref.mu[ri]
    e_mu = np.abs(pos[gi] - mu_r).max(1) / np.maximum(np.abs(mu_r).max(1), 1.0)
    q_g = rot[gi] / np.linalg.norm(rot[gi], axis=1, keepdims=True)
    Sg = O.covariance(np.exp(ls[gi]), q_g)
    Sr = O.covariance(ref.s[ri], ref.q[ri])
    e_sig = np.linalg.norm(Sg - Sr, axis=(1, 2)) / np.linalg.norm(Sr, axis=(1, 2))
    e_al = np.abs(1.0 / (1.0 + np.exp(-op[gi])) - ref.alpha[ri])
    f_r = ref.f[ri]
    e_f = np.linalg.norm(sh[gi] - f_r, axis=1) / np.maximum(np.linalg.norm(f_r, axis=1), 1e-3)
    ok = ((e_mu < E2E_BARS["mu"]) & (e_sig < E2E_BARS["sigma"]) & (e_al < E2E_BARS["alpha"])
          & (e_f < E2E_BARS["f"]))
    out["within"] = float(np.mean(ok))
    return out


def compare_by_position(gpu_out, ref):
    """Final outputs matched by centre (for results that carry no
    provenance): the fraction of oracle splats whose nearest GPU centre lies
    within the centre bar and whose covariance, opacity and SH there are
    within their bars."""
    from scipy.spatial import cKDTree
    pos, ls, rot, op, sh = (np.asarray(a, dtype=np.float64) for a in gpu_out)
    d, gi = cKDTree(pos).query(ref.mu, k=1)
    e_mu = d / np.maximum(np.abs(ref.mu).max(1), 1.0)
    q_g = rot[gi] / np.linalg.norm(rot[gi], axis=1, keepdims=True)
    Sg = O.covariance(np.exp(ls[gi]), q_g)
    Sr = O.covariance(ref.s, ref.q)
    e_sig = np.linalg.norm(Sg - Sr, axis=(1, 2)) / np.linalg.norm(Sr, axis=(1, 2))
    e_al = np.abs(1.0 / (1.0 + np.exp(-op[gi])) - ref.alpha)
    e_f = np.linalg.norm(sh[gi] - ref.f, axis=1) / np.maximum(np.linalg.norm(ref.f, axis=1), 1e-3)
    ok = ((e_mu < E2E_BARS["mu"]) & (e_sig < E2E_BARS["sigma"]) & (e_al < E2E_BARS["alpha"])
          & (e_f < E2E_BARS["f"]))
    return {"within": float(np.mean(ok)), "n_gpu": int(pos.shape[0]), "n_ref": int(ref.n)}
