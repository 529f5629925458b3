"""Coarse-to-fine hierarchy of the loop: every pass's set, and the parent
map from each level to the next.  Checked against the loop's own result
(bit for bit), the provenance trace, the mass-preserved moment matching of
each merged splat's two children (teacher-forced on the GPU's own level) and
the oracle's hierarchy sizes."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2603_16103_amd.synth import gen_scene

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _act(g):
    """Stored-form level -> float64 activated state (the oracle's activation)."""
    pos, ls, rot, op, sh = (x.cpu().numpy() for x in (g.pos, g.log_scale, g.rot, g.opacity, g.sh))
    return O.activate(pos, ls, rot, op, sh)


@pytest.mark.parametrize("n,target", [(20000, 10000), (4000, 400)])
def test_lod_hierarchy(gpu_lib, n, target):
    import torch
    ng = gpu_lib
    sc = gen_scene(n, 70)
    g = ng.GaussianTensors.from_scene(sc)
    trace = torch.full((n, 2), -1, dtype=torch.int32, device="cuda")
    origin = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    res, levels, parents, stats = ng.simplify_lod(
        g, target, k=16, opts=ng.options(d_trace=trace, d_origin=origin))
    plain = ng.simplify(g, target, k=16)
    for a, b in zip(res.numpy(), plain.numpy()):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert len(levels) == stats["rounds"]
    assert [lv.n for lv in levels] == stats["n_per_round"][:stats["rounds"]]
    # level 0 is the input
    l0 = levels[0].numpy()
    np.testing.assert_array_equal(l0[0], sc.pos)
    np.testing.assert_array_equal(l0[4], sc.sh)
    # parents, provenance and merged values, level by level
    tr = trace.cpu().numpy()
    org = np.arange(n)
    off = 0
    sizes = [lv.n for lv in levels] + [res.n]
    for r, (lv, par_t) in enumerate(zip(levels, parents)):
        par = par_t.cpu().numpy()
        cnt = np.bincount(par, minlength=sizes[r + 1])
        assert par.min() >= 0 and par.max() < sizes[r + 1] and set(cnt.tolist()) <= {1, 2}
        two = np.nonzero(cnt == 2)[0]
        pairs_r = tr[off:off + stats["pairs_per_round"][r]]
        off += len(pairs_r)
        kids = [np.nonzero(par == p)[0] for p in two]
        got = sorted((int(org[a]), int(org[b])) for a, b in kids)
        assert got == sorted(map(tuple, pairs_r.tolist()))
        nxt = np.full(sizes[r + 1], n, np.int64)
        np.minimum.at(nxt, par, org)
        # merged splats = MPMM of their two children (teacher-forced)
        st = _act(lv)
        up = _act(levels[r + 1]) if r + 1 < len(levels) else _act(res)
        ka = np.array([k[0] for k in kids])
        kb = np.array([k[1] for k in kids])
        mu_r, S_r, al_r, f_r = O.mpmm(st.mu[ka], st.s[ka], st.q[ka], st.alpha[ka], st.f[ka],
                                      st.mu[kb], st.s[kb], st.q[kb], st.alpha[kb], st.f[kb])
        e_mu = np.max(np.abs(up.mu[two] - mu_r) / np.maximum(np.abs(mu_r).max(1, keepdims=True), 1))
        S_g = O.covariance(up.s[two], up.q[two])
        e_s = np.max(np.linalg.norm(S_g - S_r, axis=(1, 2)) / np.linalg.norm(S_r, axis=(1, 2)))
        e_a = np.max(np.abs(up.alpha[two] - al_r))
        e_f = np.max(np.linalg.norm(up.f[two] - f_r, axis=1)
                     / np.maximum(np.linalg.norm(f_r, axis=1), 1e-3))
        log("level", r, "size", lv.n, "merged", two.size, "errors", e_mu, e_s, e_a, e_f)
        assert e_mu < 1.01e-5 and e_s < 1e-5 and e_a < 1e-5 and e_f < 1e-5
        # lone splats pass through unchanged
        one = np.nonzero(cnt == 1)[0]
        src = np.array([np.nonzero(par == p)[0][0] for p in one[:2000]])
        nl = levels[r + 1].numpy() if r + 1 < len(levels) else res.numpy()
        np.testing.assert_array_equal(nl[0][one[:2000]], lv.numpy()[0][src])
        org = nxt
    np.testing.assert_array_equal(np.sort(org), np.sort(origin.cpu().numpy()[:res.n]))
    # the oracle's hierarchy has the same sizes
    lod = []
    ref = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, target, 16, lod=lod)
    assert [lv.n for lv, _ in lod] == [lv.n for lv in levels] and ref.n == res.n
