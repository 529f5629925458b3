"""Continuous batching: requests replayed in real time through the batched
server must each get the same bytes as the same request simplified alone,
also when a small HBM budget makes later requests wait for admission and
join while earlier ones are running; the plain one-at-a-time server gives
the same results."""
import sys

import numpy as np
import pytest

from paper_2603_16103_amd.synth import gen_scene

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests():
    from paper_2603_16103_amd import serve
    rng = np.random.default_rng(9)
    reqs = []
    for rid in range(10):
        n = int(rng.integers(2000, 30000))
        sc = gen_scene(n, 500 + rid, n_planes=int(rng.integers(1, 6)),
                       n_spheres=int(rng.integers(0, 3)))
        ratio = float(rng.choice([0.5, 0.1, 0.01]))
        k = int(rng.choice([16, 24]))
        reqs.append(serve.Request(rid, 0.02 * rid, sc, max(int(np.ceil(ratio * n)), 1), k,
                                  seed=77 + rid))
    return reqs


def _alone(ng, req):
    res = ng.simplify(ng.GaussianTensors.from_scene(req.scene), req.target, k=req.k,
                      opts=ng.options(seed=req.seed))
    return [x.cpu().numpy() for x in (res.pos, res.log_scale, res.rot, res.opacity, res.sh)]


def _check_same(reqs, ng):
    for r in reqs:
        ref = _alone(ng, r)
        assert r.result is not None, r.rid
        assert r.n_out == ref[0].shape[0], (r.rid, r.n_out, ref[0].shape)
        for a, b in zip(r.result, ref):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), r.rid


@pytest.mark.parametrize("budget_mb", [4096, 96])
def test_served_results_equal_alone(gpu_lib, budget_mb):
    from paper_2603_16103_amd import serve
    ng = gpu_lib
    reqs = _requests()
    hosts = [serve._HostScene(r.scene) for r in reqs]
    srv = serve.BatchServer(budget_mb * 2**20, max_k=24, max_jobs=8, keep_results=True)
    log("rows", srv.rows, "budget MB", budget_mb)
    rep = srv.serve(reqs, hosts)
    log(rep)
    assert rep["requests"] == len(reqs) and rep["served"] == len(reqs)
    assert rep["latency_p99_s"] is not None
    if budget_mb == 96:
        assert srv.rows < sum(r.n for r in reqs)  # admission had to wait
    srv.batch.close()
    _check_same(reqs, ng)


def test_plain_server_matches(gpu_lib):
    from paper_2603_16103_amd import serve
    ng = gpu_lib
    reqs = _requests()[:4]
    hosts = [serve._HostScene(r.scene) for r in reqs]
    rep = serve.PlainServer(max(r.n for r in reqs), keep_results=True).serve(reqs, hosts)
    log(rep)
    _check_same(reqs, ng)


def test_served_request_against_the_oracle(gpu_lib):
    """One request served in real time among others, against the oracle's
    own loop on its scene: the same count, and >= 97% of the oracle's output
    splats found at a served splat within the end-to-end field bars.  The
    request is the largest with a ratio of at least 0.1 (a few passes: at
    1% one different merge early on changes a sizeable share of the ~100-splat
    clusters, as the precision-stress table shows)."""
    import oracle as O
    from paper_2603_16103_amd import serve
    from tests.e2e_compare import compare_by_position
    reqs = _requests()[:5]
    hosts = [serve._HostScene(r.scene) for r in reqs]
    srv = serve.BatchServer(256 * 2**20, max_k=24, max_jobs=8, keep_results=True)
    srv.serve(reqs, hosts)
    srv.batch.close()
    r = max((q for q in reqs if q.target >= 0.1 * q.n), key=lambda q: q.n)
    ref = O.simplify(r.scene.pos, r.scene.log_scale, r.scene.rot, r.scene.opacity, r.scene.sh,
                     r.target, r.k, seed=r.seed)
    assert r.n_out == ref.n
    err = compare_by_position(r.result, ref)
    log("served request", r.rid, r.n, "->", r.n_out, "vs oracle", err)
    assert err["within"] >= 0.97
