"""Precision stress workload on one GPU: 6,000,000 splats on 64 random
planes where every splat has one log-scale ~ N(-7, 0.5) (flat) and 5% have
two (needles), k = 24, simplified to 1%.

Reports the whole loop (time, passes, edges, pairs and FP64-fallback edges
per pass) and the error of the FP32 path (with its FP64 fallback) against
the FP64 oracle on the first pass, teacher-forced on the same float32 state:
edge costs on a sample of the pass's edges and merged splats on a sample of
its pairs.  The oracle is test infrastructure; this script uses it only for
that error table.

``python -m paper_2603_16103_amd.stress [--n 6000000] [--sample 20000]``
prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2603_16103_amd import nanogs as ng  # noqa: E402
from paper_2603_16103_amd.synth import scene_precision_stress  # noqa: E402


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n", type=int, default=6_000_000)
    ap.add_argument("--sample", type=int, default=20000)
    args = ap.parse_args()
    import torch
    import oracle as O

    def eprint(*a):
        print(*a, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    ng.load()
    eprint("generating", args.n)
    sc, k, target = scene_precision_stress(args.n)
    target = max(int(math.ceil(0.01 * args.n)), 1)
    g = ng.GaussianTensors.from_scene(sc)
    out = ng.GaussianTensors.empty(sc.n)
    sim = ng.Simplifier(sc.n, k, ng.options(timing=True))
    sim(g, target, out)  # warm-up
    torch.cuda.synchronize()
    st = ng.Stats()
    t0 = time.perf_counter()
    n_out = sim(g, target, out, st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    d = st.as_dict()
    eprint("loop", dt, d["n_per_round"])
    res = {"workload": f"{sc.n} splats, 64 planes, flat + 5% needle scales, k={k}, -> 1%",
           "n": sc.n, "target": target, "n_out": n_out, "seconds": round(dt, 4),
           "gaussians_per_s": round(sc.n / dt, 1), "passes": d["rounds"],
           "n_per_pass": d["n_per_round"], "edges_per_pass": d["edges_per_round"],
           "pairs_per_pass": d["pairs_per_round"], "fp64_edges_per_pass": d["fallback_per_round"],
           "fp64_fraction_pass1": d["fallback_per_round"][0] / max(d["edges_per_round"][0], 1),
           "stage_ms": {s: round(v, 3) for s, v in d["stage_ms"].items()}}
    assert n_out == target

    # teacher-forced first pass against the oracle on samples
    eprint("first pass, teacher-forced")
    st64 = O.activate(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh)
    f32 = np.float32
    act = (st64.mu.astype(f32), st64.s.astype(f32), st64.q.astype(f32),
           st64.alpha.astype(f32), st64.f.astype(f32))
    del st64
    q = act[2].astype(np.float64)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    s64 = O.State(act[0].astype(np.float64), act[1].astype(np.float64), q,
                  act[3].astype(np.float64), act[4].astype(np.float64), np.arange(sc.n))
    nbr = ng.knn(_t(act[0]), k)
    ei, ej = ng.edges(nbr)
    del nbr
    crn = O.crn_block(0, 0, 1)
    splats = ng.SplatTensors(*(_t(x) for x in act))
    cost = ng.edge_cost(splats, ei, ej, crn)
    cost64 = ng.edge_cost(splats, ei, ej, crn, ng.options(precision=ng.PREC_FP64))
    a, b, c = ei.cpu().numpy(), ej.cpu().numpy(), cost.cpu().numpy()
    c64 = cost64.cpu().numpy()
    rng = np.random.default_rng(0)
    smp = rng.choice(a.size, min(args.sample, a.size), replace=False)
    ref = O.edge_costs(s64, a[smp], b[smp], crn)[0]
    wa = O.mass(s64.s[a[smp]], s64.alpha[a[smp]])
    wb = O.mass(s64.s[b[smp]], s64.alpha[b[smp]])
    flip = np.abs(wa / (wa + wb) - float(crn[0, 0])) < 1e-6

    def err_stats(got):
        e = np.abs(got.astype(np.float64) - ref)
        rel = e / np.maximum(np.abs(ref), 1e-12)
        ok = ~flip
        bound = e <= 1e-4 * np.abs(ref) + 1e-5
        return {"max_rel": float(rel[ok].max()), "p99_99_rel": float(np.percentile(rel[ok], 99.99)),
                "max_abs": float(e[ok].max()), "within_1e-4_rel_plus_1e-5": float(bound[ok].mean()),
                "component_flips": int(np.sum(flip & ~bound))}

    res["cost_error_fp32_with_fallback"] = err_stats(c[smp])
    res["cost_error_fp64_mode"] = err_stats(c64[smp])
    res["cost_sample_edges"] = int(smp.size)
    # merged splats on sampled pairs of the pass's greedy matching
    P = sc.n - target
    partner, npairs = ng.select(ei, ej, cost, sc.n, P)
    pt = partner.cpu().numpy()
    origin = np.arange(sc.n, dtype=np.int32)
    merged = ng.merge(ng.SplatTensors(*(_t(x) for x in act), _t(origin)), partner)
    org = merged.origin.cpu().numpy()
    lo = np.nonzero((pt >= 0) & (np.arange(sc.n) < pt))[0]
    pick = lo[rng.choice(lo.size, min(args.sample, lo.size), replace=False)]
    i, j = pick, pt[pick]
    pos_of = np.full(sc.n, -1, np.int64)
    pos_of[org] = np.arange(merged.n)
    rows = pos_of[i]
    mu_r, S_r, al_r, f_r = O.mpmm(s64.mu[i], s64.s[i], s64.q[i], s64.alpha[i], s64.f[i],
                                  s64.mu[j], s64.s[j], s64.q[j], s64.alpha[j], s64.f[j])
    mu = merged.mu.cpu().numpy()[rows].astype(np.float64)
    sg = merged.scale.cpu().numpy()[rows].astype(np.float64)
    qg = merged.quat.cpu().numpy()[rows].astype(np.float64)
    al = merged.alpha.cpu().numpy()[rows].astype(np.float64)
    S_g = O.covariance(sg, qg)
    fro = np.linalg.norm(S_g - S_r, axis=(1, 2)) / np.linalg.norm(S_r, axis=(1, 2))
    ev_r = np.sort(np.linalg.eigvalsh(S_r), 1)
    res["merge_error"] = {
        "pairs_sampled": int(pick.size),
        "mu_max_rel": float(np.max(np.abs(mu - mu_r) / np.maximum(np.abs(mu_r).max(1, keepdims=True), 1))),
        "sigma_fro_max_rel": float(fro.max()),
        "sorted_scale_max_rel": float(np.max(np.abs(np.sort(sg, 1) ** 2 - ev_r) / ev_r)) / 2.0,
        "alpha_max_abs": float(np.max(np.abs(al - al_r))),
        "flat_axis_min_scale": float(np.sqrt(ev_r[:, 0]).min())}
    res["pass1_pairs"] = int(npairs)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
