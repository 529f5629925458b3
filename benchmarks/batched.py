"""Batched workload on one GPU: many scenes simplified together through the
batch API against the same scenes simplified one at a time.

Scenes come from ``synth.batch_specs`` (64 scenes, n log-uniform in
[5e4, 2e6], 4 to 64 surfaces, keep ratio 0.5 / 0.2 / 0.1, k = 16).  Every
input sits in HBM before either timed region starts.  The batched run submits
every scene to one ``nanogs.Batch`` (one launch per stage and pass for all
live scenes) and runs it to completion; the plain run calls
``nanogs_simplify`` per scene.  Each scene's batched output is checked
bitwise against its plain output.

``python benchmarks/batched.py [--scenes 64] [--hi 2e6]`` prints
one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2603_16103_amd import nanogs as ng  # noqa: E402
from paper_2603_16103_amd.synth import batch_specs, gen_scene  # noqa: E402


def _make(spec):
    n, seed, planes, spheres, _ = spec
    return gen_scene(n, seed, n_planes=planes, n_spheres=spheres)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--scenes", type=int, default=64)
    ap.add_argument("--hi", type=float, default=2e6)
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    import torch

    def eprint(*a):
        print(*a, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    ng.load()
    specs = batch_specs(args.scenes, hi=args.hi)
    total = sum(s[0] for s in specs)
    eprint("generating", len(specs), "scenes,", total, "splats")
    with ProcessPoolExecutor(args.workers) as ex:
        scenes = list(ex.map(_make, specs))
    gs = [ng.GaussianTensors.from_scene(sc) for sc in scenes]
    targets = [max(int(math.ceil(s[4] * s[0])), 1) for s in specs]
    del scenes
    torch.cuda.synchronize()

    # plain: one scene at a time
    nmax = max(s[0] for s in specs)
    simp = ng.Simplifier(nmax, 16)
    outs_plain = [ng.GaussianTensors.empty(g.n) for g in gs]
    simp(gs[0], targets[0], outs_plain[0])  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_plain = [simp(g, t, o) for g, t, o in zip(gs, targets, outs_plain)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    eprint("plain", t_plain)
    del simp

    # batched: every scene in one working set
    outs_b = [ng.GaussianTensors.empty(g.n) for g in gs]
    b = ng.Batch(total, max_k=16, max_jobs=len(gs))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ids = [b.submit(g, t, 16, seed=0, out=o) for g, t, o in zip(gs, targets, outs_b)]
    b.run()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    eprint("batched", t_batch)
    same = 0
    for i, (jid, o) in enumerate(zip(ids, outs_b)):
        state, n_out, _ = b.job(jid)
        assert state == ng.JOB_DONE and n_out == n_plain[i], (i, state, n_out, n_plain[i])
        rb, rp = o.slice(n_out), outs_plain[i].slice(n_out)
        if all(torch.equal(x, y) for x, y in zip(
                (rb.pos, rb.log_scale, rb.rot, rb.opacity, rb.sh),
                (rp.pos, rp.log_scale, rp.rot, rp.opacity, rp.sh))):
            same += 1
    b.close()
    print(json.dumps({
        "workload": f"{len(specs)} scenes, n log-uniform [5e4, {args.hi:.0e}], 4-64 surfaces, "
                    "keep 0.5/0.2/0.1, k=16",
        "scenes": len(specs), "splats": total,
        "plain_s": round(t_plain, 4), "batched_s": round(t_batch, 4),
        "plain_gaussians_per_s": round(total / t_plain, 1),
        "batched_gaussians_per_s": round(total / t_batch, 1),
        "speedup": round(t_plain / t_batch, 3),
        "identical_scenes": same}), flush=True)


if __name__ == "__main__":
    main()
