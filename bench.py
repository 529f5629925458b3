#!/usr/bin/env python3
"""Throughput of the splat-simplification hot path on one MI355X.

A step is one full nanogs_simplify call: 1,000,000 synthetic 3DGS splats
(8 planes + 4 spheres + 10% clutter, seed 2) simplified to 100,000 with a
k = 16 kNN graph and S = 1 shared draw, every pass of Algorithm 1 included
(kNN graph, union edges, edge costs, greedy disjoint pairs, merge and
compaction).  Inputs are resident in HBM before the timed region; the output
is written to preallocated device buffers.

Prints one JSON line (metric, value, roofline of the dominant kernel, the
FP64 oracle's CPU throughput on a bounded sample).  Progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_1m.json")


def eprint(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash(name):
    with open(os.path.join(ROOT, "paper_2603_16103_amd", "csrc", name), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


# Roofline terms of the single-kernel stages, per pass: (bound, algorithmic
# work, unit).  n = splats in the pass, e = edges, k = kNN size, screens =
# float distance screens the kNN block gather made (library statistics).
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published
FLOPS_PER_SCREEN = 8      # 3 sub, 1 mul, 2 fma


def stage_work(stage, n, e, k, screens):
    if stage == "knn_query":   # block gather: distance screens (FP32 ALU)
        return "alu", FLOPS_PER_SCREEN * screens
    if stage == "cost":        # cen 16 + factors 32 + SH 192 per splat; ends 8 + cost 4 +
        return "hbm", 240 * n + 36 * e  # two adjacency entries 24 per edge
    if stage == "precompute":  # shape 32 in, factors 32 out
        return "hbm", 64 * n
    return None, None


KERNEL_OF = {"knn_query": "k_knn_block<16>", "cost": "k_edge_cost", "precompute": "k_precompute"}
SOURCE_OF = {"knn_query": "knn.hip", "cost": "cost.hip", "precompute": "cost.hip"}


def traffic_for(stage):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by the copy-kernel calibration); None when absent or
    when the kernel's source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = t.get("kernels", {}).get(KERNEL_OF[stage])
    if not ent or ent.get("source_sha") != src_hash(SOURCE_OF[stage]):
        return None
    return ent["bytes_per_launch"]


def cpu_baseline(sample_n):
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:  # pragma: no cover
        lim = None
    import oracle as O
    from paper_2603_16103_amd.synth import gen_scene
    sc = gen_scene(sample_n, 2)
    target = max(int(math.ceil(0.1 * sample_n)), 1)
    t0 = time.perf_counter()
    st = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, target, 16)
    dt = time.perf_counter() - t0
    assert st.n == target
    del lim, np
    return {"value": sample_n / dt, "unit": "Gaussians/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle (numpy, one thread), {sample_n} splats from the same "
                      f"generator (seed 2) simplified to 10% with k=16, {dt:.1f} s",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--cpu-sample", type=int, default=100_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB three times (the "
                         "reference kernel for scaling the HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(one scene per GPU shards trivially; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_16103_amd import nanogs as ng
    from paper_2603_16103_amd.synth import scene_plain_gpu

    torch.cuda.set_device(0)
    if args.calib_copy_mib:
        nbytes = args.calib_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": nbytes, "copies": 3}), flush=True)
        return
    ng.load()
    eprint("generating scene", args.n)
    sc, k, target = scene_plain_gpu(args.n)
    g = ng.GaussianTensors.from_scene(sc)
    out = ng.GaussianTensors.empty(sc.n)
    simp = ng.Simplifier(sc.n, k, ng.options(timing=True))
    torch.cuda.synchronize()
    for i in range(args.warmup):
        simp(g, target, out)
        eprint(f"warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()

    stage_ms = {s: 0.0 for s in ng.STAGES}
    launches = {s: 0 for s in ng.STAGES}
    work_by_stage = {s: 0.0 for s in ng.STAGES}
    edges_total = 0
    last = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = ng.Stats()
        n_out = simp(g, target, out, st)
        d = st.as_dict()
        for s in ng.STAGES:
            stage_ms[s] += d["stage_ms"][s]
            launches[s] += d["stage_launches"][s]
        for n_r, e_r, sc_r in zip(d["n_per_round"], d["edges_per_round"],
                                  d["knn_screens_per_round"]):
            edges_total += e_r
            for s in ng.STAGES:
                _, w = stage_work(s, n_r, e_r, k, sc_r)
                if w is not None:
                    work_by_stage[s] += w
        last = d
        eprint(f"step {i + 1}/{args.steps}: {n_out} splats, {d['rounds']} passes")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert n_out == target, (n_out, target)

    ms_step = 1000.0 * dt / args.steps
    value = args.n * args.steps / dt
    def roof(stage):
        bound, _ = stage_work(stage, 1, 1, k, 1)
        avg_ms = stage_ms[stage] / launches[stage]
        per_launch = work_by_stage[stage] / launches[stage]
        if bound == "hbm":
            achieved, peak, unit = per_launch / (avg_ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            achieved, peak, unit = per_launch / (avg_ms * 1e-3) / 1e12, FP32_PEAK_TFLOPS, "TFLOP/s"
        return {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 5), "traffic": traffic_for(stage),
                "kernel": KERNEL_OF[stage], "avg_launch_us": round(1000 * avg_ms, 2),
                ("algo_bytes_per_launch" if bound == "hbm" else "algo_flops_per_launch"):
                    int(per_launch)}

    single = [s for s in KERNEL_OF if launches[s] > 0]
    dom = max(single, key=lambda s: stage_ms[s])  # the single-kernel stage with most time
    roof_dom = roof(dom)
    others = {s: roof(s) for s in single if s != dom}
    res = {
        "metric": "Gaussians simplified/s (1M→10%)",
        "value": round(value, 1),
        "unit": "Gaussians/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1M synthetic 3DGS splats (8 planes, 4 spheres, 10% clutter, "
                               "seed 2) -> 100k, k=16, S=1, FP32 costs with FP64 fallback",
                   "n": args.n, "target_n": target, "k": k, "S": 1,
                   "passes": last["rounds"], "n_per_pass": last["n_per_round"],
                   "edges_per_pass": last["edges_per_round"],
                   "fp64_edges_per_pass": last["fallback_per_round"],
                   "knn_wave_retries_per_pass": last["knn_retry_per_round"],
                   "knn_screens_per_pass": last["knn_screens_per_round"]},
        "edge_costs_per_s": round(edges_total / (stage_ms["cost"] * 1e-3), 1)
        if stage_ms["cost"] > 0 else None,
        "stage_ms_per_step": {s: round(stage_ms[s] / args.steps, 4) for s in ng.STAGES},
        "roofline": roof_dom,
        "roofline_other_kernels": others,
    }
    if not args.no_cpu_baseline:
        eprint("cpu baseline (oracle) on", args.cpu_sample, "splats")
        res["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
