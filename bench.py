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


# Roofline terms per pass: (bound, algorithmic work).  n = splats in the
# pass, e = edges, k = kNN size, screens = float distance screens of the kNN
# block gather (library statistics).  Algorithmic bytes are what the step
# must move at least: kNN reads the centres (12 B) and writes k indices
# (4k B) per splat; the edge cost reads the activated attributes (mu 12, s 12,
# q 16, alpha 4, SH 192 = 236 B) per splat and each edge's ends (8 B) and
# writes its cost (4 B); the selection reads ends and cost (12 B per edge)
# and writes a partner per splat (4 B); the factor precompute reads the
# shape (32 B) and writes the factors and the weight (40 B) per splat.
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published
FLOPS_PER_SCREEN = 8      # 3 sub, 1 mul, 2 fma (+2 for the bin/compare)


def stage_work(stage, n, e, k, screens):
    if stage == "knn_query":   # k_knn_block: the kNN's bytes
        return "hbm", (12 + 4 * k) * n
    if stage == "knn_alu":     # the same kernel on the FP32 ALU roof
        return "alu", FLOPS_PER_SCREEN * screens
    if stage == "cost":
        return "hbm", 236 * n + 12 * e
    if stage == "select":      # a stage of several kernels
        return "hbm", 12 * e + 4 * n
    if stage == "precompute":
        return "hbm", 72 * n
    return None, None


KERNEL_OF = {"knn_query": "k_knn_block<16,4>", "cost": "k_edge_cost", "precompute": "k_precompute",
             "select": "select stage (k_ld_pick, k_ld_match, k_ld_tail, k_topp_seg)",
             "knn_alu": "k_knn_block<16,4>"}
SOURCE_OF = {"knn_query": "knn.hip", "cost": "cost.hip", "precompute": "cost.hip",
             "select": "select.hip", "knn_alu": "knn.hip"}
STAGE_OF = {"knn_alu": "knn_query"}  # timed stage of a roofline entry


def traffic_for(stage):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by the copy-kernel calibration); None when absent or
    when the kernel's source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = t.get("kernels", {}).get(KERNEL_OF[stage].split()[0])
    if not ent or ent.get("source_sha") != src_hash(SOURCE_OF[stage]):
        return None
    return ent["bytes_per_launch"]


def cpu_baseline(sample_n, workers):
    """The FP64 oracle simplifying a bounded sample of the same workload
    (same generator, 10% target, k=16) on the host: once with `workers`
    threads for its per-query and per-edge steps (the reported baseline),
    once on one thread.  BLAS threads are pinned to one in both."""
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:  # pragma: no cover
        lim = None
    import oracle as O
    from paper_2603_16103_amd.synth import gen_scene
    sc = gen_scene(sample_n, 2)
    target = max(int(math.ceil(0.1 * sample_n)), 1)
    times = {}
    for w in (workers, 1):
        t0 = time.perf_counter()
        st = O.simplify(sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh, target, 16, workers=w)
        times[w] = time.perf_counter() - t0
        assert st.n == target
    del lim
    return {"value": sample_n / times[workers], "unit": "Gaussians/s", "cores": workers,
            "kind": "oracle",
            "sample": f"FP64 oracle (numpy), {sample_n} splats from the same generator (seed 2) "
                      f"simplified to 10% with k=16: {times[workers]:.1f} s on {workers} threads",
            "seconds": round(times[workers], 2),
            "single_thread": {"value": sample_n / times[1], "cores": 1,
                              "seconds": round(times[1], 2)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--cpu-sample", type=int, default=200_000)
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--flush-mib", type=int, default=0,
                    help="cold-cache variant: copy this many MiB between steps (outside the "
                         "timed calls) so no step finds its data in the caches; the value is "
                         "then the sum of the per-step times")
    ap.add_argument("--breakdown-steps", type=int, default=2,
                    help="untimed steps with every stage timed (stage breakdown)")
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

    flush = None
    if args.flush_mib:
        flush = torch.empty(args.flush_mib << 18, dtype=torch.float32, device="cuda")
        flush_dst = torch.empty_like(flush)

    def run(steps, label):
        """steps calls; returns (seconds, per-stage ms and launches, the
        algorithmic work per roofline entry, edges, the last call's stats)"""
        acc = {"ms": {s: 0.0 for s in ng.STAGES}, "launches": {s: 0 for s in ng.STAGES},
               "work": {s: 0.0 for s in KERNEL_OF}, "edges": 0, "last": None}
        cold_s = 0.0
        n_out = target
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            st = ng.Stats()
            if flush is not None:
                flush_dst.copy_(flush)
                torch.cuda.synchronize()
                tc = time.perf_counter()
            n_out = simp(g, target, out, st)
            if flush is not None:
                torch.cuda.synchronize()
                cold_s += time.perf_counter() - tc
            d = st.as_dict()
            for s in ng.STAGES:
                acc["ms"][s] += d["stage_ms"][s]
                acc["launches"][s] += d["stage_launches"][s]
            for n_r, e_r, sc_r in zip(d["n_per_round"], d["edges_per_round"],
                                      d["knn_screens_per_round"]):
                acc["edges"] += e_r
                for s in KERNEL_OF:
                    _, w = stage_work(s, n_r, e_r, k, sc_r)
                    if w is not None:
                        acc["work"][s] += w
            acc["last"] = d
            eprint(f"{label} {i + 1}/{steps}: {n_out} splats, {d['rounds']} passes")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert n_out == target, (n_out, target)
        return (cold_s if flush is not None else dt), acc

    def roof(stage, acc):
        bound, _ = stage_work(stage, 1, 1, k, 1)
        ts = STAGE_OF.get(stage, stage)
        avg_ms = acc["ms"][ts] / acc["launches"][ts]
        per_launch = acc["work"][stage] / acc["launches"][ts]
        if bound == "hbm":
            achieved, peak, unit = per_launch / (avg_ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
            tr = traffic_for(stage)
        else:
            achieved, peak, unit = per_launch / (avg_ms * 1e-3) / 1e12, FP32_PEAK_TFLOPS, "TFLOP/s"
            tr = None
        return {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 5), "traffic": tr,
                "kernel": KERNEL_OF[stage], "avg_launch_us": round(1000 * avg_ms, 2),
                ("algo_bytes_per_launch" if bound == "hbm" else "algo_flops_per_launch"):
                    int(per_launch)}

    # breakdown steps (outside the timed region) with every stage timed: the
    # per-stage times and the dominant kernel, the single-kernel stage with
    # most time
    _, bd = run(args.breakdown_steps, "breakdown step")
    single = [s for s in ("knn_query", "cost", "precompute") if bd["launches"][s] > 0]
    dom = max(single, key=lambda s: bd["ms"][s]) if single else "knn_query"
    # the timed steps record HIP events around the dominant kernel only (an
    # event record at every stage boundary costs stream time)
    simp.opts.timing = ng.options(timing=(STAGE_OF.get(dom, dom),)).timing
    dt, acc = run(args.steps, "step")
    last = acc["last"]
    ms_step = 1000.0 * dt / args.steps
    value = args.n * args.steps / dt
    roof_dom = roof(dom, acc)
    others = {s: roof(s, bd) for s in KERNEL_OF
              if s != dom and bd["launches"][STAGE_OF.get(s, s)] > 0}
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
                   "knn_screens_per_pass": last["knn_screens_per_round"],
                   "cold_cache_flush_mib": args.flush_mib or None},
        "edge_costs_per_s": round(bd["edges"] / (bd["ms"]["cost"] * 1e-3), 1)
        if bd["ms"]["cost"] > 0 else None,
        "stage_ms_per_step": {s: round(bd["ms"][s] / args.breakdown_steps, 4)
                              for s in ng.STAGES} if args.breakdown_steps else None,
        "stage_timing": f"stage_ms_per_step, edge_costs_per_s and roofline_other_kernels from "
                        f"{args.breakdown_steps} breakdown steps with every stage timed, outside "
                        f"the timed region; the timed steps time the dominant kernel's stage "
                        f"({STAGE_OF.get(dom, dom)}) only",
        "roofline": roof_dom,
        "roofline_other_kernels": others,
    }
    if not args.no_cpu_baseline:
        eprint("cpu baseline (oracle) on", args.cpu_sample, "splats")
        res["cpu_baseline"] = cpu_baseline(args.cpu_sample, args.cpu_workers)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
