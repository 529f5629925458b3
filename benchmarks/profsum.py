"""Summaries of rocprofv3 output for the committed profiles.

``python benchmarks/profsum.py stats KERNEL_STATS_CSV OUT_MD TITLE CMD``
writes a markdown table of a ``--kernel-trace --stats`` run.

``python benchmarks/profsum.py occ OUT_MD CMD PMC_CSV TRACE_CSV KERNEL ...``
tabulates an ``--pmc`` run of SQ counters (waves, VALU/LDS instructions, LDS
bank conflicts, wave and busy cycles) with the register and LDS footprint of
each named kernel from a ``--kernel-trace`` CSV.

``python benchmarks/profsum.py traffic OUT_JSON OUT_MD CMD
FETCH_CSV WRITE_CSV CALIB_FETCH_CSV CALIB_WRITE_CSV CALIB_BYTES KERNEL[=SOURCE] ...``
turns two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of the benchmark
and the same two counters on a plain copy of CALIB_BYTES into HBM bytes per
launch of each named kernel: each counter (KiB per dispatch) is scaled by the
ratio of the copy's known bytes to what that counter read for the copy.  The
JSON records the hash of each kernel's source file, so a reader can tell when
the kernel changed after the counters were taken.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2603_16103_amd")


def short(name: str) -> str:
    m = re.search(r"(k_\w+|__amd\w+)(<[\d, ]+>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "").replace(" ", "")
    m = re.search(r"(\w*[Cc]opy\w*)", name)
    return m.group(1) if m else name[:48]


def src_hash(fname: str) -> str:
    with open(os.path.join(HERE, "csrc", fname), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def stats(csv_path, out_md, title, cmd):
    rows = list(csv.DictReader(open(csv_path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    with open(out_md, "w") as f:
        f.write(f"# rocprofv3 kernel statistics: {title}\n\n")
        f.write("Command (from the repository root on one MI355X):\n\n```\n" + cmd + "\n```\n\n")
        f.write("| kernel | calls | total ms | avg us | min us | max us | % |\n")
        f.write("|---|---|---|---|---|---|---|\n")
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
            f.write(f"| {short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} "
                    f"| {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} "
                    f"| {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |\n")
        f.write(f"\nTotal kernel time {tot / 1e6:.2f} ms.\n")


def per_kernel(csv_path, counter):
    """kernel -> list of per-dispatch counter values (KiB)."""
    vals = defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter:
            vals[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


def traffic(out_json, out_md, cmd, fetch_csv, write_csv, cfetch_csv, cwrite_csv, calib_bytes,
            kernels):
    calib_bytes = float(calib_bytes)
    cf = per_kernel(cfetch_csv, "FETCH_SIZE")
    cw = per_kernel(cwrite_csv, "WRITE_SIZE")
    # the copy kernel: the dispatch class with the largest counts
    copy_f = max(cf.items(), key=lambda kv: max(kv[1]))
    copy_w = max(cw.items(), key=lambda kv: max(kv[1]))
    sf = calib_bytes / (max(copy_f[1]) * 1024.0)
    sw = calib_bytes / (max(copy_w[1]) * 1024.0)
    fe = per_kernel(fetch_csv, "FETCH_SIZE")
    wr = per_kernel(write_csv, "WRITE_SIZE")
    out = {"copy_kernel": copy_f[0], "calib_bytes": calib_bytes,
           "fetch_scale": sf, "write_scale": sw, "kernels": {}}
    for spec in kernels:
        name, _, src = spec.partition("=")
        f = fe.get(name, [])
        w = wr.get(name, [])
        if not f or not w:
            continue
        fk = sum(f) / len(f)
        wk = sum(w) / len(w)
        out["kernels"][name] = {"launches": len(f), "fetch_kib_avg": fk, "write_kib_avg": wk,
                                "bytes_per_launch": fk * 1024.0 * sf + wk * 1024.0 * sw,
                                "source": src or None,
                                "source_sha": src_hash(src) if src else None}
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1)
    with open(out_md, "w") as fh:
        fh.write("# HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE)\n\n")
        fh.write("Commands (from the repository root on one MI355X):\n\n```\n" + cmd + "\n```\n\n")
        fh.write(f"Calibration: `{copy_f[0]}` copying {calib_bytes / 2**20:.0f} MiB reads "
                 f"{max(copy_f[1]):.0f} KiB (FETCH_SIZE) and writes {max(copy_w[1]):.0f} KiB "
                 f"(WRITE_SIZE) per dispatch; scale factors {sf:.4f} (fetch), {sw:.4f} (write).\n\n")
        fh.write("| kernel | launches | FETCH KiB/launch | WRITE KiB/launch | HBM bytes/launch (scaled) |\n")
        fh.write("|---|---|---|---|---|\n")
        for name, e in out["kernels"].items():
            fh.write(f"| {name} | {e['launches']} | {e['fetch_kib_avg']:.0f} | {e['write_kib_avg']:.0f} "
                     f"| {e['bytes_per_launch']:.4g} |\n")


def occ(out_md, cmd, pmc_csv, trace_csv, kernels):
    sums = defaultdict(lambda: defaultdict(float))
    for r in csv.DictReader(open(pmc_csv)):
        sums[short(r["Kernel_Name"])][r["Counter_Name"]] += float(r["Counter_Value"])
    res = {}
    for r in csv.DictReader(open(trace_csv)):
        k = short(r["Kernel_Name"])
        if k not in res:
            res[k] = (int(r["VGPR_Count"]), int(r["Accum_VGPR_Count"]), int(r["LDS_Block_Size"]),
                      int(r["Workgroup_Size_X"]))
    with open(out_md, "w") as fh:
        fh.write("# Occupancy, instruction mix and LDS bank conflicts (rocprofv3 --pmc)\n\n")
        fh.write("Commands (from the repository root on one MI355X):\n\n```\n" + cmd + "\n```\n\n")
        fh.write("Registers and LDS per workgroup from the kernel trace.  Waves/SIMD by "
                 "registers: min(8, 512 / (VGPR + AGPR rounded up to 8)).  Resident waves "
                 "per CU: SQ_WAVE_CYCLES / SQ_BUSY_CU_CYCLES.  Per-wave counts: counter / "
                 "SQ_WAVES.  Bank-conflict share: SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS.\n\n")
        fh.write("| kernel | VGPR | AGPR | LDS B/WG | WG | waves/SIMD (regs) | waves | resident "
                 "waves/CU | VALU/wave | VMEM rd/wave | LDS/wave | LDS conflict share |\n")
        fh.write("|---|---|---|---|---|---|---|---|---|---|---|---|\n")
        for k in kernels:
            c = sums.get(k)
            if not c:
                continue
            v, a, lds, wg = res.get(k, (0, 0, 0, 0))
            regs = ((v + a + 7) // 8) * 8
            lim = min(8, 512 // regs) if regs else 8
            waves = c.get("SQ_WAVES", 0.0) or 1.0
            resident = c.get("SQ_WAVE_CYCLES", 0.0) / max(c.get("SQ_BUSY_CU_CYCLES", 0.0), 1.0)
            conf = c.get("SQ_LDS_BANK_CONFLICT", 0.0) / max(c.get("SQ_ACTIVE_INST_LDS", 0.0), 1.0)
            fh.write(f"| {k} | {v} | {a} | {lds} | {wg} | {lim} | {waves:.0f} | {resident:.1f} "
                     f"| {c.get('SQ_INSTS_VALU', 0) / waves:.0f} "
                     f"| {c.get('SQ_INSTS_VMEM_RD', 0) / waves:.0f} "
                     f"| {c.get('SQ_INSTS_LDS', 0) / waves:.0f} | {conf:.3f} |\n")


def bench(out_md, default_json, cold_json, tree, traffic_json):
    """Summary of two bench.py lines (default run and cold-cache run)."""
    def last_json(path):
        for line in reversed(open(path).read().splitlines()):
            if line.startswith("{"):
                return json.loads(line)
        raise SystemExit(f"no JSON line in {path}")
    d, c = last_json(default_json), last_json(cold_json)
    tr = json.load(open(traffic_json)).get("kernels", {})
    with open(out_md, "w") as fh:
        fh.write("# bench.py on one MI355X: 1M synthetic splats -> 100k, k=16, S=1\n\n")
        fh.write(f"Tree: {tree}.\n\nCommands (from the repository root):\n\n```\n"
                 "python3 bench.py\n"
                 "python3 bench.py --steps 5 --warmup 1 --no-cpu-baseline --flush-mib 1024\n"
                 f"python benchmarks/profsum.py bench {out_md} <default line> <cold line> {tree} "
                 f"{traffic_json}\n```\n\n")
        fh.write("| run | Gaussians/s | ms/step |\n|---|---|---|\n")
        fh.write(f"| default ({d['steps']} steps) | {d['value']:.4g} | {d['ms_per_step']} |\n")
        fh.write(f"| cold caches (1 GiB copied before each step, steps timed alone) "
                 f"| {c['value']:.4g} | {c['ms_per_step']} |\n\n")
        fh.write("Stage times per step (ms, HIP events on the call's stream):\n\n")
        fh.write("| stage | default | cold |\n|---|---|---|\n")
        for k, v in d["stage_ms_per_step"].items():
            fh.write(f"| {k} | {v} | {c['stage_ms_per_step'].get(k)} |\n")
        fh.write("\nRoofline of the dominant kernel and the others (algorithmic bytes per unit: "
                 "kNN 12 + 4k B per splat; edge cost 236 B per splat + 12 B per edge; selection "
                 "12 B per edge + 4 B per splat; factor precompute 72 B per splat):\n\n")
        fh.write("| entry | kernel | avg launch us | algorithmic per launch | achieved | frac of peak "
                 "| counted traffic per launch |\n|---|---|---|---|---|---|---|\n")
        ents = [("dominant", d["roofline"])] + list(d.get("roofline_other_kernels", {}).items())
        for name, r in ents:
            algo = r.get("algo_bytes_per_launch") or r.get("algo_flops_per_launch")
            unit = "B" if "algo_bytes_per_launch" in r else "flop"
            t = tr.get(r["kernel"], {}).get("bytes_per_launch")
            fh.write(f"| {name} | {r['kernel']} | {r['avg_launch_us']} | {algo:.4g} {unit} "
                     f"| {r['achieved']} {r['unit']} | {r['frac']} "
                     f"| {f'{t:.4g} B' if t else '-'} |\n")
        cb = d.get("cpu_baseline")
        if cb:
            fh.write(f"\nCPU baseline (the FP64 oracle): {cb['sample']}; {cb['value']:.4g} "
                     f"Gaussians/s on {cb['cores']} threads, "
                     f"{cb['single_thread']['value']:.4g} on one thread.\n")


def main(argv):
    if argv[0] == "stats":
        stats(*argv[1:5])
    elif argv[0] == "occ":
        occ(argv[1], argv[2], argv[3], argv[4], argv[5:])
    elif argv[0] == "traffic":
        traffic(*argv[1:9], argv[9:])
    elif argv[0] == "bench":
        bench(*argv[1:6])
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
