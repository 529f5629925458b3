"""Markdown summary of the precision-stress error table.

``python benchmarks/stress_table.py TABLE_JSON OUT_MD CMD TREE`` turns the
JSON that tests/test_gpu_stress_table.py writes (NANOGS_STRESS_OUT) into the
committed summary: per pass, every stage's output against the FP64 oracle
teacher-forced on the GPU's own state, then the final outputs of the fused
loop against the oracle's loop.
"""
import json
import sys


def fmt(x):
    return f"{x:.3g}" if isinstance(x, float) else str(x)


def main(table_json, out_md, cmd, tree):
    t = json.load(open(table_json))
    with open(out_md, "w") as f:
        f.write(f"# Precision stress: {t['workload']} (one MI355X)\n\n")
        f.write(f"Tree: {tree}.  Command (repository root):\n\n```\n{cmd}\n```\n\n")
        f.write("Every pass runs through the stage entry points on the GPU's own float32 state; "
                "each stage's output is compared with the FP64 oracle teacher-forced on that "
                f"state ({t['sample']} sampled rows, edges and pairs per pass; the union edges "
                "and the greedy characterisation over every edge).\n\n")
        f.write("| pass | N | kNN rows equal | edges | edges equal | cost max rel (FP32+fallback) "
                "| cost max abs | within 1e-4 abs(C) + 1e-5 | cost max rel (FP64 mode) | pairs | greedy "
                "| mu max rel | Sigma max rel | scales max rel | alpha max abs | f max rel |\n")
        f.write("|" + "---|" * 16 + "\n")
        for r in t["passes"]:
            c, c64, m = r["cost_fp32_fallback"], r["cost_fp64_mode"], r["merge"]
            f.write(f"| {r['pass']} | {r['N']} | {r['knn_rows_equal']}/{r['knn_rows_checked']} "
                    f"| {r['edges']} | {r['edges_equal']} | {fmt(c['max_rel'])} | {fmt(c['max_abs'])} "
                    f"| {fmt(c['within_bar'])} | {fmt(c64['max_rel'])} | {r['pairs']} "
                    f"| {r['greedy_characterisation']} | {fmt(m['mu_max_rel'])} "
                    f"| {fmt(m['sigma_fro_max_rel'])} | {fmt(m['sorted_scale_max_rel'])} "
                    f"| {fmt(m['alpha_max_abs'])} | {fmt(m['f_max_rel'])} |\n")
        f.write(f"\nChained stages equal the fused loop bit for bit: {t['chained_equals_fused']}.\n")
        fo = t.get("final_outputs")
        if fo:
            f.write(f"\n## Final outputs against the oracle's own loop ({fo['n']} stress splats -> "
                    f"{fo['target']}, k={fo['k']}, {fo['passes']} passes)\n\n")
            f.write(f"Identical provenance pairs: {fmt(fo['identical_pairs'])} (per pass "
                    f"{', '.join(fmt(x) for x in fo['identical_pairs_per_pass'])}); FP64-fallback "
                    f"edges per pass {fo['fallback_per_pass']}; clusters with identical membership "
                    f"{fmt(fo['identical_clusters'])} of {fo['clusters']}.\n\n")
            f.write("| output | max | p99 |\n|---|---|---|\n")
            for name, what in (("mu", "centre, relative to max(abs(mu), 1)"),
                               ("sigma", "covariance, Frobenius relative"),
                               ("alpha", "opacity, absolute"), ("f", "SH, relative")):
                if name + "_max" in fo:
                    f.write(f"| {what} | {fmt(fo[name + '_max'])} | {fmt(fo[name + '_p99'])} |\n")


if __name__ == "__main__":
    main(*sys.argv[1:5])
