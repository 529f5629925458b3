"""Autotuner of the kernel launch shapes (``nanogs_tuning``).

For each size bucket (N < 2^16, N < 2^19, larger) the tuner builds a
representative synthetic scene (40k, 250k and 1M splats), runs one pass of
the simplification loop (``max_rounds = 1``, so every timed pass has that
bucket's size) and times it with the library's HIP-event stage timers.  It
then does a coordinate search: each parameter in turn takes every candidate
value, timed by the stages it affects (median of ``reps`` runs), and keeps
the fastest.  Launch shapes never change results; the tuner checks that by
hashing the output of every candidate run and refusing to write a table if
any two differ.

``python -m paper_2603_16103_amd.tune --out FILE`` writes the JSON table
that ``nanogs.load()`` applies when it sits next to the library as
``tuning_gfx950.json``.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2603_16103_amd import nanogs as ng  # noqa: E402
from paper_2603_16103_amd.synth import gen_scene  # noqa: E402

BUCKET_SIZES = (40_000, 250_000, 1_000_000)
CANDIDATES = {
    "cost_block": ((64, 128, 256), ("cost",)),
    "knn_block": ((64, 128, 256), ("knn_query",)),
    "knn_block_min": ((24, 32, 48, 64), ("knn_query", "knn_exact", "knn_wave")),
    "knn_lane_rows": ((192, 256, 384, 512, 768), ("knn_query", "knn_exact", "knn_wave")),
    "knn_wave_grid": ((4096, 16384, 65536), ("knn_wave",)),
    "knn_level_bias": ((-1, 0), ("knn_tree", "knn_query", "knn_exact", "knn_wave")),
    "select_check": ((2, 4, 8), ("select",)),
}
DEFAULT = {"cost_block": 256, "knn_block": 128, "knn_wave_grid": 16384, "knn_level_bias": 0,
           "select_check": 4, "knn_block_min": 32, "knn_lane_rows": 256}


def _digest(res) -> str:
    h = hashlib.sha256()
    for x in (res.pos, res.log_scale, res.rot, res.opacity, res.sh):
        h.update(x.cpu().numpy().tobytes())
    return h.hexdigest()


def _time(sim, g, target, out, stages, reps):
    import statistics
    times = []
    digest = None
    for _ in range(reps):
        st = ng.Stats()
        n_out = sim(g, target, out, st)
        d = st.as_dict()["stage_ms"]
        times.append(sum(d[s] for s in stages))
        digest = _digest(out.slice(n_out))
    return statistics.median(times), digest


def tune(reps: int = 3, log=print):
    import torch
    torch.cuda.set_device(0)
    ng.load()
    table = {"arch": "gfx950", "buckets": [], "measured_ms": []}
    for b, n in enumerate(BUCKET_SIZES):
        sc = gen_scene(n, 40 + b)
        g = ng.GaussianTensors.from_scene(sc)
        out = ng.GaussianTensors.empty(n)
        target = max(n // 10, 1)
        sim = ng.Simplifier(n, 16, ng.options(timing=True, max_rounds=1))
        best = dict(DEFAULT)
        ng.set_tuning(b, **best)
        sim(g, target, out)  # warm-up
        digests = set()
        measured = {}
        for name, (values, stages) in CANDIDATES.items():
            scores = {}
            for v in values:
                ng.set_tuning(b, **dict(best, **{name: v}))
                t, dg = _time(sim, g, target, out, stages, reps)
                digests.add(dg)
                scores[v] = t
                log(f"bucket {b} (n={n}) {name}={v}: {t:.3f} ms")
            best[name] = min(scores, key=scores.get)
            measured[name] = {str(k): round(v, 4) for k, v in scores.items()}
            ng.set_tuning(b, **best)
        if len(digests) != 1:
            raise RuntimeError(f"bucket {b}: launch shapes changed the result ({len(digests)} "
                               "distinct outputs)")
        table["buckets"].append(best)
        table["measured_ms"].append({"n": n, "stages": measured})
        log(f"bucket {b}: {best}")
    table["identical_outputs"] = True
    return table


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=ng.TUNING_FILE)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    table = tune(args.reps, log=lambda *a: print(*a, file=sys.stderr, flush=True))
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
    print(json.dumps({"written": args.out, "buckets": table["buckets"]}), flush=True)


if __name__ == "__main__":
    main()
