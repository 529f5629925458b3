"""Per-stage timing: every stage, a chosen subset, or none, with results that
do not depend on it (the events only observe the stream)."""
import sys

import numpy as np
import pytest

from paper_2603_16103_amd.synth import gen_scene

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_stage_timing_subsets(gpu_lib):
    ng = gpu_lib
    sc = gen_scene(20000, 71)
    g = ng.GaussianTensors.from_scene(sc)
    runs = {}
    for name, timing in (("off", False), ("all", True), ("knn", ("knn_query", "cost"))):
        log("timing", name)
        res, st = ng.simplify(g, 2000, k=16, opts=ng.options(timing=timing), return_stats=True)
        runs[name] = (res.numpy(), st)
    base = runs["off"][0]
    for name in ("all", "knn"):
        for a, b in zip(runs[name][0], base):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    rounds = runs["all"][1]["rounds"]
    assert rounds >= 2
    assert all(v == 0 for v in runs["off"][1]["stage_launches"].values())
    assert runs["all"][1]["stage_launches"]["knn_query"] == rounds
    assert runs["all"][1]["stage_launches"]["merge"] == rounds
    sub = runs["knn"][1]["stage_launches"]
    assert sub["knn_query"] == rounds and sub["cost"] == rounds
    assert all(v == 0 for s, v in sub.items() if s not in ("knn_query", "cost"))
    assert runs["knn"][1]["stage_ms"]["knn_query"] > 0
