"""Launch shapes never change results: the same scene simplified under
extreme settings of every tunable launch parameter gives identical bytes."""
import numpy as np
import pytest

from paper_2603_16103_amd.synth import gen_scene

pytestmark = pytest.mark.gpu

# knn_block_min and knn_lane_rows route queries between the one-lane block
# search and the one-wave best-first search: their extremes send almost every
# query one way or the other
SETTINGS = [
    dict(cost_block=64, knn_block=256, knn_wave_grid=256, knn_level_bias=-2, select_check=1,
         knn_block_min=17, knn_lane_rows=64),
    dict(cost_block=128, knn_block=128, knn_wave_grid=65536, knn_level_bias=1, select_check=16,
         knn_block_min=1024, knn_lane_rows=4096),
    dict(cost_block=256, knn_block=64, knn_wave_grid=4096, knn_level_bias=-1, select_check=3,
         knn_block_min=17, knn_lane_rows=4096),
    dict(cost_block=256, knn_block=128, knn_wave_grid=1024, knn_level_bias=0, select_check=4,
         knn_block_min=1024, knn_lane_rows=64),
]


def _run(ng, sc, target, k):
    res = ng.simplify(ng.GaussianTensors.from_scene(sc), target, k=k, opts=ng.options(seed=5))
    return [x.cpu().numpy() for x in (res.pos, res.log_scale, res.rot, res.opacity, res.sh)]


@pytest.mark.parametrize("n,k", [(20000, 16), (70000, 24)])
def test_results_do_not_depend_on_launch_shapes(gpu_lib, n, k):
    ng = gpu_lib
    sc = gen_scene(n, 8)
    target = n // 10
    saved = [ng.get_tuning(b) for b in range(ng.TUNE_BUCKETS)]
    try:
        ref = _run(ng, sc, target, k)
        for s in SETTINGS:
            ng.set_tuning(-1, **s)
            got = _run(ng, sc, target, k)
            for a, b in zip(got, ref):
                assert a.shape == b.shape, s
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), s
    finally:
        for b, t in enumerate(saved):
            ng.set_tuning(b, **t)


def test_bad_tuning_values_are_rejected(gpu_lib):
    ng = gpu_lib
    with pytest.raises(ng.NanoGSError):
        ng.set_tuning(0, cost_block=96)
    with pytest.raises(ng.NanoGSError):
        ng.set_tuning(5, cost_block=64)
