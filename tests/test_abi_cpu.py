"""The C-ABI library without a GPU: it loads, exports every declared symbol,
answers size queries, rejects bad arguments before touching the device, and
its host-side draw generator matches the stored known answers bit for bit."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2603_16103_amd import nanogs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nanogs.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nanogs_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(nanogs.LIB_PATH):
        pytest.skip("library not built")
    return nanogs.load()


def test_every_declared_symbol_is_exported(lib):
    decl = _declared()
    assert len(decl) == len(set(nanogs.exported_symbols()))
    out = subprocess.run(["nm", "-D", "--defined-only", nanogs.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (nanogs_\w+)", out))
    missing = [d for d in decl if d not in exported]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(decl) <= set(nanogs.exported_symbols())


def test_crn_matches_known_answers(lib):
    from tests.golden.make_golden import load_crn_golden
    for (seed, r, S), vals in load_crn_golden().items():
        got = nanogs.crn(seed, r, S)
        np.testing.assert_array_equal(got.view(np.uint32), vals.view(np.uint32))


def test_default_options(lib):
    o = nanogs.Options()
    lib.nanogs_default_options(ctypes.byref(o))
    assert o.S == 1 and o.app_dims == 48 and o.precision == 0
    assert abs(o.fb_ratio - 1 / 256) < 1e-9 and o.seed == 0 and o.max_rounds == 0


def test_workspace_queries_are_monotone(lib):
    o = nanogs.Options()
    lib.nanogs_default_options(ctypes.byref(o))
    a = lib.nanogs_simplify_workspace_bytes(1000, 16, ctypes.byref(o))
    b = lib.nanogs_simplify_workspace_bytes(100000, 16, ctypes.byref(o))
    c = lib.nanogs_simplify_workspace_bytes(100000, 24, ctypes.byref(o))
    assert 0 < a < b < c
    assert lib.nanogs_simplify_workspace_bytes(10, 0, ctypes.byref(o)) == 0
    for fn, args in (("nanogs_knn_workspace_bytes", (5000, 16)),
                     ("nanogs_edges_workspace_bytes", (5000, 16)),
                     ("nanogs_edge_cost_workspace_bytes", (5000, 50000)),
                     ("nanogs_select_workspace_bytes", (5000, 50000)),
                     ("nanogs_merge_workspace_bytes", (5000,))):
        assert getattr(lib, fn)(*args) > 0


def test_bad_arguments_fail_before_any_launch(lib):
    g = nanogs.Gaussians()
    n_out = ctypes.c_int64(-7)
    st = lib.nanogs_simplify(ctypes.byref(g), 0, 1, 16, None, ctypes.byref(g),
                             ctypes.byref(n_out), None, None, 0, None)
    assert st == 1 and b"n must be" in lib.nanogs_last_error()
    st = lib.nanogs_simplify(ctypes.byref(g), 10, 0, 16, None, ctypes.byref(g),
                             ctypes.byref(n_out), None, None, 0, None)
    assert st == 1 and b"target_n" in lib.nanogs_last_error()
    st = lib.nanogs_simplify(ctypes.byref(g), 10, 5, 33, None, ctypes.byref(g),
                             ctypes.byref(n_out), None, None, 0, None)
    assert st == 1 and b"k must be" in lib.nanogs_last_error()
    st = lib.nanogs_simplify(ctypes.byref(g), 10, 5, 16, None, ctypes.byref(g),
                             ctypes.byref(n_out), None, None, 0, None)
    assert st == 1 and b"is null" in lib.nanogs_last_error()
    assert n_out.value == -7
    # misaligned SH pointer
    fake = nanogs.Gaussians(16, 16, 16, 16, 20)
    st = lib.nanogs_simplify(ctypes.byref(fake), 10, 5, 16, None, ctypes.byref(fake),
                             ctypes.byref(n_out), None, None, 0, None)
    assert st == 1 and b"aligned" in lib.nanogs_last_error()
    # bad options
    o = nanogs.Options()
    lib.nanogs_default_options(ctypes.byref(o))
    o.S = 0
    ok = nanogs.Gaussians(256, 512, 768, 1024, 1280)
    out = nanogs.Gaussians(2048, 2304, 2560, 2816, 3072)
    st = lib.nanogs_simplify(ctypes.byref(ok), 10, 5, 16, ctypes.byref(o), ctypes.byref(out),
                             ctypes.byref(n_out), None, None, 0, None)
    assert st == 1 and b"options.S" in lib.nanogs_last_error()
    for bad in (2, 1 << 20, nanogs.TIME_SOME | (1 << nanogs.NTIMED)):
        lib.nanogs_default_options(ctypes.byref(o))
        o.timing = bad
        st = lib.nanogs_simplify(ctypes.byref(ok), 10, 5, 16, ctypes.byref(o), ctypes.byref(out),
                                 ctypes.byref(n_out), None, None, 0, None)
        assert st == 1 and b"options.timing" in lib.nanogs_last_error()
    # the binding's stage selection
    o = nanogs.options(timing=("knn_query", "cost"))
    assert o.timing == nanogs.TIME_SOME | (1 << 2) | (1 << 4)
    assert nanogs.options(timing=True).timing == 1 and nanogs.options().timing == 0
    # workspace too small
    lib.nanogs_default_options(ctypes.byref(o))
    st = lib.nanogs_simplify(ctypes.byref(ok), 10, 5, 16, ctypes.byref(o), ctypes.byref(out),
                             ctypes.byref(n_out), None, ctypes.c_void_p(4096), 16, None)
    assert st == 2 and b"workspace" in lib.nanogs_last_error()
    # n * k limit
    st = lib.nanogs_knn(ctypes.c_void_p(256), 1 << 27, 16, ctypes.c_void_p(256), None, 0, None)
    assert st == 1


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(nanogs, "_lib", None)
    monkeypatch.setattr(nanogs, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        nanogs.load()


def test_engine_size_limit_rejected_before_any_launch(lib):
    """The round engine keeps two int32 adjacency entries per edge and at
    most n * k edges per pass: 2 * n * k must stay below 2^31."""
    ok = nanogs.Gaussians(256, 512, 768, 1024, 1280)
    out = nanogs.Gaussians(2048, 2304, 2560, 2816, 3072)
    n_out = ctypes.c_int64(-7)
    n = 70_000_000  # n * 16 < 2^31, 2 * n * 16 > 2^31
    st = lib.nanogs_simplify(ctypes.byref(ok), n, 10, 16, None, ctypes.byref(out),
                             ctypes.byref(n_out), None, None, 0, None)
    assert st == 1 and b"2 * n * k" in lib.nanogs_last_error()
    b = ctypes.c_void_p()
    st = lib.nanogs_batch_create(60_000_000, 24, 4, None, ctypes.c_void_p(256), 1 << 40, None,
                                 ctypes.byref(b))
    assert st == 1 and b"2 * n * k" in lib.nanogs_last_error() and not b.value
    assert n_out.value == -7
