"""Python binding of libnanogs.so (argument marshalling only).

Every function takes torch tensors that live on the GPU, passes their device
pointers and the current HIP stream to the C ABI of ``include/nanogs.h``, and
raises ``NanoGSError`` on a non-OK status.  All arithmetic runs in the
library's HIP kernels; there is no fallback path: if the library is missing
or no GPU is present these functions raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnanogs.so")

SH = 48
MAX_K = 32
MAX_S = 16
MAX_ROUNDS = 64
PREC_FP32 = 0
PREC_FP64 = 1
COST_MC = 0
COST_STRAT = 1
COST_BOUND = 2
REFRESH_FULL = 0
REFRESH_LOCAL = 1
STAGES = ("precompute", "knn_tree", "knn_query", "edges", "cost", "cost_fp64", "select",
          "merge", "setup", "output", "knn_exact", "knn_wave")
NTIMED = len(STAGES)
TIME_SOME = 0x40000000  # options.timing: the low NTIMED bits select stages

STATUS = {0: "OK", 1: "EINVAL", 2: "EWORKSPACE", 3: "ENONFINITE", 4: "EHIP", 5: "ENOTREADY",
          6: "ENOMEM", 7: "ECANCELLED"}
ECANCELLED = 7


class NanoGSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Gaussians(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("log_scale", ctypes.c_void_p),
                ("rot", ctypes.c_void_p), ("opacity", ctypes.c_void_p),
                ("sh", ctypes.c_void_p)]


class Splats(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("quat", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
                ("sh", ctypes.c_void_p), ("origin", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("app_dims", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("fb_ratio", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("max_rounds", ctypes.c_int32),
                ("d_trace", ctypes.c_void_p), ("d_origin", ctypes.c_void_p),
                ("timing", ctypes.c_int32), ("tau", ctypes.c_float),
                ("cost_mode", ctypes.c_int32), ("refresh", ctypes.c_int32),
                ("pass_frac", ctypes.c_float)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("early_exit", ctypes.c_int32),
                ("n_out", ctypes.c_int64),
                ("n_per_round", ctypes.c_int64 * MAX_ROUNDS),
                ("edges_per_round", ctypes.c_int64 * MAX_ROUNDS),
                ("pairs_per_round", ctypes.c_int64 * MAX_ROUNDS),
                ("fallback_per_round", ctypes.c_int64 * MAX_ROUNDS),
                ("ld_iters_per_round", ctypes.c_int32 * MAX_ROUNDS),
                ("knn_retry_per_round", ctypes.c_int64 * MAX_ROUNDS),
                ("knn_screens_per_round", ctypes.c_int64 * MAX_ROUNDS),
                ("stage_ms", ctypes.c_double * NTIMED),
                ("stage_launches", ctypes.c_int32 * NTIMED),
                ("n_kept", ctypes.c_int64),
                ("requery_per_round", ctypes.c_int64 * MAX_ROUNDS)]

    def as_dict(self):
        r = self.rounds + (1 if self.early_exit else 0)
        r = min(r, MAX_ROUNDS)
        return {"rounds": self.rounds, "early_exit": bool(self.early_exit),
                "n_out": self.n_out,
                "n_per_round": list(self.n_per_round[:r]),
                "edges_per_round": list(self.edges_per_round[:r]),
                "pairs_per_round": list(self.pairs_per_round[:r]),
                "fallback_per_round": list(self.fallback_per_round[:r]),
                "ld_iters_per_round": list(self.ld_iters_per_round[:r]),
                "knn_retry_per_round": list(self.knn_retry_per_round[:r]),
                "knn_screens_per_round": list(self.knn_screens_per_round[:r]),
                "requery_per_round": list(self.requery_per_round[:r]),
                "stage_ms": dict(zip(STAGES, self.stage_ms)),
                "stage_launches": dict(zip(STAGES, self.stage_launches)),
                "n_kept": self.n_kept}


class Tuning(ctypes.Structure):
    _fields_ = [("cost_block", ctypes.c_int32), ("knn_block", ctypes.c_int32),
                ("knn_wave_grid", ctypes.c_int32), ("knn_level_bias", ctypes.c_int32),
                ("select_check", ctypes.c_int32), ("knn_block_min", ctypes.c_int32),
                ("knn_lane_rows", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


TUNE_BUCKETS = 3
TUNE_BUCKET_LIMITS = (65536, 524288, None)  # N below the limit -> bucket
TUNING_FILE = os.path.join(HERE, "tuning_gfx950.json")

_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SZ = ctypes.c_size_t

_SIGS = {
    "nanogs_default_options": (None, [ctypes.POINTER(Options)]),
    "nanogs_last_error": (ctypes.c_char_p, []),
    "nanogs_crn": (None, [ctypes.c_uint64, _I32, _I32, _P]),
    "nanogs_simplify_workspace_bytes": (_SZ, [_I64, _I32, ctypes.POINTER(Options)]),
    "nanogs_simplify": (ctypes.c_int, [ctypes.POINTER(Gaussians), _I64, _I64, _I32,
                                       ctypes.POINTER(Options), ctypes.POINTER(Gaussians),
                                       ctypes.POINTER(_I64), ctypes.POINTER(Stats), _P, _SZ, _P]),
    "nanogs_activate": (ctypes.c_int, [ctypes.POINTER(Gaussians), _I64, ctypes.POINTER(Splats),
                                       _P, _P]),
    "nanogs_deactivate": (ctypes.c_int, [ctypes.POINTER(Splats), _I64,
                                         ctypes.POINTER(Gaussians), _P]),
    "nanogs_knn_workspace_bytes": (_SZ, [_I64, _I32]),
    "nanogs_knn": (ctypes.c_int, [_P, _I64, _I32, _P, _P, _SZ, _P]),
    "nanogs_edges_workspace_bytes": (_SZ, [_I64, _I32]),
    "nanogs_edges": (ctypes.c_int, [_P, _I64, _I32, _P, _P, _P, _P, _SZ, _P]),
    "nanogs_edge_cost_workspace_bytes": (_SZ, [_I64, _I64]),
    "nanogs_edge_cost": (ctypes.c_int, [ctypes.POINTER(Splats), _I64, _P, _P, _I64, _P,
                                        ctypes.POINTER(Options), _P, _P, _P, _SZ, _P]),
    "nanogs_edge_cost_noalloc": (ctypes.c_int, [ctypes.POINTER(Splats), _I64, _P, _P, _I64,
                                                _P, ctypes.POINTER(Options), _P, _P, _P]),
    "nanogs_simplify_lod": (ctypes.c_int, [ctypes.POINTER(Gaussians), _I64, _I64, _I32,
                                           ctypes.POINTER(Options), ctypes.POINTER(Gaussians),
                                           ctypes.POINTER(_I64), ctypes.POINTER(Gaussians), _P,
                                           _I64, ctypes.POINTER(_I64), ctypes.POINTER(_I32),
                                           ctypes.POINTER(Stats), _P, _SZ, _P]),
    "nanogs_prune_workspace_bytes": (_SZ, [_I64]),
    "nanogs_prune": (ctypes.c_int, [ctypes.POINTER(Splats), _I64, ctypes.c_float,
                                    ctypes.POINTER(Splats), _P, _P, _SZ, _P]),
    "nanogs_edge_cost_dev": (ctypes.c_int, [ctypes.POINTER(Splats), _I64, _P, _P, _P, _I64, _P,
                                            ctypes.POINTER(Options), _P, _P, _P, _SZ, _P]),
    "nanogs_select_dev": (ctypes.c_int, [_P, _P, _P, _P, _I64, _I64, _P, _P, _P, _P, _SZ, _P]),
    "nanogs_batch_cancel": (ctypes.c_int, [_P, _I32]),
    "nanogs_select_workspace_bytes": (_SZ, [_I64, _I64]),
    "nanogs_select": (ctypes.c_int, [_P, _P, _P, _I64, _I64, _I64, _P, _P, _P, _SZ, _P]),
    "nanogs_merge_workspace_bytes": (_SZ, [_I64]),
    "nanogs_set_tuning": (ctypes.c_int, [_I32, ctypes.POINTER(Tuning)]),
    "nanogs_get_tuning": (ctypes.c_int, [_I32, ctypes.POINTER(Tuning)]),
    "nanogs_batch_workspace_bytes": (_SZ, [_I64, _I32, _I32]),
    "nanogs_batch_create": (ctypes.c_int, [_I64, _I32, _I32, ctypes.POINTER(Options), _P, _SZ,
                                           _P, ctypes.POINTER(_P)]),
    "nanogs_batch_destroy": (None, [_P]),
    "nanogs_batch_submit": (ctypes.c_int, [_P, ctypes.POINTER(Gaussians), _I64, _I64, _I32,
                                           ctypes.c_uint64, ctypes.POINTER(Gaussians), _P,
                                           ctypes.POINTER(_I32)]),
    "nanogs_batch_step": (ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
    "nanogs_batch_run": (ctypes.c_int, [_P]),
    "nanogs_batch_job": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I64),
                                        ctypes.POINTER(Stats)]),
    "nanogs_batch_rows_in_use": (_I64, [_P]),
    "nanogs_merge": (ctypes.c_int, [ctypes.POINTER(Splats), _I64, _P, ctypes.POINTER(Splats),
                                    _P, _P, _SZ, _P]),
}


def load():
    """Loads the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2603_16103_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    apply_tuning_file(TUNING_FILE)
    return lib


def exported_symbols():
    return list(_SIGS)


def _check(status):
    if status != 0:
        msg = load().nanogs_last_error().decode(errors="replace")
        raise NanoGSError(status, msg)


# ---------------------------------------------------------------------------
# torch plumbing
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes: int):
    torch = _torch()
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


def options(S=1, app_dims=SH, precision=PREC_FP32, fb_ratio=1.0 / 256, seed=0, max_rounds=0,
            d_trace=None, d_origin=None, timing=False, tau=-1.0, cost_mode=COST_MC,
            refresh=REFRESH_FULL, pass_frac=0.0) -> Options:
    """nanogs_options.  timing: False, True (every stage) or stage names
    (STAGES) to time only those stages."""
    o = Options()
    load().nanogs_default_options(ctypes.byref(o))
    o.S, o.app_dims, o.precision, o.fb_ratio = S, app_dims, precision, fb_ratio
    o.seed, o.max_rounds = seed, max_rounds
    o.d_trace = _ptr(d_trace).value if d_trace is not None else None
    o.d_origin = _ptr(d_origin).value if d_origin is not None else None
    if timing is True or timing is False or isinstance(timing, int):
        o.timing = 1 if timing else 0
    else:  # stage names: only those stages are timed
        o.timing = TIME_SOME | sum(1 << STAGES.index(s) for s in set(timing))
    o.tau = tau
    o.cost_mode = cost_mode
    o.refresh = refresh
    o.pass_frac = pass_frac
    return o


@dataclass
class GaussianTensors:
    """Stored-form tensors on the GPU (float32, contiguous)."""

    pos: object        # [n, 3]
    log_scale: object  # [n, 3]
    rot: object        # [n, 4]
    opacity: object    # [n]
    sh: object         # [n, 48]

    @property
    def n(self):
        return int(self.pos.shape[0])

    def struct(self):
        return Gaussians(_ptr(self.pos), _ptr(self.log_scale), _ptr(self.rot),
                         _ptr(self.opacity), _ptr(self.sh))

    @staticmethod
    def empty(n, device="cuda"):
        torch = _torch()
        f = torch.float32
        return GaussianTensors(torch.empty((n, 3), dtype=f, device=device),
                               torch.empty((n, 3), dtype=f, device=device),
                               torch.empty((n, 4), dtype=f, device=device),
                               torch.empty((n,), dtype=f, device=device),
                               torch.empty((n, SH), dtype=f, device=device))

    @staticmethod
    def from_scene(scene, device="cuda"):
        torch = _torch()
        return GaussianTensors(*(torch.from_numpy(x).to(device).contiguous()
                                 for x in (scene.pos, scene.log_scale, scene.rot,
                                           scene.opacity, scene.sh)))

    def slice(self, n):
        return GaussianTensors(self.pos[:n], self.log_scale[:n], self.rot[:n],
                               self.opacity[:n], self.sh[:n])

    def numpy(self):
        return tuple(x.cpu().numpy() for x in (self.pos, self.log_scale, self.rot,
                                               self.opacity, self.sh))


@dataclass
class SplatTensors:
    """Activated tensors on the GPU (float32, contiguous)."""

    mu: object     # [n, 3]
    scale: object  # [n, 3]
    quat: object   # [n, 4]
    alpha: object  # [n]
    sh: object     # [n, 48]
    origin: object = None  # [n] int32

    @property
    def n(self):
        return int(self.mu.shape[0])

    def struct(self):
        return Splats(_ptr(self.mu), _ptr(self.scale), _ptr(self.quat), _ptr(self.alpha),
                      _ptr(self.sh), _ptr(self.origin) if self.origin is not None else None)

    @staticmethod
    def empty(n, with_origin=False, device="cuda"):
        torch = _torch()
        f = torch.float32
        return SplatTensors(torch.empty((n, 3), dtype=f, device=device),
                            torch.empty((n, 3), dtype=f, device=device),
                            torch.empty((n, 4), dtype=f, device=device),
                            torch.empty((n,), dtype=f, device=device),
                            torch.empty((n, SH), dtype=f, device=device),
                            torch.empty((n,), dtype=torch.int32, device=device)
                            if with_origin else None)


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------
def crn(seed: int, round_idx: int, S: int):
    """Host-side shared draws [S, 4] float32 (numpy)."""
    import numpy as np
    out = np.zeros((S, 4), dtype=np.float32)
    load().nanogs_crn(ctypes.c_uint64(seed & ((1 << 64) - 1)), round_idx, S,
                      out.ctypes.data_as(ctypes.c_void_p))
    return out


class Simplifier:
    """Reusable simplify call: keeps the workspace between calls."""

    def __init__(self, n_max: int, k: int = 16, opts: Options | None = None):
        lib = load()
        self.k = k
        self.opts = opts if opts is not None else options()
        self.ws_bytes = lib.nanogs_simplify_workspace_bytes(n_max, k, ctypes.byref(self.opts))
        self.ws = _workspace(self.ws_bytes)
        self.n_max = n_max

    def __call__(self, g: GaussianTensors, target_n: int, out: GaussianTensors,
                 stats: Stats | None = None) -> int:
        if g.n > self.n_max:
            raise ValueError("scene larger than the workspace was sized for")
        lib = load()
        n_out = ctypes.c_int64(0)
        gs, os_ = g.struct(), out.struct()
        _check(lib.nanogs_simplify(ctypes.byref(gs), g.n, target_n, self.k,
                                   ctypes.byref(self.opts), ctypes.byref(os_),
                                   ctypes.byref(n_out),
                                   ctypes.byref(stats) if stats is not None else None,
                                   _ptr(self.ws), self.ws_bytes, _stream()))
        return int(n_out.value)


def simplify(g: GaussianTensors, target_n: int | None = None, k: int = 16,
             ratio: float | None = None, opts: Options | None = None, out=None,
             return_stats: bool = False):
    """Simplifies g to target_n splats (or max(ceil(ratio*n), 1)); returns
    (GaussianTensors of length n_out[, stats dict])."""
    if target_n is None:
        if ratio is None:
            raise ValueError("give target_n or ratio")
        target_n = max(int(math.ceil(ratio * g.n)), 1)
    out = out if out is not None else GaussianTensors.empty(g.n)
    st = Stats()
    n_out = Simplifier(g.n, k, opts)(g, target_n, out, st)
    res = out.slice(n_out)
    return (res, st.as_dict()) if return_stats else res


def simplify_lod(g: GaussianTensors, target_n: int, k: int = 16, opts: Options | None = None,
                 capacity: int | None = None):
    """simplify that also returns the coarse-to-fine hierarchy: (result,
    levels, parents, stats) where levels[r] is the stored-form set at the
    start of pass r (GaussianTensors), parents[r] maps each splat of level r
    to its index in level r+1 (the last level is the result)."""
    torch = _torch()
    lib = load()
    opts = opts if opts is not None else options()
    cap = capacity if capacity is not None else 2 * g.n
    out = GaussianTensors.empty(g.n)
    lod = GaussianTensors.empty(max(cap, 1))
    parent = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    nb = lib.nanogs_simplify_workspace_bytes(g.n, k, ctypes.byref(opts))
    ws = _workspace(nb)
    n_out = ctypes.c_int64(0)
    offs = (ctypes.c_int64 * (MAX_ROUNDS + 1))()
    nlev = ctypes.c_int32(0)
    st = Stats()
    gi, go, gl = g.struct(), out.struct(), lod.struct()
    _check(lib.nanogs_simplify_lod(ctypes.byref(gi), g.n, target_n, k, ctypes.byref(opts),
                                   ctypes.byref(go), ctypes.byref(n_out), ctypes.byref(gl),
                                   _ptr(parent), cap, offs, ctypes.byref(nlev), ctypes.byref(st),
                                   _ptr(ws), nb, _stream()))
    L = int(nlev.value)
    levels = [GaussianTensors(lod.pos[offs[r]:offs[r + 1]], lod.log_scale[offs[r]:offs[r + 1]],
                              lod.rot[offs[r]:offs[r + 1]], lod.opacity[offs[r]:offs[r + 1]],
                              lod.sh[offs[r]:offs[r + 1]]) for r in range(L)]
    parents = [parent[offs[r]:offs[r + 1]] for r in range(L)]
    return out.slice(int(n_out.value)), levels, parents, st.as_dict()


def activate(g: GaussianTensors, s: SplatTensors | None = None, check_finite: bool = True):
    torch = _torch()
    s = s if s is not None else SplatTensors.empty(g.n)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda") if check_finite else None
    gs, ss = g.struct(), s.struct()
    _check(load().nanogs_activate(ctypes.byref(gs), g.n, ctypes.byref(ss), _ptr(flag), _stream()))
    if check_finite and int(flag.item()) != 0:
        raise NanoGSError(3, "input contains a non-finite value")
    return s


def deactivate(s: SplatTensors, g: GaussianTensors | None = None):
    g = g if g is not None else GaussianTensors.empty(s.n)
    ss, gs = s.struct(), g.struct()
    _check(load().nanogs_deactivate(ctypes.byref(ss), s.n, ctypes.byref(gs), _stream()))
    return g


def knn(mu, k: int, ws=None):
    """mu [n,3] float32 cuda -> nbr [n,k] int32.  Reads nothing back."""
    torch = _torch()
    lib = load()
    n = int(mu.shape[0])
    nbr = torch.empty((n, k), dtype=torch.int32, device="cuda")
    nb = lib.nanogs_knn_workspace_bytes(n, k)
    ws = ws if ws is not None else _workspace(nb)
    _check(lib.nanogs_knn(_ptr(mu), n, k, _ptr(nbr), _ptr(ws), nb, _stream()))
    return nbr


def edges(nbr):
    """nbr [n,k] int32 -> (ei, ej) int32 of length m."""
    torch = _torch()
    lib = load()
    n, k = int(nbr.shape[0]), int(nbr.shape[1])
    ei = torch.empty(max(n * k, 1), dtype=torch.int32, device="cuda")
    ej = torch.empty(max(n * k, 1), dtype=torch.int32, device="cuda")
    dm = torch.zeros(1, dtype=torch.int64, device="cuda")
    nb = lib.nanogs_edges_workspace_bytes(n, k)
    ws = _workspace(nb)
    _check(lib.nanogs_edges(_ptr(nbr), n, k, _ptr(ei), _ptr(ej), _ptr(dm), _ptr(ws), nb,
                            _stream()))
    m = int(dm.item())
    return ei[:m], ej[:m]


def edge_cost(s: SplatTensors, ei, ej, crn_block, opts: Options | None = None,
              with_dgeo: bool = False):
    """Cost of edges (ei[e], ej[e]); crn_block is a host [S,4] float32 array."""
    import numpy as np
    torch = _torch()
    lib = load()
    m = int(ei.shape[0])
    opts = opts if opts is not None else options()
    blk = np.ascontiguousarray(crn_block, dtype=np.float32)
    opts.S = int(blk.shape[0])
    cost = torch.empty(max(m, 1), dtype=torch.float32, device="cuda")
    dgeo = torch.empty(max(m, 1), dtype=torch.float32, device="cuda") if with_dgeo else None
    nb = lib.nanogs_edge_cost_workspace_bytes(s.n, m)
    ws = _workspace(nb)
    ss = s.struct()
    _check(lib.nanogs_edge_cost(ctypes.byref(ss), s.n, _ptr(ei), _ptr(ej), m,
                                blk.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts),
                                _ptr(cost), _ptr(dgeo), _ptr(ws), nb, _stream()))
    return (cost[:m], dgeo[:m]) if with_dgeo else cost[:m]


NOALLOC_MAX_N = 131072
NOALLOC_MAX_M = 2097152


def edge_cost_noalloc(s: SplatTensors, ei, ej, crn_block, opts: Options | None = None,
                      cost=None):
    """edge_cost through the entry point that allocates nothing (the library's
    fixed per-GPU scratch); `cost` (float32 [m] on the GPU) may be given so
    that this call allocates nothing either."""
    import numpy as np
    torch = _torch()
    lib = load()
    m = int(ei.shape[0])
    opts = opts if opts is not None else options()
    blk = np.ascontiguousarray(crn_block, dtype=np.float32)
    opts.S = int(blk.shape[0])
    if cost is None:
        cost = torch.empty(max(m, 1), dtype=torch.float32, device="cuda")
    ss = s.struct()
    _check(lib.nanogs_edge_cost_noalloc(ctypes.byref(ss), s.n, _ptr(ei), _ptr(ej), m,
                                        blk.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts),
                                        _ptr(cost), None, _stream()))
    return cost[:m]


def prune(s: SplatTensors, tau: float) -> SplatTensors:
    """Opacity pre-filter: the splats with alpha >= min(tau, median alpha),
    in order (origin carried when s has one)."""
    torch = _torch()
    lib = load()
    out = SplatTensors.empty(s.n, with_origin=s.origin is not None)
    d_n = torch.zeros(1, dtype=torch.int64, device="cuda")
    nb = lib.nanogs_prune_workspace_bytes(s.n)
    ws = _workspace(nb)
    si, so = s.struct(), out.struct()
    _check(lib.nanogs_prune(ctypes.byref(si), s.n, float(tau), ctypes.byref(so), _ptr(d_n),
                            _ptr(ws), nb, _stream()))
    k = int(d_n.item())
    return SplatTensors(out.mu[:k], out.scale[:k], out.quat[:k], out.alpha[:k], out.sh[:k],
                        out.origin[:k] if out.origin is not None else None)


def select(ei, ej, cost, n: int, max_pairs: int):
    """Greedy disjoint pairs -> (partner [n] int32, npairs)."""
    torch = _torch()
    lib = load()
    m = int(ei.shape[0])
    partner = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    dn = torch.zeros(1, dtype=torch.int64, device="cuda")
    nb = lib.nanogs_select_workspace_bytes(n, m)
    ws = _workspace(nb)
    _check(lib.nanogs_select(_ptr(ei) if m else None, _ptr(ej) if m else None,
                             _ptr(cost) if m else None, m, n, max_pairs, _ptr(partner), _ptr(dn),
                             _ptr(ws), nb, _stream()))
    return partner[:n], int(dn.item())


def edge_cost_dev(s: SplatTensors, ei, ej, d_m, d_crn, opts: Options | None = None, ws=None):
    """edge_cost with the edge count on the device: d_m int64 [1] cuda,
    ei/ej of capacity m_cap >= *d_m, d_crn float32 [S,4] cuda.  Returns cost
    [m_cap] (entries at and past *d_m untouched).  Reads nothing back, so it
    may be captured into a CUDA/HIP graph (pass ws to avoid allocating)."""
    torch = _torch()
    lib = load()
    m_cap = int(ei.shape[0])
    opts = opts if opts is not None else options()
    opts.S = int(d_crn.shape[0])
    cost = torch.empty(max(m_cap, 1), dtype=torch.float32, device="cuda")
    nb = lib.nanogs_edge_cost_workspace_bytes(s.n, m_cap)
    ws = ws if ws is not None else _workspace(nb)
    ss = s.struct()
    _check(lib.nanogs_edge_cost_dev(ctypes.byref(ss), s.n, _ptr(ei), _ptr(ej), _ptr(d_m), m_cap,
                                    _ptr(d_crn), ctypes.byref(opts), _ptr(cost), None, _ptr(ws),
                                    nb, _stream()))
    return cost[:m_cap]


def select_dev(ei, ej, cost, d_m, n: int, d_max_pairs, ws=None):
    """select with the edge count and the budget on the device (int64 [1]
    cuda tensors) -> (partner [n] int32, d_npairs int64 [1] cuda).  Reads
    nothing back."""
    torch = _torch()
    lib = load()
    m_cap = int(ei.shape[0])
    partner = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    dn = torch.empty(1, dtype=torch.int64, device="cuda")
    nb = lib.nanogs_select_workspace_bytes(n, m_cap)
    ws = ws if ws is not None else _workspace(nb)
    _check(lib.nanogs_select_dev(_ptr(ei), _ptr(ej), _ptr(cost), _ptr(d_m), m_cap, n,
                                 _ptr(d_max_pairs), _ptr(partner), _ptr(dn), _ptr(ws), nb,
                                 _stream()))
    return partner[:n], dn


def edges_dev(nbr, ws=None):
    """edges with the count left on the device: (ei, ej) of capacity n*k and
    d_m (int64 [1] cuda).  Reads nothing back."""
    torch = _torch()
    lib = load()
    n, k = int(nbr.shape[0]), int(nbr.shape[1])
    ei = torch.empty(max(n * k, 1), dtype=torch.int32, device="cuda")
    ej = torch.empty(max(n * k, 1), dtype=torch.int32, device="cuda")
    dm = torch.empty(1, dtype=torch.int64, device="cuda")
    nb = lib.nanogs_edges_workspace_bytes(n, k)
    ws = ws if ws is not None else _workspace(nb)
    _check(lib.nanogs_edges(_ptr(nbr), n, k, _ptr(ei), _ptr(ej), _ptr(dm), _ptr(ws), nb,
                            _stream()))
    return ei, ej, dm


def merge_dev(s: SplatTensors, partner, ws=None):
    """merge with the new count left on the device: (SplatTensors of capacity
    n, d_nout int64 [1] cuda).  Reads nothing back."""
    torch = _torch()
    lib = load()
    out = SplatTensors.empty(s.n, with_origin=s.origin is not None)
    dn = torch.empty(1, dtype=torch.int64, device="cuda")
    nb = lib.nanogs_merge_workspace_bytes(s.n)
    ws = ws if ws is not None else _workspace(nb)
    si, so = s.struct(), out.struct()
    _check(lib.nanogs_merge(ctypes.byref(si), s.n, _ptr(partner), ctypes.byref(so), _ptr(dn),
                            _ptr(ws), nb, _stream()))
    return out, dn


def merge(s: SplatTensors, partner):
    """MPMM merge + compaction -> SplatTensors of the new count."""
    torch = _torch()
    lib = load()
    out = SplatTensors.empty(s.n, with_origin=s.origin is not None)
    dn = torch.zeros(1, dtype=torch.int64, device="cuda")
    nb = lib.nanogs_merge_workspace_bytes(s.n)
    ws = _workspace(nb)
    si, so = s.struct(), out.struct()
    _check(lib.nanogs_merge(ctypes.byref(si), s.n, _ptr(partner), ctypes.byref(so), _ptr(dn),
                            _ptr(ws), nb, _stream()))
    k = int(dn.item())
    return SplatTensors(out.mu[:k], out.scale[:k], out.quat[:k], out.alpha[:k], out.sh[:k],
                        out.origin[:k] if out.origin is not None else None)


# ---------------------------------------------------------------------------
# batched / served form
# ---------------------------------------------------------------------------
JOB_QUEUED, JOB_RUNNING, JOB_DONE = 0, 1, 2


def batch_workspace_bytes(max_rows: int, max_k: int, max_jobs: int) -> int:
    return int(load().nanogs_batch_workspace_bytes(max_rows, max_k, max_jobs))


class Batch:
    """Many simplification jobs in one working set (nanogs_batch_*).

    Jobs are submitted with their own device input/output tensors, join at
    pass boundaries while rows are free, and leave when done.  step() runs
    one pass for every job in the working set; run() steps until all jobs
    are done.  Bound to the stream current at construction."""

    def __init__(self, max_rows: int, max_k: int = 32, max_jobs: int = 64,
                 opts: Options | None = None):
        lib = load()
        self.opts = opts if opts is not None else options()
        self.ws_bytes = batch_workspace_bytes(max_rows, max_k, max_jobs)
        if self.ws_bytes == 0:
            raise ValueError("bad batch sizes")
        self.ws = _workspace(self.ws_bytes)
        self._h = ctypes.c_void_p()
        self._stream = _stream()
        _check(lib.nanogs_batch_create(max_rows, max_k, max_jobs, ctypes.byref(self.opts),
                                       _ptr(self.ws), self.ws_bytes, self._stream,
                                       ctypes.byref(self._h)))
        self._keep = {}  # job id -> tensors that must stay alive
        self.max_rows = max_rows

    def close(self):
        if self._h:
            load().nanogs_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass

    def submit(self, g: GaussianTensors, target_n: int, k: int = 16, seed: int = 0,
               out: GaussianTensors | None = None, origin=None) -> int:
        out = out if out is not None else GaussianTensors.empty(g.n)
        gs, os_ = g.struct(), out.struct()
        jid = ctypes.c_int32(-1)
        _check(load().nanogs_batch_submit(self._h, ctypes.byref(gs), g.n, target_n, k,
                                          ctypes.c_uint64(seed & ((1 << 64) - 1)),
                                          ctypes.byref(os_), _ptr(origin), ctypes.byref(jid)))
        self._keep[jid.value] = (g, out, origin)
        return jid.value

    def cancel(self, jid: int):
        """Cancels a queued or running job (state -ECANCELLED); no effect on
        a finished one.  Its tensors are kept until release()."""
        _check(load().nanogs_batch_cancel(self._h, jid))

    def step(self) -> int:
        d = ctypes.c_int32(0)
        _check(load().nanogs_batch_step(self._h, ctypes.byref(d)))
        return d.value

    def run(self):
        _check(load().nanogs_batch_run(self._h))

    def job(self, jid: int):
        """(state, n_out, stats dict); state 0 queued, 1 running, 2 done,
        negative: failed with that status."""
        st = ctypes.c_int32(0)
        n = ctypes.c_int64(0)
        stats = Stats()
        _check(load().nanogs_batch_job(self._h, jid, ctypes.byref(st), ctypes.byref(n),
                                       ctypes.byref(stats)))
        return st.value, int(n.value), stats.as_dict()

    def result(self, jid: int) -> GaussianTensors:
        state, n, _ = self.job(jid)
        if state != JOB_DONE:
            raise NanoGSError(-state if state < 0 else 5, f"job {jid} is not done")
        return self._keep[jid][1].slice(n)

    def release(self, jid: int):
        """Drops the binding's references to a finished job's tensors."""
        self._keep.pop(jid, None)

    def rows_in_use(self) -> int:
        return int(load().nanogs_batch_rows_in_use(self._h))


# ---------------------------------------------------------------------------
# launch shapes
# ---------------------------------------------------------------------------
def get_tuning(bucket: int) -> dict:
    t = Tuning()
    _check(load().nanogs_get_tuning(bucket, ctypes.byref(t)))
    return t.as_dict()


def set_tuning(bucket: int, **values):
    """Sets launch parameters of one bucket (-1: all); unspecified fields keep
    their current values.  Results do not depend on these values."""
    lib = load()
    cur = get_tuning(0 if bucket < 0 else bucket)
    cur.update(values)
    t = Tuning(**cur)
    _check(lib.nanogs_set_tuning(bucket, ctypes.byref(t)))


def apply_tuning_file(path: str) -> bool:
    """Applies a tuning table written by paper_2603_16103_amd.tune (if the
    file exists and was tuned for this architecture)."""
    import json
    try:
        with open(path) as fh:
            tab = json.load(fh)
    except (OSError, ValueError):
        return False
    if tab.get("arch") != "gfx950":
        return False
    for b, vals in enumerate(tab.get("buckets", [])[:TUNE_BUCKETS]):
        t = Tuning()
        _check(_lib.nanogs_get_tuning(b, ctypes.byref(t)))  # fields the table lacks keep theirs
        for f, _ in Tuning._fields_:
            if f in vals:
                setattr(t, f, int(vals[f]))
        _check(_lib.nanogs_set_tuning(b, ctypes.byref(t)))
    return True

