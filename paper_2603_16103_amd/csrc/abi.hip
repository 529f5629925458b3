// C ABI entry points: argument checks, workspace layout, and the round driver
// of Algorithm 1 (kNN graph -> union edges -> edge costs -> greedy disjoint
// pairs -> merge, until the target count or a pass without pairs).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/nanogs.h"
#include "engine.h"

namespace ng {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }

namespace {

nanogs_status read_opts(const nanogs_options* o, Opts* out) {
  Opts r;
  if (o) {
    r.S = o->S;
    r.app_dims = o->app_dims;
    r.precision = o->precision;
    r.fb_ratio = o->fb_ratio;
    r.seed = o->seed;
    r.max_rounds = o->max_rounds;
    r.d_trace = o->d_trace;
    r.d_origin = o->d_origin;
    r.timing = o->timing;
    r.tau = o->tau;
    r.cost_mode = o->cost_mode;
    r.refresh = o->refresh;
    r.pass_frac = o->pass_frac;
  }
  if (r.S < 1 || r.S > NANOGS_MAX_S) {
    set_error("options.S must be in [1, 16]");
    return NANOGS_EINVAL;
  }
  if (r.app_dims < 0 || r.app_dims > NG_SH) {
    set_error("options.app_dims must be in [0, 48]");
    return NANOGS_EINVAL;
  }
  if (r.precision != NANOGS_PREC_FP32 && r.precision != NANOGS_PREC_FP64) {
    set_error("options.precision must be NANOGS_PREC_FP32 or NANOGS_PREC_FP64");
    return NANOGS_EINVAL;
  }
  if (!(r.fb_ratio >= 0.0f && r.fb_ratio <= 1.0f)) {
    set_error("options.fb_ratio must be in [0, 1]");
    return NANOGS_EINVAL;
  }
  if (r.max_rounds < 0) {
    set_error("options.max_rounds must be >= 0");
    return NANOGS_EINVAL;
  }
  if (r.timing != 0 && r.timing != 1 &&
      ((r.timing & ~(NANOGS_TIME_SOME | ((1 << NANOGS_NTIMED) - 1))) != 0 ||
       (r.timing & NANOGS_TIME_SOME) == 0)) {
    set_error("options.timing must be 0, 1 or NANOGS_TIME_SOME with stage bits");
    return NANOGS_EINVAL;
  }
  if (std::isnan(r.tau) || std::isinf(r.tau)) {
    set_error("options.tau must be finite (< 0 turns the opacity pre-filter off)");
    return NANOGS_EINVAL;
  }
  if (r.cost_mode != NANOGS_COST_MC && r.cost_mode != NANOGS_COST_STRAT &&
      r.cost_mode != NANOGS_COST_BOUND) {
    set_error("options.cost_mode must be NANOGS_COST_MC, NANOGS_COST_STRAT or NANOGS_COST_BOUND");
    return NANOGS_EINVAL;
  }
  if (r.refresh != NANOGS_REFRESH_FULL && r.refresh != NANOGS_REFRESH_LOCAL) {
    set_error("options.refresh must be NANOGS_REFRESH_FULL or NANOGS_REFRESH_LOCAL");
    return NANOGS_EINVAL;
  }
  if (!(r.pass_frac >= 0.0f && r.pass_frac <= 1.0f)) {
    set_error("options.pass_frac must be in [0, 1]");
    return NANOGS_EINVAL;
  }
  *out = r;
  return NANOGS_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

nanogs_status check_ptr(const void* p, size_t align, const char* name) {
  if (!p) {
    set_error(std::string(name) + " is null");
    return NANOGS_EINVAL;
  }
  if (!aligned(p, align)) {
    set_error(std::string(name) + " is not " + std::to_string(align) + "-byte aligned");
    return NANOGS_EINVAL;
  }
  return NANOGS_OK;
}

#define NG_CHECK(expr)                     \
  do {                                     \
    nanogs_status _s = (expr);             \
    if (_s != NANOGS_OK) return _s;        \
  } while (0)

nanogs_status check_gaussians(const nanogs_gaussians* g, const char* name) {
  if (!g) {
    set_error(std::string(name) + " is null");
    return NANOGS_EINVAL;
  }
  NG_CHECK(check_ptr(g->pos, 4, "pos"));
  NG_CHECK(check_ptr(g->log_scale, 4, "log_scale"));
  NG_CHECK(check_ptr(g->rot, 4, "rot"));
  NG_CHECK(check_ptr(g->opacity, 4, "opacity"));
  NG_CHECK(check_ptr(g->sh, 16, "sh"));
  return NANOGS_OK;
}

nanogs_status check_splats(const nanogs_splats* s, const char* name) {
  if (!s) {
    set_error(std::string(name) + " is null");
    return NANOGS_EINVAL;
  }
  NG_CHECK(check_ptr(s->mu, 4, "mu"));
  NG_CHECK(check_ptr(s->scale, 4, "scale"));
  NG_CHECK(check_ptr(s->quat, 4, "quat"));
  NG_CHECK(check_ptr(s->alpha, 4, "alpha"));
  NG_CHECK(check_ptr(s->sh, 16, "sh"));
  return NANOGS_OK;
}

nanogs_status check_n(long long n, long long k) {
  if (n < 0) {
    set_error("n must be >= 0");
    return NANOGS_EINVAL;
  }
  if (k < 1 || k > NANOGS_MAX_K) {
    set_error("k must be in [1, 32]");
    return NANOGS_EINVAL;
  }
  if (n * k >= (1ll << 31) - 1) {
    set_error("n * k must be below 2^31");
    return NANOGS_EINVAL;
  }
  return NANOGS_OK;
}

// The round engine's adjacency holds two entries per edge (one at each end)
// with int32 offsets, and a pass has at most n * k edges.
nanogs_status check_engine_n(long long n, long long k) {
  NG_CHECK(check_n(n, k));
  if (2 * n * k >= (1ll << 31) - 1) {
    set_error("2 * n * k must be below 2^31 (int32 adjacency offsets)");
    return NANOGS_EINVAL;
  }
  return NANOGS_OK;
}

nanogs_status check_ws(void* ws, size_t have, size_t need) {
  if (need == 0) return NANOGS_OK;
  if (!ws || have < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes, got " +
              std::to_string(have));
    return NANOGS_EWORKSPACE;
  }
  if (!aligned(ws, 256)) {
    set_error("workspace must be 256-byte aligned");
    return NANOGS_EINVAL;
  }
  return NANOGS_OK;
}

template <class F>
nanogs_status guarded(F&& f) {
  try {
    g_error.clear();
    return f();
  } catch (const HipError& e) {
    set_error(e.msg);
    return e.code == hipErrorOutOfMemory ? NANOGS_ENOMEM : NANOGS_EHIP;
  } catch (const std::bad_alloc& e) {
    set_error(std::string("host allocation failed: ") + e.what());
    return NANOGS_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return NANOGS_EHIP;
  }
}

// ---------------------------------------------------------------------------
// simplify: one job on an engine sized for it
// ---------------------------------------------------------------------------
// Stored-form copy of the splats the opacity pre-filter keeps, and the input
// index of each.
struct PrunedInput {
  nanogs_gaussians g;
  int* kept;
  void* temp;
};

PrunedInput take_pruned(void* base, long long n, size_t* bytes) {
  Carver c(base);
  PrunedInput p;
  p.g.pos = c.take<float>(3 * n);
  p.g.log_scale = c.take<float>(3 * n);
  p.g.rot = c.take<float>(4 * n);
  p.g.opacity = c.take<float>(n);
  p.g.sh = c.take<float>(NG_SH * n);
  p.kept = c.take<int>(n);
  p.temp = base ? (char*)base + c.bytes() : nullptr;
  if (bytes) *bytes = c.bytes() + prune_temp_bytes(n);
  return p;
}

size_t simplify_bytes(long long n, int k, bool prune) {
  if (n < 1) n = 1;
  size_t b = Engine::workspace_bytes(n, k, 1);
  if (prune) {
    size_t pb = 0;
    take_pruned(nullptr, n, &pb);
    b += pb + 256;
  }
  return b;
}

struct LodOut {
  nanogs_gaussians* lod = nullptr;
  int32_t* parent = nullptr;
  long long cap = 0;
  int64_t* offsets = nullptr;
  int32_t* levels = nullptr;
};

nanogs_status run_simplify(const nanogs_gaussians* in, long long n, long long target_n, int k,
                           const Opts& o, nanogs_gaussians* out, int64_t* n_out,
                           nanogs_stats* stats, void* ws, hipStream_t st,
                           const LodOut& lod = LodOut()) {
  thread_local StageTimer T;
  T.begin_call(o.timing, st);
  // opacity pre-filter (Algorithm 1, before the loop): the loop runs on the
  // survivors; provenance is mapped back to input indices at the end
  nanogs_gaussians src = *in;
  long long n_run = n;
  const int* kept = nullptr;
  if (o.tau >= 0.0f) {
    const size_t eb = Engine::workspace_bytes(n < 2 ? 2 : n, k, 1);
    PrunedInput pin = take_pruned((char*)ws + ((eb + 255) & ~(size_t)255), n, nullptr);
    bool nonfinite = false;
    n_run = prune_stored(in->pos, in->log_scale, in->rot, in->opacity, in->sh, (int)n, o.tau,
                         pin.g.pos, pin.g.log_scale, pin.g.rot, pin.g.opacity, pin.g.sh, pin.kept,
                         &nonfinite, pin.temp, st);
    if (nonfinite) {
      set_error("input contains a non-finite value");
      return NANOGS_ENONFINITE;
    }
    src = pin.g;
    kept = pin.kept;
  }
  Engine E(n, k, 1, o, ws, st);
  JobSpec js;
  js.in = src;
  js.out = *out;
  js.n = n_run;
  js.target = target_n;
  js.k = k;
  js.seed = o.seed;
  js.d_origin = o.d_origin;
  js.d_trace = o.d_trace;
  long long lod_offsets[NANOGS_MAX_ROUNDS + 1] = {0};
  if (lod.lod) {
    js.lod = *lod.lod;
    js.lod_parent = lod.parent;
    js.lod_cap = lod.cap;
    js.lod_offsets = lod_offsets;
  }
  const int id = E.submit(js);
  E.run(&T);
  if (lod.lod) {
    const int lv = E.job(id).lod_levels;
    *lod.levels = lv;
    for (int r = 0; r <= lv; ++r) lod.offsets[r] = lod_offsets[r];
  }
  nanogs_stats local = E.job(id).stats;
  T.collect(local.stage_ms, local.stage_launches);
  const Job& j = E.job(id);
  if (j.state == JOB_FAILED) {
    set_error(j.error);
    if (stats) *stats = local;
    return (nanogs_status)j.status;
  }
  local.n_out = j.stats.n_out;
  local.n_kept = n_run;
  *n_out = j.stats.n_out;
  if (kept) {
    if (o.d_origin) remap_indices(o.d_origin, j.stats.n_out, kept, st);
    if (o.d_trace) {
      long long traced = 0;
      for (int r = 0; r < j.stats.rounds && r < NANOGS_MAX_ROUNDS; ++r)
        traced += j.stats.pairs_per_round[r];
      remap_indices(o.d_trace, 2 * traced, kept, st);
    }
    NG_HIP(hipStreamSynchronize(st));
  }
  if (stats) *stats = local;
  return NANOGS_OK;
}

// ---------------------------------------------------------------------------
// stage workspaces
// ---------------------------------------------------------------------------
struct Packed {
  float4* cen;
  int* lg;
  float4* shp;
  int* org;
};

Packed take_packed(Carver& c, long long n) {
  Packed p;
  p.cen = c.take<float4>(n);
  p.lg = c.take<int>(n);
  p.shp = c.take<float4>(2 * n);
  p.org = c.take<int>(n);
  return p;
}

size_t cost_bytes(long long n, long long m) {
  Carver c(nullptr);
  take_packed(c, n);
  c.take<float4>(pre_float4s(n));
  c.take<int>(m);
  c.take<int>(64);
  c.take<float>(NG_CRN_ROW);
  return c.bytes();
}

size_t merge_ws_bytes(long long n) {
  Carver c(nullptr);
  take_packed(c, n);
  take_packed(c, n);
  c.take<int>(64);
  return c.bytes() + merge_temp_bytes(n);
}

}  // namespace
}  // namespace ng

using namespace ng;

struct nanogs_batch {
  Engine* eng;
  Opts opts;
  int kmax;
};

extern "C" {

void nanogs_default_options(nanogs_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->S = 1;
  opt->app_dims = NANOGS_SH_COEFFS;
  opt->precision = NANOGS_PREC_FP32;
  opt->fb_ratio = 1.0f / 256.0f;
  opt->seed = 0;
  opt->max_rounds = 0;
  opt->timing = 0;
  opt->tau = -1.0f;
  opt->cost_mode = NANOGS_COST_MC;
  opt->refresh = NANOGS_REFRESH_FULL;
  opt->pass_frac = 0.0f;
}

const char* nanogs_last_error(void) { return g_error.c_str(); }

void nanogs_crn(uint64_t seed, int32_t round, int32_t S, float* out) {
  if (!out || S <= 0) return;
  crn_host(seed, round, S, out);
}

size_t nanogs_simplify_workspace_bytes(int64_t n, int32_t k, const nanogs_options* opt) {
  (void)opt;
  if (n < 1 || k < 1 || k > NANOGS_MAX_K) return 0;
  return simplify_bytes(n, k, opt && opt->tau >= 0.0f);
}

nanogs_status nanogs_simplify(const nanogs_gaussians* in, int64_t n, int64_t target_n, int32_t k,
                              const nanogs_options* opt, nanogs_gaussians* out, int64_t* n_out,
                              nanogs_stats* stats, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    if (n < 1) {
      set_error("n must be >= 1");
      return NANOGS_EINVAL;
    }
    if (target_n < 1) {
      set_error("target_n must be >= 1");
      return NANOGS_EINVAL;
    }
    if (!n_out) {
      set_error("n_out is null");
      return NANOGS_EINVAL;
    }
    NG_CHECK(check_engine_n(n, k));
    NG_CHECK(check_gaussians(in, "in"));
    NG_CHECK(check_gaussians(out, "out"));
    if (in->pos == out->pos || in->sh == out->sh) {
      set_error("in and out may not alias");
      return NANOGS_EINVAL;
    }
    Opts o;
    NG_CHECK(read_opts(opt, &o));
    NG_CHECK(check_ws(ws, ws_bytes, simplify_bytes(n, k, o.tau >= 0.0f)));
    return run_simplify(in, n, target_n, k, o, out, n_out, stats, ws, stream);
  });
}

nanogs_status nanogs_simplify_lod(const nanogs_gaussians* in, int64_t n, int64_t target_n,
                                  int32_t k, const nanogs_options* opt, nanogs_gaussians* out,
                                  int64_t* n_out, nanogs_gaussians* lod, int32_t* lod_parent,
                                  int64_t lod_capacity, int64_t* lod_offsets,
                                  int32_t* lod_levels, nanogs_stats* stats, void* ws,
                                  size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    if (n < 1 || target_n < 1) {
      set_error("n and target_n must be >= 1");
      return NANOGS_EINVAL;
    }
    if (!n_out || !lod_offsets || !lod_levels) {
      set_error("n_out, lod_offsets and lod_levels (host) must not be null");
      return NANOGS_EINVAL;
    }
    if (lod_capacity < 0) {
      set_error("lod_capacity must be >= 0");
      return NANOGS_EINVAL;
    }
    NG_CHECK(check_engine_n(n, k));
    NG_CHECK(check_gaussians(in, "in"));
    NG_CHECK(check_gaussians(out, "out"));
    NG_CHECK(check_gaussians(lod, "lod"));
    NG_CHECK(check_ptr(lod_parent, 4, "lod_parent"));
    if (in->pos == out->pos || in->sh == out->sh || lod->pos == in->pos || lod->pos == out->pos) {
      set_error("in, out and lod may not alias");
      return NANOGS_EINVAL;
    }
    Opts o;
    NG_CHECK(read_opts(opt, &o));
    NG_CHECK(check_ws(ws, ws_bytes, simplify_bytes(n, k, o.tau >= 0.0f)));
    LodOut lo;
    lo.lod = lod;
    lo.parent = lod_parent;
    lo.cap = lod_capacity;
    lo.offsets = lod_offsets;
    lo.levels = lod_levels;
    return run_simplify(in, n, target_n, k, o, out, n_out, stats, ws, stream, lo);
  });
}

nanogs_status nanogs_activate(const nanogs_gaussians* g, int64_t n, nanogs_splats* s,
                              int32_t* d_nonfinite, hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    NG_CHECK(check_n(n, 1));
    if (n == 0) return NANOGS_OK;
    NG_CHECK(check_gaussians(g, "g"));
    NG_CHECK(check_splats(s, "s"));
    launch_activate_plain(g->pos, g->log_scale, g->rot, g->opacity, (int)n, s->mu, s->scale,
                          s->quat, s->alpha, d_nonfinite, stream);
    if (d_nonfinite) launch_check_finite(g->sh, n * NG_SH, d_nonfinite, stream);
    if (s->sh != g->sh)
      NG_HIP(hipMemcpyAsync(s->sh, g->sh, n * NG_SH * sizeof(float), hipMemcpyDeviceToDevice,
                            stream));
    return NANOGS_OK;
  });
}

nanogs_status nanogs_deactivate(const nanogs_splats* s, int64_t n, nanogs_gaussians* g,
                                hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    NG_CHECK(check_n(n, 1));
    if (n == 0) return NANOGS_OK;
    NG_CHECK(check_splats(s, "s"));
    NG_CHECK(check_gaussians(g, "g"));
    launch_deactivate_plain(s->mu, s->scale, s->quat, s->alpha, (int)n, g->pos, g->log_scale,
                            g->rot, g->opacity, stream);
    if (s->sh != g->sh)
      NG_HIP(hipMemcpyAsync(g->sh, s->sh, n * NG_SH * sizeof(float), hipMemcpyDeviceToDevice,
                            stream));
    return NANOGS_OK;
  });
}

size_t nanogs_knn_workspace_bytes(int64_t n, int32_t k) {
  return knn_plain_bytes(n < 1 ? 1 : n, k < 1 ? 1 : (k > NANOGS_MAX_K ? NANOGS_MAX_K : k));
}

nanogs_status nanogs_knn(const float* mu, int64_t n, int32_t k, int32_t* nbr, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    NG_CHECK(check_n(n, k));
    if (n == 0) return NANOGS_OK;
    NG_CHECK(check_ptr(mu, 4, "mu"));
    NG_CHECK(check_ptr(nbr, 4, "nbr"));
    NG_CHECK(check_ws(ws, ws_bytes, knn_plain_bytes(n, k)));
    if (n == 1) {
      fill_i32(nbr, -1, k, stream);
      return NANOGS_OK;
    }
    const int keff = (int)std::min<long long>(k, n - 1);
    knn_plain(mu, (int)n, k, keff, nbr, ws, stream);
    return NANOGS_OK;
  });
}

size_t nanogs_edges_workspace_bytes(int64_t n, int32_t k) {
  if (n < 1) n = 1;
  if (k < 1) k = 1;
  return edges_public_bytes(n, k);
}

nanogs_status nanogs_edges(const int32_t* nbr, int64_t n, int32_t k, int32_t* ei, int32_t* ej,
                           int64_t* d_m, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    NG_CHECK(check_n(n, k));
    NG_CHECK(check_ptr(d_m, 8, "d_m"));
    if (n == 0) {
      set_i64((long long*)d_m, 0, stream);
      return NANOGS_OK;
    }
    NG_CHECK(check_ptr(nbr, 4, "nbr"));
    NG_CHECK(check_ptr(ei, 4, "ei"));
    NG_CHECK(check_ptr(ej, 4, "ej"));
    NG_CHECK(check_ws(ws, ws_bytes, edges_public_bytes(n, k)));
    union_edges_public(nbr, (int)n, k, ei, ej, (long long*)d_m, ws, stream);
    return NANOGS_OK;
  });
}

size_t nanogs_edge_cost_workspace_bytes(int64_t n, int64_t m) {
  return cost_bytes(n < 1 ? 1 : n, m < 1 ? 1 : m);
}

}  // extern "C"

namespace {

nanogs_status check_edge_cost_args(const nanogs_splats* s, int64_t n, const int32_t* ei,
                                   const int32_t* ej, int64_t m, const float* crn,
                                   const nanogs_options* opt, float* cost, Opts* o) {
  NG_CHECK(check_n(n, 1));
  if (m < 0 || m >= (1ll << 31)) {
    set_error("m must be in [0, 2^31)");
    return NANOGS_EINVAL;
  }
  NG_CHECK(read_opts(opt, o));
  if (m == 0) return NANOGS_OK;
  NG_CHECK(check_splats(s, "s"));
  NG_CHECK(check_ptr(ei, 4, "ei"));
  NG_CHECK(check_ptr(ej, 4, "ej"));
  NG_CHECK(check_ptr(crn, 4, "crn"));
  NG_CHECK(check_ptr(cost, 4, "cost"));
  return NANOGS_OK;
}

// The stage's launches over scratch memory ws of cost_bytes(n, m) bytes.
// With d_m (device int64) the edge count is *d_m clamped to m, which then
// only bounds it, and crn is a device array; otherwise crn is host memory.
void edge_cost_run(const nanogs_splats* s, int64_t n, const int32_t* ei, const int32_t* ej,
                   int64_t m, const float* crn, const Opts& o, float* cost, float* dgeo,
                   void* ws, hipStream_t stream, const int64_t* d_m = nullptr) {
    Carver c(ws);
    Packed p = take_packed(c, n);
    float4* pre = c.take<float4>(pre_float4s(n));
    int* fb_list = c.take<int>(m);
    int* counters = c.take<int>(64);  // [0] fallback count, [2] edge count (d_m)
    float* dcrn = c.take<float>(NG_CRN_ROW);
    const int* mcount = nullptr;
    if (d_m) {
      count_to_i32((const long long*)d_m, m, counters + 2, stream);
      mcount = counters + 2;
    } else {
      NG_HIP(hipMemcpyAsync(dcrn, crn, sizeof(float) * 4 * o.S, hipMemcpyHostToDevice, stream));
    }
    const CrnTab args{d_m ? crn : dcrn, o.S, nullptr, nullptr, o.cost_mode};
    launch_pack_splats(s->mu, s->scale, s->quat, s->alpha, s->origin, (int)n, p.cen, p.lg, p.shp,
                       p.org, stream);
    if (o.precision == NANOGS_PREC_FP64) {
      launch_edge_cost_fp64(p.cen, p.shp, s->sh, o.app_dims, ei, ej, (int)n, false, nullptr,
                            mcount, (int)m, args, cost, dgeo, AdjOut{}, stream);
    } else {
      launch_precompute(p.shp, (int)n, pre, stream);
      fill_i32(counters, 0, 1, stream);
      launch_edge_cost(p.cen, pre, s->sh, o.app_dims, ei, ej, (int)m, (int)n, false, args,
                       o.fb_ratio, cost, dgeo, fb_list, counters, AdjOut{}, stream, mcount);
      launch_edge_cost_fp64(p.cen, p.shp, s->sh, o.app_dims, ei, ej, (int)n, false, fb_list,
                            counters, (int)m, args, cost, dgeo, AdjOut{}, stream);
    }
}

// Scratch of the allocation-free edge-cost entry point: one array per GPU,
// in the library's code object (it lives as long as the process).  Host code
// never uses the symbol's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kScratchBytes = (size_t)32 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_ptr() {
  int dev = 0;
  NG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw HipError{"device index out of range"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    NG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

nanogs_status nanogs_edge_cost(const nanogs_splats* s, int64_t n, const int32_t* ei,
                               const int32_t* ej, int64_t m, const float* crn,
                               const nanogs_options* opt, float* cost, float* dgeo, void* ws,
                               size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    Opts o;
    NG_CHECK(check_edge_cost_args(s, n, ei, ej, m, crn, opt, cost, &o));
    if (m == 0) return NANOGS_OK;
    NG_CHECK(check_ws(ws, ws_bytes, cost_bytes(n, m)));
    edge_cost_run(s, n, ei, ej, m, crn, o, cost, dgeo, ws, stream);
    return NANOGS_OK;
  });
}

nanogs_status nanogs_edge_cost_dev(const nanogs_splats* s, int64_t n, const int32_t* ei,
                                   const int32_t* ej, const int64_t* d_m, int64_t m_cap,
                                   const float* d_crn, const nanogs_options* opt, float* cost,
                                   float* dgeo, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    Opts o;
    NG_CHECK(check_edge_cost_args(s, n, ei, ej, m_cap, d_crn, opt, cost, &o));
    NG_CHECK(check_ptr(d_m, 8, "d_m"));
    if (m_cap == 0) return NANOGS_OK;
    NG_CHECK(check_ws(ws, ws_bytes, cost_bytes(n, m_cap)));
    edge_cost_run(s, n, ei, ej, m_cap, d_crn, o, cost, dgeo, ws, stream, d_m);
    return NANOGS_OK;
  });
}

nanogs_status nanogs_edge_cost_noalloc(const nanogs_splats* s, int64_t n, const int32_t* ei,
                                       const int32_t* ej, int64_t m, const float* crn,
                                       const nanogs_options* opt, float* cost, float* dgeo,
                                       hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    Opts o;
    NG_CHECK(check_edge_cost_args(s, n, ei, ej, m, crn, opt, cost, &o));
    if (m == 0) return NANOGS_OK;
    if (n > NANOGS_NOALLOC_MAX_N || m > NANOGS_NOALLOC_MAX_M ||
        cost_bytes(n, m) > kScratchBytes) {
      set_error("nanogs_edge_cost_noalloc: n must be <= " +
                std::to_string(NANOGS_NOALLOC_MAX_N) + " and m <= " +
                std::to_string(NANOGS_NOALLOC_MAX_M) + " (fixed scratch of " +
                std::to_string(kScratchBytes >> 20) + " MiB)");
      return NANOGS_EINVAL;
    }
    edge_cost_run(s, n, ei, ej, m, crn, o, cost, dgeo, scratch_ptr(), stream);
    return NANOGS_OK;
  });
}

size_t nanogs_select_workspace_bytes(int64_t n, int64_t m) {
  if (n < 1) n = 1;
  if (m < 1) m = 1;
  return select_adj_bytes(n, m) + select_temp_bytes(n, m, 1) + 256;
}

nanogs_status nanogs_select(const int32_t* ei, const int32_t* ej, const float* cost, int64_t m,
                            int64_t n, int64_t max_pairs, int32_t* partner, int64_t* d_npairs,
                            void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    NG_CHECK(check_n(n, 1));
    if (m < 0 || m >= (1ll << 30)) {
      set_error("m must be in [0, 2^30)");
      return NANOGS_EINVAL;
    }
    if (max_pairs < 0) {
      set_error("max_pairs must be >= 0");
      return NANOGS_EINVAL;
    }
    NG_CHECK(check_ptr(d_npairs, 8, "d_npairs"));
    if (n == 0) {
      set_i64((long long*)d_npairs, 0, stream);
      return NANOGS_OK;
    }
    NG_CHECK(check_ptr(partner, 4, "partner"));
    if (m > 0) {
      NG_CHECK(check_ptr(ei, 4, "ei"));
      NG_CHECK(check_ptr(ej, 4, "ej"));
      NG_CHECK(check_ptr(cost, 4, "cost"));
    }
    const long long mm = m < 1 ? 1 : m;
    NG_CHECK(check_ws(ws, ws_bytes, select_adj_bytes(n, mm) + select_temp_bytes(n, mm, 1)));
    Adjacency adj;
    build_adjacency(ei, ej, cost, m, (int)n, &adj, ws, stream);
    void* temp = (char*)ws + select_adj_bytes(n, mm);
    const long long P = max_pairs;
    select_pairs(adj, (int)n, nullptr, nullptr, 1, &P, partner, temp, stream,
                 (long long*)d_npairs, nullptr);
    return NANOGS_OK;
  });
}

nanogs_status nanogs_select_dev(const int32_t* ei, const int32_t* ej, const float* cost,
                                const int64_t* d_m, int64_t m_cap, int64_t n,
                                const int64_t* d_max_pairs, int32_t* partner, int64_t* d_npairs,
                                void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    NG_CHECK(check_n(n, 1));
    if (m_cap < 0 || m_cap >= (1ll << 30)) {
      set_error("m_cap must be in [0, 2^30)");
      return NANOGS_EINVAL;
    }
    NG_CHECK(check_ptr(d_m, 8, "d_m"));
    NG_CHECK(check_ptr(d_max_pairs, 8, "d_max_pairs"));
    NG_CHECK(check_ptr(d_npairs, 8, "d_npairs"));
    if (n == 0) {
      set_i64((long long*)d_npairs, 0, stream);
      return NANOGS_OK;
    }
    NG_CHECK(check_ptr(partner, 4, "partner"));
    if (m_cap > 0) {
      NG_CHECK(check_ptr(ei, 4, "ei"));
      NG_CHECK(check_ptr(ej, 4, "ej"));
      NG_CHECK(check_ptr(cost, 4, "cost"));
    }
    const long long mm = m_cap < 1 ? 1 : m_cap;
    const size_t body = select_adj_bytes(n, mm) + select_temp_bytes(n, mm, 1);
    NG_CHECK(check_ws(ws, ws_bytes, body + 256));
    int* mcount = (int*)((char*)ws + body);
    count_to_i32((const long long*)d_m, m_cap, mcount, stream);
    Adjacency adj;
    build_adjacency(ei, ej, cost, m_cap, (int)n, &adj, ws, stream, mcount);
    void* temp = (char*)ws + select_adj_bytes(n, mm);
    select_pairs(adj, (int)n, nullptr, nullptr, 1, nullptr, partner, temp, stream,
                 (long long*)d_npairs, nullptr, (const long long*)d_max_pairs);
    return NANOGS_OK;
  });
}

size_t nanogs_merge_workspace_bytes(int64_t n) { return merge_ws_bytes(n < 1 ? 1 : n); }

nanogs_status nanogs_merge(const nanogs_splats* in, int64_t n, const int32_t* partner,
                           nanogs_splats* out, int64_t* d_nout, void* ws, size_t ws_bytes,
                           hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    NG_CHECK(check_n(n, 1));
    NG_CHECK(check_ptr(d_nout, 8, "d_nout"));
    if (n == 0) {
      set_i64((long long*)d_nout, 0, stream);
      return NANOGS_OK;
    }
    NG_CHECK(check_splats(in, "in"));
    NG_CHECK(check_splats(out, "out"));
    NG_CHECK(check_ptr(partner, 4, "partner"));
    if (in->sh == out->sh || in->mu == out->mu) {
      set_error("in and out may not alias");
      return NANOGS_EINVAL;
    }
    NG_CHECK(check_ws(ws, ws_bytes, merge_ws_bytes(n)));
    Carver c(ws);
    Packed a = take_packed(c, n);
    Packed b = take_packed(c, n);
    int* dcount = c.take<int>(64);
    void* temp = (char*)ws + c.bytes();
    launch_pack_splats(in->mu, in->scale, in->quat, in->alpha, in->origin, (int)n, a.cen, a.lg,
                       a.shp, a.org, stream);
    // the new count stays on the device (no host read: capturable)
    merge_compact(a.cen, nullptr, a.shp, in->sh, a.org, (int)n, partner, b.cen, b.lg, b.shp,
                  out->sh, b.org, nullptr, temp, stream, dcount, nullptr, nullptr, nullptr, 1,
                  nullptr, false);
    launch_unpack_splats(b.cen, b.shp, b.org, (int)n, out->mu, out->scale, out->quat,
                         out->alpha, (in->origin && out->origin) ? out->origin : nullptr, stream,
                         dcount);
    widen_i32(dcount, (long long*)d_nout, stream);
    return NANOGS_OK;
  });
}

size_t nanogs_prune_workspace_bytes(int64_t n) { return prune_temp_bytes(n < 1 ? 1 : n); }

nanogs_status nanogs_prune(const nanogs_splats* in, int64_t n, float tau, nanogs_splats* out,
                           int64_t* d_nout, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> nanogs_status {
    NG_CHECK(check_n(n, 1));
    NG_CHECK(check_ptr(d_nout, 8, "d_nout"));
    if (std::isnan(tau) || std::isinf(tau)) {
      set_error("tau must be finite");
      return NANOGS_EINVAL;
    }
    if (n == 0) {
      set_i64((long long*)d_nout, 0, stream);
      return NANOGS_OK;
    }
    NG_CHECK(check_splats(in, "in"));
    NG_CHECK(check_splats(out, "out"));
    if (in->sh == out->sh || in->mu == out->mu) {
      set_error("in and out may not alias");
      return NANOGS_EINVAL;
    }
    NG_CHECK(check_ws(ws, ws_bytes, prune_temp_bytes(n)));
    prune_splats(in->mu, in->scale, in->quat, in->alpha, in->sh, in->origin, (int)n, tau, out->mu,
                 out->scale, out->quat, out->alpha, out->sh,
                 (in->origin && out->origin) ? out->origin : nullptr, (long long*)d_nout, ws,
                 stream);
    return NANOGS_OK;
  });
}

// ---- batched and served form ----------------------------------------------

size_t nanogs_batch_workspace_bytes(int64_t max_rows, int32_t max_k, int32_t max_jobs) {
  if (max_rows < 1 || max_k < 1 || max_k > NANOGS_MAX_K || max_jobs < 1) return 0;
  return Engine::workspace_bytes(max_rows, max_k, max_jobs);
}

nanogs_status nanogs_batch_create(int64_t max_rows, int32_t max_k, int32_t max_jobs,
                                  const nanogs_options* opt, void* ws, size_t ws_bytes,
                                  hipStream_t stream, nanogs_batch** out) {
  return guarded([&]() -> nanogs_status {
    if (!out) {
      set_error("out is null");
      return NANOGS_EINVAL;
    }
    *out = nullptr;
    if (max_rows < 1 || max_jobs < 1 || max_jobs > 4096) {
      set_error("max_rows must be >= 1 and max_jobs in [1, 4096]");
      return NANOGS_EINVAL;
    }
    NG_CHECK(check_engine_n(max_rows, max_k));
    Opts o;
    NG_CHECK(read_opts(opt, &o));
    if (o.d_trace || o.d_origin) {
      set_error("batch options take no trace/origin buffers (origin is per job)");
      return NANOGS_EINVAL;
    }
    if (o.tau >= 0.0f) {
      set_error("the opacity pre-filter (options.tau) is applied by nanogs_simplify and "
                "nanogs_prune, not by batches");
      return NANOGS_EINVAL;
    }
    if (o.refresh != NANOGS_REFRESH_FULL) {
      set_error("the local neighbourhood refresh (options.refresh) is applied by "
                "nanogs_simplify, not by batches");
      return NANOGS_EINVAL;
    }
    NG_CHECK(check_ws(ws, ws_bytes, Engine::workspace_bytes(max_rows, max_k, max_jobs)));
    nanogs_batch* b = new nanogs_batch;
    b->eng = new Engine(max_rows, max_k, max_jobs, o, ws, stream);
    b->opts = o;
    b->kmax = max_k;
    *out = b;
    return NANOGS_OK;
  });
}

void nanogs_batch_destroy(nanogs_batch* b) {
  if (!b) return;
  delete b->eng;
  delete b;
}

nanogs_status nanogs_batch_submit(nanogs_batch* b, const nanogs_gaussians* in, int64_t n,
                                  int64_t target_n, int32_t k, uint64_t seed,
                                  nanogs_gaussians* out, int32_t* d_origin, int32_t* job_id) {
  return guarded([&]() -> nanogs_status {
    if (!b || !job_id) {
      set_error("batch or job_id is null");
      return NANOGS_EINVAL;
    }
    if (n < 1 || n > b->eng->capacity()) {
      set_error("n must be in [1, max_rows]");
      return NANOGS_EINVAL;
    }
    if (target_n < 1) {
      set_error("target_n must be >= 1");
      return NANOGS_EINVAL;
    }
    if (k < 1 || k > b->kmax) {
      set_error("k must be in [1, max_k]");
      return NANOGS_EINVAL;
    }
    NG_CHECK(check_gaussians(in, "in"));
    NG_CHECK(check_gaussians(out, "out"));
    if (in->pos == out->pos || in->sh == out->sh) {
      set_error("in and out may not alias");
      return NANOGS_EINVAL;
    }
    if (d_origin) NG_CHECK(check_ptr(d_origin, 4, "d_origin"));
    JobSpec js;
    js.in = *in;
    js.out = *out;
    js.n = n;
    js.target = target_n;
    js.k = k;
    js.seed = seed;
    js.d_origin = d_origin;
    *job_id = b->eng->submit(js);
    return NANOGS_OK;
  });
}

nanogs_status nanogs_batch_cancel(nanogs_batch* b, int32_t job_id) {
  return guarded([&]() -> nanogs_status {
    if (!b || job_id < 0 || job_id >= b->eng->num_jobs()) {
      set_error("bad batch or job id");
      return NANOGS_EINVAL;
    }
    b->eng->cancel(job_id);
    return NANOGS_OK;
  });
}

nanogs_status nanogs_batch_step(nanogs_batch* b, int32_t* n_done) {
  return guarded([&]() -> nanogs_status {
    if (!b) {
      set_error("batch is null");
      return NANOGS_EINVAL;
    }
    const int d = b->eng->step(nullptr);
    if (n_done) *n_done = d;
    return NANOGS_OK;
  });
}

nanogs_status nanogs_batch_run(nanogs_batch* b) {
  return guarded([&]() -> nanogs_status {
    if (!b) {
      set_error("batch is null");
      return NANOGS_EINVAL;
    }
    b->eng->run(nullptr);
    return NANOGS_OK;
  });
}

nanogs_status nanogs_batch_job(const nanogs_batch* b, int32_t job_id, int32_t* state,
                               int64_t* n_out, nanogs_stats* stats) {
  if (!b || !state || job_id < 0 || job_id >= b->eng->num_jobs()) {
    set_error("bad batch, job id or state pointer");
    return NANOGS_EINVAL;
  }
  const Job& j = b->eng->job(job_id);
  switch (j.state) {
    case JOB_QUEUED: *state = 0; break;
    case JOB_RUNNING: *state = 1; break;
    case JOB_DRAINING:
    case JOB_DONE: *state = 2; break;
    default: *state = -j.status; break;
  }
  if (n_out) *n_out = (j.state == JOB_DRAINING || j.state == JOB_DONE) ? j.stats.n_out : 0;
  if (stats) *stats = j.stats;
  return NANOGS_OK;
}

int64_t nanogs_batch_rows_in_use(const nanogs_batch* b) { return b ? b->eng->rows_in_use() : 0; }

// ---- launch shapes ---------------------------------------------------------

nanogs_status nanogs_set_tuning(int32_t bucket, const nanogs_tuning* t) {
  if (!t || bucket < -1 || bucket >= NANOGS_TUNE_BUCKETS) {
    set_error("bad bucket or null tuning");
    return NANOGS_EINVAL;
  }
  const bool ok = (t->cost_block == 64 || t->cost_block == 128 || t->cost_block == 256) &&
                  (t->knn_block == 64 || t->knn_block == 128 || t->knn_block == 256) &&
                  t->knn_wave_grid >= 256 && t->knn_wave_grid <= 65536 &&
                  t->knn_level_bias >= -2 && t->knn_level_bias <= 1 && t->select_check >= 1 &&
                  t->select_check <= 16 && t->knn_block_min >= 17 && t->knn_block_min <= 1024 &&
                  t->knn_lane_rows >= 64 && t->knn_lane_rows <= 4096;
  if (!ok) {
    set_error("tuning value out of range");
    return NANOGS_EINVAL;
  }
  Tuning v;
  v.cost_block = t->cost_block;
  v.knn_block = t->knn_block;
  v.knn_wave_grid = t->knn_wave_grid;
  v.knn_level_bias = t->knn_level_bias;
  v.select_check = t->select_check;
  v.knn_block_min = t->knn_block_min;
  v.knn_lane_rows = t->knn_lane_rows;
  for (int b = 0; b < NANOGS_TUNE_BUCKETS; ++b)
    if (bucket < 0 || bucket == b) set_tuning(b, v);
  return NANOGS_OK;
}

nanogs_status nanogs_get_tuning(int32_t bucket, nanogs_tuning* t) {
  if (!t || bucket < 0 || bucket >= NANOGS_TUNE_BUCKETS) {
    set_error("bad bucket or null tuning");
    return NANOGS_EINVAL;
  }
  const long long rep = bucket == 0 ? 1 : bucket == 1 ? 65536 : 524288;
  const Tuning& v = tuning_for(rep);
  t->cost_block = v.cost_block;
  t->knn_block = v.knn_block;
  t->knn_wave_grid = v.knn_wave_grid;
  t->knn_level_bias = v.knn_level_bias;
  t->select_check = v.select_check;
  t->knn_block_min = v.knn_block_min;
  t->knn_lane_rows = v.knn_lane_rows;
  return NANOGS_OK;
}

}  // extern "C"

