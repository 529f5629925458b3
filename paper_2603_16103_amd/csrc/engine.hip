// Round driver of Algorithm 1 for one or many scenes at once.
//
// The engine keeps every live scene ("job") as a segment of one working set
// (rows [row0, row0 + N) of each scene, which are also its logical indices;
// see internal.h).  One step is one pass of Algorithm 1 for every live
// segment together, one launch per stage:
//   precompute -> cell tables -> kNN -> union edges -> edge costs (+ FP64
//   fallback) -> greedy pairs with a budget P = N - N_tgt per segment ->
//   merge + compaction (rows re-sorted by (segment, Morton key)).
// Jobs queued with submit() join at the next step when their rows fit; a job
// whose segment reaches its target (or finds no pair) is written to its
// output buffers in the stored form at the end of that step, and its rows are
// dropped by the next compaction.  Each job's draws are keyed by its own
// (seed, pass), so a job's result does not depend on what else is in the
// batch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nanogs.h"
#include "engine.h"

namespace ng {

namespace {

__global__ void k_iota_e(int* v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// The counts of a pass, gathered into one block for a single readback:
// out[0] edges, [1] order violation flag, [2] kNN retries, [3] kNN float
// screens, [4] rows re-queried by the local refresh, [5] FP64-fallback
// edges, [6] iterations of the matching's finish, [8 + s] pairs kept by
// segment s.  The kNN's statistics are taken right after the search (the
// temporary area that holds them is reused), the rest after the selection.
__global__ void k_stats_knn(const int* __restrict__ unsorted, const int* __restrict__ kc,
                            const int* __restrict__ dcount, long long* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[1] = *unsorted;
    out[2] = kc[1];
    long long s = 0;
    for (int i = 0; i < kScreenSlots; ++i)
      s += *(const long long*)(kc + kScreenBase + i * kScreenStride);
    out[3] = s;
    out[4] = dcount ? *dcount : 0;
  }
}

__global__ void k_stats_select(const int* __restrict__ m, const int* __restrict__ fb,
                               const int* __restrict__ tail, const int* __restrict__ mseg,
                               int nseg, long long* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    out[0] = *m;
    out[5] = *fb;
    out[6] = *tail;
  }
  if (i < nseg) out[8 + i] = mseg[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
namespace {

Work take_work_e(Carver& c, long long n) {
  Work w;
  w.cen = c.take<float4>(n);
  w.lg = c.take<int>(n);
  w.shp = c.take<float4>(2 * n);
  w.sh = c.take<float>(n * NG_SH);
  w.org = c.take<int>(n);
  w.sg = c.take<int>(n);
  return w;
}

long long table_bound(long long rows, int jobs) {
  // per segment: 8^LT + 1 entries with LT at most one level above the
  // smallest level with 8^L >= n (8^L < 8n), and LT <= 8
  const long long by_rows = 64 * rows + 72ll * jobs;
  const long long by_cap = (long long)jobs * ((1ll << 24) + 1);
  return std::min(by_rows, by_cap) + 16ll * jobs + 16;
}

}  // namespace

struct EngineWs {
  Work w[2];
  float4* pre;
  int* nbr;
  int* src;
  int* tgt;
  int* islot;
  int* eoff;
  int* ioff;
  int* aoff;
  float* cost;
  unsigned long long* akey;
  int* au;
  int* fb_list;
  int* partner;
  int* nbr_log;  // local refresh: last lists by logical index, parent map, scratch
  int* parent;
  int* pcount;
  int* dlist;
  unsigned* keys;
  int* perm;
  int* counters;
  long long* stats;  // a pass's counts (k_stats_knn / k_stats_select)
  SegInfo* seg;
  float* crn;
  long long* budget;  // pairs allowed this pass, per segment
  unsigned* boxes;  // [jobs][8]
  void* temp;
  size_t bytes;
};

static_assert((sizeof(SegInfo) + NG_CRN_ROW * sizeof(float)) % alignof(long long) == 0,
              "the budgets of the staging layout must be aligned");
static size_t stage_bytes(int J) {
  return (size_t)J * (sizeof(SegInfo) + NG_CRN_ROW * sizeof(float) + sizeof(long long)) + 256;
}

static EngineWs carve_engine(void* base, long long R, int K, int J) {
  Carver c(base);
  EngineWs s;
  s.w[0] = take_work_e(c, R);
  s.w[1] = take_work_e(c, R);
  s.pre = c.take<float4>(pre_float4s(R));
  s.nbr = c.take<int>(R * K);
  s.src = c.take<int>(R * K);
  s.tgt = c.take<int>(R * K);
  s.islot = c.take<int>(R * K);
  s.eoff = c.take<int>(R + 1);
  s.ioff = c.take<int>(R + 1);
  s.aoff = c.take<int>(R + 1);
  s.cost = c.take<float>(R * K);
  s.akey = c.take<unsigned long long>(2 * R * K);
  s.au = c.take<int>(2 * R * K);
  s.fb_list = c.take<int>(R * K);
  s.partner = c.take<int>(R);
  s.nbr_log = c.take<int>(R * K);
  s.parent = c.take<int>(R);
  s.pcount = c.take<int>(R);
  s.dlist = c.take<int>(R);
  s.keys = c.take<unsigned>(R);
  s.perm = c.take<int>(R);
  s.counters = c.take<int>(64);
  s.stats = c.take<long long>(8 + (size_t)J);
  // segment table, draws and budgets in the page-locked staging layout, so
  // one copy uploads all three
  char* up = c.take<char>(stage_bytes(J));
  s.seg = (SegInfo*)up;
  s.crn = (float*)(up + (size_t)J * sizeof(SegInfo));
  s.budget = (long long*)(up + (size_t)J * (sizeof(SegInfo) + NG_CRN_ROW * sizeof(float)));
  s.boxes = c.take<unsigned>((size_t)J * 8);
  s.temp = base ? (char*)base + c.bytes() : nullptr;
  size_t kb = 0;
  carve_knn(nullptr, R, table_bound(R, J), K, &kb);
  size_t t = sort_temp_bytes(R);
  t = std::max(t, kb);
  t = std::max(t, edges_temp_bytes(R, K));
  t = std::max(t, select_temp_bytes(R, R * K, J));
  t = std::max(t, merge_temp_bytes(R));
  s.bytes = c.bytes() + t + 4096;
  return s;
}

size_t Engine::workspace_bytes(long long rows, int kmax, int jobs) {
  if (rows < 2) rows = 2;
  return carve_engine(nullptr, rows, kmax, jobs).bytes;
}


Engine::Engine(long long rows, int kmax, int jobs, const Opts& o, void* ws, hipStream_t st)
    : R_(rows < 2 ? 2 : rows), K_(kmax), J_(jobs), o_(o), st_(st) {
  W_ = new EngineWs(carve_engine(ws, R_, K_, J_));
  NG_HIP(hipHostMalloc((void**)&stage_, stage_bytes(J_), hipHostMallocDefault));
  NG_HIP(hipHostMalloc((void**)&hb_, (16 + (size_t)J_) * sizeof(long long),
                       hipHostMallocDefault));
}

Engine::~Engine() {
  (void)hipHostFree(stage_);
  (void)hipHostFree(hb_);
  delete W_;
}

int Engine::submit(const JobSpec& spec) {
  Job j;
  j.spec = spec;
  j.id = (int)jobs_.size();
  j.N = spec.n;
  std::memset(&j.stats, 0, sizeof(j.stats));
  jobs_.push_back(j);
  queue_.push_back(j.id);
  return j.id;
}

long long Engine::rows_in_use() const { return Ntot_; }

bool Engine::cancel(int id) {
  Job& j = jobs_[id];
  if (j.state == JOB_QUEUED) {
    queue_.erase(std::find(queue_.begin(), queue_.end(), id));
  } else if (j.state != JOB_RUNNING) {
    return false;
  }
  // a running job stays in live_ until the next pass, which treats every
  // segment that is not running as rows to drop
  j.state = JOB_FAILED;
  j.status = NANOGS_ECANCELLED;
  j.error = "cancelled";
  return true;
}

// ---------------------------------------------------------------------------
// job set-up: Morton order of the job's centres, activation into rows
// [Ntot, Ntot + n) of the working set, SH rows, non-finite check
// ---------------------------------------------------------------------------
bool Engine::setup_job(Job& j, int pos) {
  EngineWs& W = *W_;
  const long long n = j.spec.n;
  const Work& a = W.w[cur_];
  unsigned* box = W.boxes + 8 * (size_t)pos;  // scratch for the bounds
  long long* host = pinned_host();
  launch_morton_keys(j.spec.in.pos, nullptr, (int)n, W.keys, box, st_);
  k_iota_e<<<blocks_for(n, 256), 256, 0, st_>>>(W.perm, (int)n);
  NG_LAUNCH_CHECK();
  sort_pairs_u32(W.keys, W.perm, n, kSortKeyBits, W.temp, st_);
  fill_i32(W.counters, 0, 1, st_);
  const long long r0 = Ntot_;
  launch_activate_stored(j.spec.in.pos, j.spec.in.log_scale, j.spec.in.rot, j.spec.in.opacity,
                         W.perm, (int)n, (int)r0, a.cen + r0, a.lg + r0, a.shp + 2 * r0, a.org + r0,
                         a.sg + r0, pos, W.counters, st_,
                         // (the other working set is free between passes: its
                         // first n rows hold the rows in input order)
                         W.w[cur_ ^ 1].cen, W.w[cur_ ^ 1].shp);
  // the SH rows are checked for non-finite values while they are copied
  launch_copy_sh_rows(j.spec.in.sh, W.perm, a.sh + r0 * NG_SH, nullptr, 0, (int)n, st_,
                      W.counters);
  NG_HIP(hipMemcpyAsync(host, W.counters, sizeof(int), hipMemcpyDeviceToHost, st_));
  NG_HIP(hipMemcpyAsync(host + 1, box, 6 * sizeof(unsigned), hipMemcpyDeviceToHost, st_));
  NG_HIP(hipStreamSynchronize(st_));
  std::memcpy(j.box, host + 1, 6 * sizeof(unsigned));
  if (*(int*)host != 0) {
    j.state = JOB_FAILED;
    j.status = NANOGS_ENONFINITE;
    j.error = "input contains a non-finite value";
    return false;
  }
  j.row0 = r0;
  j.state = JOB_RUNNING;
  Ntot_ += n;
  return true;
}

// Writes job j's rows [row0, row0 + N) of working set w to its outputs.
void Engine::finish_job(Job& j, const Work& w) {
  const long long r0 = j.row0, N = j.N;
  launch_deactivate_work(w.cen + r0, w.lg + r0, w.shp + 2 * r0, w.org + r0, (int)N, (int)r0,
                         j.spec.out.pos, j.spec.out.log_scale, j.spec.out.rot, j.spec.out.opacity,
                         j.spec.d_origin, st_);
  launch_copy_sh_rows(w.sh + r0 * NG_SH, nullptr, j.spec.out.sh, w.lg + r0, (int)r0, (int)N, st_);
  j.stats.n_out = N;
  j.state = JOB_DRAINING;
}

// ---------------------------------------------------------------------------
// one pass
// ---------------------------------------------------------------------------
int Engine::step(StageTimer* T) {
  EngineWs& W = *W_;
  int tk;
  int finished = 0;

  // 1. admit queued jobs whose rows fit (in submission order)
  tk = T ? T->start(NANOGS_T_SETUP) : -1;
  while (!queue_.empty()) {
    Job& j = jobs_[queue_.front()];
    if (j.spec.n > R_) {
      queue_.erase(queue_.begin());
      j.state = JOB_FAILED;
      j.status = NANOGS_EINVAL;
      j.error = "job larger than the batch capacity";
      ++finished;
      continue;
    }
    if (Ntot_ + j.spec.n > R_ || (int)live_.size() >= J_) break;
    queue_.erase(queue_.begin());
    const int pos = (int)live_.size();
    if (!setup_job(j, pos)) {
      ++finished;
      continue;
    }
    live_.push_back(j.id);
    if (j.N <= j.spec.target || j.N <= 1) {
      finish_job(j, W.w[cur_]);
      ++finished;
    }
  }
  if (T) T->stop(tk);

  // 2. segment table: searching segments (running), draining ones (rows
  // dropped by this pass's compaction).  The table, the draws and the
  // budgets go up from page-locked memory: no copy here waits for the
  // device (the last pass ended with a synchronisation, so the device has
  // read the previous contents).
  SegInfo* hs = (SegInfo*)stage_;
  float* hcrn = (float*)(stage_ + (size_t)J_ * sizeof(SegInfo));
  long long* hP = (long long*)(stage_ + (size_t)J_ * (sizeof(SegInfo) + NG_CRN_ROW * sizeof(float)));
  for (size_t i = 0; i < live_.size(); ++i) hP[i] = 0;
  long long entries = 0;
  unsigned class_mask = 0u;
  int searching = 0, next = 0;
  for (size_t i = 0; i < live_.size(); ++i) {
    const Job& j = jobs_[live_[i]];
    SegInfo& S = hs[i];
    std::memset(&S, 0, sizeof(S));
    std::memcpy(S.box, j.box, sizeof(S.box));
    S.row0 = (int)j.row0;
    S.nrows = (int)j.N;
    S.crn = (int)i;
    // a segment without a table keeps the next table's offset (the cell
    // table build orders rows by it)
    S.toff = (int)entries;
    if (j.state == JOB_RUNNING) {
      S.LT = table_level(j.N);
      entries += table_entries(S.LT);
      S.keff = (int)std::min<long long>(std::max(1, j.spec.k), j.N - 1);
      S.kclass = kclass_of(S.keff);
      class_mask |= class_bit(S.kclass);
      S.next = next++;
      hP[i] = j.N - j.spec.target;
      if (o_.pass_frac > 0.0f) {
        // progressive collapses: at most max(1, floor(f N)) pairs per pass
        const long long cap = (long long)std::floor((double)o_.pass_frac * (double)j.N);
        hP[i] = std::min(hP[i], std::max(1ll, cap));
      }
      ++searching;
    } else {
      S.next = -1;
    }
  }
  if (live_.empty()) return finished;
  const int nseg = (int)live_.size();
  if (searching == 0) {
    // only draining segments: the working set empties
    Ntot_ = 0;
    live_.clear();
    for (Job& j : jobs_)
      if (j.state == JOB_DRAINING) j.state = JOB_DONE;
    NG_HIP(hipStreamSynchronize(st_));
    return finished;
  }
  // draws of every segment's current pass
  std::memset(hcrn, 0, (size_t)nseg * NG_CRN_ROW * sizeof(float));
  for (int i = 0; i < nseg; ++i) {
    const Job& j = jobs_[live_[i]];
    crn_host(j.spec.seed, j.round, o_.S, &hcrn[(size_t)i * NG_CRN_ROW]);
  }
  // one upload: the segment table, the draws and the budgets (the device
  // block has the staging layout; the slots past nseg go up unused)
  NG_HIP(hipMemcpyAsync(W.seg, stage_, (char*)(hP + nseg) - (char*)stage_, hipMemcpyHostToDevice,
                        st_));

  const Work& a = W.w[cur_];
  const Work& b = W.w[cur_ ^ 1];
  const long long N = Ntot_;
  const int* sg = a.sg;

  tk = T ? T->start(NANOGS_T_PRECOMPUTE) : -1;
  launch_precompute(a.shp, (int)N, W.pre, st_);
  if (T) T->stop(tk);
  tk = T ? T->start(NANOGS_T_KNN_TREE) : -1;
  // counters [1] FP64-fallback edges, [2] the row order flag
  fill_i32(W.counters + 1, 0, 2, st_);
  knn_build(a.cen, (int)N, sg, W.seg, entries, W.temp, W.counters + 2, st_);
  if (T) T->stop(tk);
  // local neighbourhood refresh (one scene): from the second pass on, only
  // the splats a merge touched are queried
  Job* j1 = (nseg == 1 && searching == 1) ? &jobs_[live_[0]] : nullptr;
  const bool refresh_local = o_.refresh == NANOGS_REFRESH_LOCAL && j1;
  const bool incremental = refresh_local && j1->round > 0 && j1->prev_n > 0 &&
                           j1->prev_keff == hs[0].keff;
  int* dcount = W.counters + 16;
  if (incremental) {
    knn_refresh(a.cen, (int)N, (int)j1->prev_n, K_, hs[0].keff, sg, W.seg, entries, W.temp,
                W.parent, W.pcount, W.nbr_log, W.dlist, dcount, W.nbr, T, st_);
  } else {
    knn_query(a.cen, (int)N, K_, sg, W.seg, class_mask, entries, W.temp, true, 0, W.nbr, T, st_);
  }
  if (refresh_local) knn_save_log(a.lg, W.nbr, (int)N, K_, hs[0].keff, W.nbr_log, st_);
  // the kNN's statistics live in the temporary area the next stages reuse
  k_stats_knn<<<1, 64, 0, st_>>>(W.counters + 2, carve_knn(W.temp, N, entries, K_, nullptr).counters,
                                 incremental ? dcount : nullptr, W.stats);
  NG_LAUNCH_CHECK();
  tk = T ? T->start(NANOGS_T_EDGES) : -1;
  const EdgeSet es{W.src, W.tgt, W.eoff, W.ioff, W.islot, W.aoff};
  launch_union_edges(W.nbr, a.lg, (int)N, K_, es, nullptr, W.temp, st_);
  if (T) T->stop(tk);
  // the edge count stays on the device (eoff[N], at most N * k): the cost
  // launches cover N * k edges and read it there
  const int m_cap = (int)(N * K_);
  const int* mcount = W.eoff + N;

  const CrnTab ct{W.crn, o_.S, sg, W.seg, o_.cost_mode};
  const AdjOut adj_out{W.eoff, W.ioff, W.islot, W.akey, W.au};
  int* fb_count = W.counters + 1;  // (zeroed with the order flag)
  if (o_.precision == NANOGS_PREC_FP64) {
    tk = T ? T->start(NANOGS_T_COST_FP64) : -1;
    launch_edge_cost_fp64(a.cen, a.shp, a.sh, o_.app_dims, W.src, W.tgt, (int)N, true, nullptr,
                          mcount, m_cap, ct, W.cost, nullptr, adj_out, st_);
    if (T) T->stop(tk);
  } else {
    tk = T ? T->start(NANOGS_T_COST) : -1;
    launch_edge_cost(a.cen, W.pre, a.sh, o_.app_dims, W.src, W.tgt, m_cap, (int)N, true, ct,
                     o_.fb_ratio, W.cost, nullptr, W.fb_list, fb_count, adj_out, st_, mcount);
    if (T) T->stop(tk);
    tk = T ? T->start(NANOGS_T_COST_FP64) : -1;
    launch_edge_cost_fp64(a.cen, a.shp, a.sh, o_.app_dims, W.src, W.tgt, (int)N, true, W.fb_list,
                          fb_count, m_cap, ct, W.cost, nullptr, adj_out, st_);
    if (T) T->stop(tk);
  }

  tk = T ? T->start(NANOGS_T_SELECT) : -1;
  const Adjacency adj{W.aoff, W.akey, W.au};
  const int* d_mseg = nullptr;
  const int* d_tail = nullptr;
  const int grid_iters = select_pairs_async(adj, (int)N, a.lg, sg, nseg, W.budget, W.partner,
                                            W.temp, st_, &d_mseg, &d_tail);
  if (T) T->stop(tk);

  // the pass's counts come back with the merge's synchronisation
  long long* hb = hb_;

  // single running job with a trace buffer: provenance pairs of this pass
  int* trace = nullptr;
  int* parent = nullptr;
  if (searching == 1 && nseg == 1) {
    Job& j = jobs_[live_[0]];
    if (j.spec.d_trace) trace = j.spec.d_trace + 2 * j.traced;
    // hierarchy level of this pass: the set before its merges, and where
    // each of its splats goes
    if (j.spec.lod.pos && j.lod_levels < NANOGS_MAX_ROUNDS && j.lod_used + j.N <= j.spec.lod_cap) {
      const long long o = j.lod_used;
      nanogs_gaussians& L = j.spec.lod;
      launch_deactivate_work(a.cen + j.row0, a.lg + j.row0, a.shp + 2 * j.row0, a.org + j.row0,
                             (int)j.N, (int)j.row0, L.pos + 3 * o, L.log_scale + 3 * o,
                             L.rot + 4 * o, L.opacity + o, nullptr, st_);
      launch_copy_sh_rows(a.sh + j.row0 * NG_SH, nullptr, L.sh + o * NG_SH, a.lg + j.row0,
                          (int)j.row0, (int)j.N, st_);
      parent = j.spec.lod_parent + o - j.row0;
      j.spec.lod_offsets[j.lod_levels] = o;
      j.lod_used = o + j.N;
      j.spec.lod_offsets[j.lod_levels + 1] = j.lod_used;
      ++j.lod_levels;
    }
  }
  k_stats_select<<<blocks_for(nseg, 256), 256, 0, st_>>>(mcount, fb_count, d_tail, d_mseg, nseg,
                                                          W.stats);
  NG_LAUNCH_CHECK();
  NG_HIP(hipMemcpyAsync(hb, W.stats, (8 + (size_t)nseg) * sizeof(long long),
                        hipMemcpyDeviceToHost, st_));
  tk = T ? T->start(NANOGS_T_MERGE) : -1;
  // the local refresh of the next pass needs the new index of every splat
  int* par = parent ? parent : (refresh_local ? W.parent : nullptr);
  const long long nn = merge_compact(a.cen, a.lg, a.shp, a.sh, a.org, (int)N, W.partner, b.cen,
                                     b.lg, b.shp, b.sh, b.org, trace, W.temp, st_, nullptr, sg,
                                     b.sg, W.seg, nseg, par);
  if (refresh_local && par != W.parent)
    NG_HIP(hipMemcpyAsync(W.parent, par, N * sizeof(int), hipMemcpyDeviceToDevice, st_));
  if (refresh_local) {
    j1->prev_n = N;
    j1->prev_keff = hs[0].keff;
  }
  if (T) T->stop(tk);
  // merge_compact synchronised the stream: the counts are in hb
  const long long m = hb[0];
  if (hb[1] != 0) throw HipError{"internal: working set not in Morton order"};
  const long long knn_retries = hb[2];
  const long long knn_screens = hb[3];
  const long long requeried = incremental ? hb[4] : N;
  const long long fb = o_.precision != NANOGS_PREC_FP64 ? hb[5] : m;
  if (hb[6] < 0) throw HipError{"internal: the matching did not converge"};
  const int ld_iters = grid_iters + (int)hb[6];
  std::vector<long long> hM(nseg, 0);
  for (int i = 0; i < nseg; ++i) hM[i] = hb[8 + i];

  // per-job bookkeeping of the pass
  for (int i = 0; i < nseg; ++i) {
    Job& j = jobs_[live_[i]];
    if (j.state != JOB_RUNNING) continue;
    const int r = j.round;
    if (r < NANOGS_MAX_ROUNDS) {
      j.stats.n_per_round[r] = j.N;
      j.stats.edges_per_round[r] = searching == 1 ? m : 0;
      j.stats.pairs_per_round[r] = hM[i];
      j.stats.fallback_per_round[r] = searching == 1 ? fb : 0;
      j.stats.ld_iters_per_round[r] = ld_iters;
      j.stats.knn_retry_per_round[r] = searching == 1 ? knn_retries : 0;
      j.stats.knn_screens_per_round[r] = searching == 1 ? knn_screens : 0;
      j.stats.requery_per_round[r] = searching == 1 ? requeried : 0;
    }
  }

  cur_ ^= 1;
  Ntot_ = nn;

  // new segment rows (same order, draining segments gone) and job states
  std::vector<int> still;
  long long row = 0;
  for (int i = 0; i < nseg; ++i) {
    Job& j = jobs_[live_[i]];
    if (j.state != JOB_RUNNING) {
      if (j.state == JOB_DRAINING) j.state = JOB_DONE;
      continue;
    }
    j.N -= hM[i];
    j.row0 = row;
    row += j.N;
    if (hM[i] > 0) {
      j.stats.rounds = ++j.round;
      j.traced += hM[i];
    }
    still.push_back(j.id);
    const bool stop = j.N <= j.spec.target || hM[i] == 0 ||
                      (o_.max_rounds > 0 && j.round >= o_.max_rounds);
    if (hM[i] == 0 && j.N > j.spec.target) j.stats.early_exit = 1;
    if (stop) {
      finish_job(j, W.w[cur_]);
      ++finished;
    }
  }
  live_ = still;
  return finished;
}

bool Engine::idle() const { return queue_.empty() && live_.empty(); }

void Engine::run(StageTimer* T) {
  while (!idle()) step(T);
  NG_HIP(hipStreamSynchronize(st_));
}

}  // namespace ng
