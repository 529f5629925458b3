// Internal declarations shared by the library's translation units.
//
// Working layout (the library keeps its own copy of the splats, in an order
// chosen for locality; every result is still defined on the caller's order,
// called the logical order here):
//   cen[p]        float4 (x, y, z, logical index as int bits)
//   lg[p]         int32 logical index (same value as cen[p].w)
//   shp[2p]       float4 (s0, s1, s2, alpha)      activated scales, opacity
//   shp[2p+1]     float4 (qw, qx, qy, qz)         unit quaternion
//   sh[p*48 ..]   float[48]                        appearance feature f
//   org[p]        int32 provenance (smallest input index absorbed)
// Per pass, per splat (cost kernel input):
//   pre[2p]       float4 (L00, L10, L11, L20)     Cholesky factor of Sigma
//   pre[2p+1]     float4 (L21, L22, log det L, w~) with w~ = ((a*s0)*s1)*s2
//   after the 2n float4: n doubles, the same weight in double (the mixture
//   weight pi that picks a draw's component is taken in double)
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#define NG_DEV __device__ __forceinline__
#define NG_SH 48

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace ng {

void set_error(const std::string& msg);

struct HipError {
  std::string msg;
  hipError_t code = hipErrorUnknown;
};

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError{std::string(what) + ": " + hipGetErrorString(e), e};
}
#define NG_HIP(x) ::ng::hip_check((x), #x)
#define NG_LAUNCH_CHECK() ::ng::hip_check(hipGetLastError(), "kernel launch")

inline unsigned blocks_for(long long n, int bs) {
  long long b = (n + bs - 1) / bs;
  return (unsigned)(b < 1 ? 1 : b);
}

// ---------------------------------------------------------------------------
// workspace carving (256-byte aligned sub-buffers)
// ---------------------------------------------------------------------------
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t bytes() const { return (off + 255) & ~(size_t)255; }
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
// Order-preserving map of a float to uint32 (-0 and +0 map to one key).
NG_DEV uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  if (u == 0x80000000u) u = 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

NG_DEV int lane_id() { return (int)(threadIdx.x & 63); }

// Block index with each XCD's share of the grid contiguous.  Workgroups are
// dispatched to the 8 XCDs in turn (dispatch index b runs on XCD b % 8), and
// each XCD has its own L2; for kernels whose blocks cover consecutive rows
// of the Morton-ordered working set, giving every XCD one contiguous range
// keeps the rows a block shares with its neighbours in one L2.  A bijection
// of [0, gridDim.x): XCD x takes blocks [x*per + min(x, rem), +count_x).
constexpr unsigned kXcds = 8;
NG_DEV unsigned xcd_block() {
  const unsigned b = blockIdx.x, G = gridDim.x;
  const unsigned per = G / kXcds, rem = G % kXcds, x = b % kXcds;
  return x * per + (x < rem ? x : rem) + b / kXcds;
}

NG_DEV float ord2f(unsigned u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

NG_DEV unsigned spread10(unsigned v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// 30-bit Morton key of a point on the 1024^3 grid over the bounding cube
// whose per-axis bounds box[0..2] (min) and box[3..5] (max) are stored as
// f2ord values.  Points outside the box clamp to its faces.
// Rows only need to be ordered by their cell at the finest table level
// (at most 8): the sort key is the level-8 cell, the top 24 bits of the key.
constexpr int kSortKeyBits = 24;
constexpr int kSortKeyShift = 30 - kSortKeyBits;

NG_DEV unsigned morton_key(float x, float y, float z, const unsigned* box) {
  float lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = ord2f(box[a]);
    hi[a] = ord2f(box[3 + a]);
  }
  const float ext = fmaxf(fmaxf(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
  const float sc = ext > 0.f ? 1023.0f / ext : 0.f;
  const float v[3] = {x, y, z};
  unsigned q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float t = (v[a] - lo[a]) * sc;
    t = fminf(fmaxf(t, 0.f), 1023.f);  // NaN -> 0
    q[a] = (unsigned)t;
  }
  return (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
}

// A segment = one scene of a batch, rows [row0, row0 + nrows) of the working
// set, which is also its range of logical indices.  A single scene is one
// segment.
struct SegInfo {
  unsigned box[6];  // Morton bounds: f2ord of the min and max corner
  int row0;
  int nrows;
  int LT;      // cell table level (0: no search this pass)
  int toff;    // first entry of its cell table
  int keff;    // kNN size in use this pass
  int kclass;  // kernel class serving it (8, 16, 24, 32), 0: no search
  int crn;     // its row of the draw table
  int next;    // its position after this pass's compaction, -1: its rows are dropped
};

// Launch parameters per size bucket (see nanogs_tuning); util.hip.
struct Tuning {
  int cost_block = 256;
  int knn_block = 128;
  int knn_wave_grid = 16384;
  int knn_level_bias = 0;
  int select_check = 4;
  int knn_block_min = 32;
  int knn_lane_rows = 256;
};
constexpr int TUNE_BUCKETS = 3;
int tune_bucket(long long n);
const Tuning& tuning_for(long long n);
void set_tuning(int bucket, const Tuning& t);

// ---------------------------------------------------------------------------
// host-side launchers (each defined in the .hip file named in the comment)
// ---------------------------------------------------------------------------

// util.hip -- exclusive prefix sums, fills
size_t scan_temp_bytes(long long n);
// out[i] = sum_{j<i} in[j]; *total (device, nullable) = sum of all.
void scan_exclusive_i32(const int* in, int* out, long long n, int* total, void* temp,
                        hipStream_t st);
// Two exclusive scans of n ints each in one pair of launches (out_a of in_a,
// out_b of in_b; totals nullable); temp of scan_temp_bytes(n).
void scan_exclusive2_i32(const int* in_a, int* out_a, int* total_a, const int* in_b, int* out_b,
                         int* total_b, long long n, void* temp, hipStream_t st);
void fill_i32(int* p, int v, long long n, hipStream_t st);
// *out = min(max(*d, 0), cap) as int32 (device to device, one thread).
void count_to_i32(const long long* d, long long cap, int* out, hipStream_t st);
void fill_u64(unsigned long long* p, unsigned long long v, long long n, hipStream_t st);
void set_i64(long long* d, long long v, hipStream_t st);
// *d = *s (device int32 -> device int64, one thread).
void widen_i32(const int* s, long long* d, hipStream_t st);
// Small page-locked host buffer (64 int64 slots) for counts read back by the
// host; one per calling thread, kept for the life of the process.
long long* pinned_host();

// sort.hip -- stable LSD radix sort of (uint32 key, int32 value) pairs
size_t sort_temp_bytes(long long n);
// Sorts keys/vals in place (using temp for the second buffers and counts).
// With out_vals, an odd number of digit passes leaves the sorted pairs in
// temp instead and *out_vals points at the sorted values there (the keys are
// then not copied back either); otherwise *out_vals = vals.
void sort_pairs_u32(unsigned* keys, int* vals, long long n, int key_bits, void* temp,
                    hipStream_t st, int** out_vals = nullptr);

// activate.hip -- boundary conversions and packing
// Stored form -> working layout; row p takes input row i = perm[p] (perm
// nullable: identity), gets logical index lbase + i, provenance i and (sg
// nullable) segment sgid.  cen_t / shp_t (nullable, n and 2n rows of
// scratch): with perm, the rows are activated in input order there first,
// then gathered.
void launch_activate_stored(const float* pos, const float* log_scale, const float* rot,
                            const float* opacity, const int* perm, int n, int lbase, float4* cen,
                            int* lg, float4* shp, int* org, int* sg, int sgid, int* nonfinite,
                            hipStream_t st, float4* cen_t = nullptr, float4* shp_t = nullptr);
// Checks the SH rows for non-finite values.
void launch_check_finite(const float* x, long long count, int* nonfinite, hipStream_t st);
// Row copy of [rows][48] float arrays: dst[dst_row(r)] = src[src_row(r)],
// dst_row = dst_map ? dst_map[r] - dst_base : r, src_row = src_map ? src_map[r] : r;
// *nonfinite (nullable) is set to 1 if a copied value is not finite.
void launch_copy_sh_rows(const float* src, const int* src_map, float* dst, const int* dst_map,
                         int dst_base, int rows, hipStream_t st, int* nonfinite = nullptr);
// Working layout -> stored form at the logical positions minus lbase.
void launch_deactivate_work(const float4* cen, const int* lg, const float4* shp, const int* org,
                            int n, int lbase, float* pos, float* log_scale, float* rot,
                            float* opacity, int* origin_out, hipStream_t st);
// Activated plain arrays <-> working layout (stage entry points).
void launch_pack_splats(const float* mu, const float* scale, const float* quat, const float* alpha,
                        const int* origin, int n, float4* cen, int* lg, float4* shp, int* org,
                        hipStream_t st);
void launch_unpack_splats(const float4* cen, const float4* shp, const int* org, int n, float* mu,
                          float* scale, float* quat, float* alpha, int* origin, hipStream_t st, const int* d_n = nullptr);
void launch_activate_plain(const float* pos, const float* log_scale, const float* rot,
                           const float* opacity, int n, float* mu, float* scale, float* quat,
                           float* alpha, int* nonfinite, hipStream_t st);
void launch_deactivate_plain(const float* mu, const float* scale, const float* quat,
                             const float* alpha, int n, float* pos, float* log_scale, float* rot,
                             float* opacity, hipStream_t st);

// knn.hip -- spatial order and exact kNN
// Morton keys of the centres over their bounding cube (10 bits per axis);
// the bounds go to temp[0..5] (f2ord values).
void launch_morton_keys(const float* pos_xyz3, const float4* cen4, int n, unsigned* keys,
                        void* temp, hipStream_t st);
int table_level(long long n);
int table_level_max(long long n);
int kclass_of(int keff);
unsigned class_bit(int kclass);
long long table_entries(int LT);
// kNN scratch: concatenated per-segment cell tables, logical -> working
// inverse, sparse-query list.
struct StageTimer;
// The block gather's screen count is summed by each wave into one of
// kScreenSlots 64-bit counters, each on a 128-byte line of its own, from
// counters[kScreenBase] (kScreenStride ints apart): atomics from every wave
// of the chip to one address serialise.
constexpr int kScreenBase = 64;
constexpr int kScreenSlots = 64;
constexpr int kScreenStride = 32;
constexpr int kKnnCounters = kScreenBase + kScreenSlots * kScreenStride;
struct KnnMem {
  int* table;
  int* inv;      // logical index -> working row
  int2* retry;   // (row, 0) of the queries the wave search finishes
  int2* ginfo;   // per query: (rows buffered by the block gather or -1, level)
  int* counters;  // [1]: retry count; the screen sums from kScreenBase
  int* gbuf;     // [slot][n] rows buffered by the block gather
};
KnnMem carve_knn(void* base, long long n, long long entries, int kmax, size_t* bytes);
// Cell tables of every segment with LT > 0 (rows sorted by Morton key within
// each segment; *d_unsorted or-ed with 1 if not), and the logical -> working
// inverse (rows carry their logical index in cen[].w).
void knn_build(const float4* cen, int n, const int* sg, const SegInfo* dseg, long long entries,
               void* mem, int* d_unsorted, hipStream_t st);
// Exact kNN of every row of a segment with kclass > 0 among the rows of its
// segment: nbr[p][t], t < keff of the segment, key (d2, logical); rows of
// other segments get -1.  Entries are working rows (use_inv) or logical
// indices; rows_logical: row index = logical index.  class_mask: bits of
// the kernel classes present (class_bit).
void knn_query(const float4* cen, int n, int k_out, const int* sg, const SegInfo* dseg,
               unsigned class_mask, long long entries, void* mem, bool use_inv, int rows_logical,
               int* nbr, StageTimer* T, hipStream_t st);
// Local neighbourhood refresh (Sec. 3.4) of a one-segment working set of
// n_new rows after a pass over n_old rows: parent[o] = new logical index of
// old logical index o, nbr_log[o][t] = its old list (old logical indices,
// t < keff; keff unchanged).  A new splat formed by a merge, or whose old list
// names a splat that merged, gets its exact kNN (as knn_query; the rows go
// to dlist, their count to device *dcount); every other row's list is its
// old list carried to the new indices.  Entries are working rows.  Needs
// knn_build of the new set first.  pcount: scratch [n_new].
void knn_refresh(const float4* cen, int n_new, int n_old, int k_out, int keff, const int* sg,
                 const SegInfo* dseg, long long entries, void* mem, const int* parent,
                 int* pcount, const int* nbr_log, int* dlist, int* dcount, int* nbr, StageTimer* T,
                 hipStream_t st);
// nbr_log[lg[p]][t] = lg[nbr[p][t]] for t < keff, -1 after (lists by logical index).
void knn_save_log(const int* lg, const int* nbr, int n, int k_out, int keff, int* nbr_log,
                  hipStream_t st);
// Exact kNN of centres given in caller order (mu[n][3]); rows by caller index.
size_t knn_plain_bytes(long long n, int k);
void knn_plain(const float* mu, int n, int k, int keff, int* nbr, void* ws, hipStream_t st);

// edges.hip -- union edges and the incidence structure of the selection
struct EdgeSet {
  int* src;    // [n*k] emitting row of edge e (physical)
  int* tgt;    // [n*k] the listed neighbour (physical)
  int* eoff;   // [n+1] first edge of each row; eoff[n] = m
  int* ioff;   // [n+1] start of each splat's incoming edges (nullable: none)
  int* islot;  // [n*k] rank of e among the edges into tgt[e]
  int* aoff;   // [n+1] eoff + ioff: adjacency range of each splat
};
size_t edges_temp_bytes(long long n, int k);
// Emits the union edges of the lists in nbr (entries < 0 skipped) in
// emission order; order between the two ends by lg (nullable: identity).
// The count goes to *d_m (device int64, nullable) and to es.eoff[n].
void launch_union_edges(const int* nbr, const int* lg, int n, int k, EdgeSet es, long long* d_m,
                        void* temp, hipStream_t st);
// Stage entry point: ei < ej in the caller's numbering, emission order.
size_t edges_public_bytes(long long n, int k);
void union_edges_public(const int* nbr, int n, int k, int* ei, int* ej, long long* d_m, void* ws,
                        hipStream_t st);

// cost.hip -- per-splat precompute and the edge cost
// Shared draws of a pass (Appendix A): tab[r * NG_CRN_ROW + 4 s + c] is draw
// s (u, z0, z1, z2) of table row r; a segment reads row seg[sg[p]].crn (row
// 0 when sg is null).
#define NG_CRN_ROW 64
struct CrnTab {
  const float* tab;  // device
  int S;
  const int* sg;
  const SegInfo* seg;
  int mode = 0;  // geometric term (NANOGS_COST_*)
};
// Adjacency entries written by the cost kernels: each edge (src, tgt) puts
// key (orderable cost << 32 | logical index of the other end) and the other
// end's physical index at both ends' positions (see edges.hip).
struct AdjOut {
  const int* eoff;
  const int* ioff;
  const int* islot;
  unsigned long long* akey;
  int* au;
};
// pre holds pre_float4s(n) float4: the factors of every splat, then their
// double weights.
inline long long pre_float4s(long long n) { return 2 * n + (n + 1) / 2; }
inline double* pre_weights(float4* pre, long long n) { return (double*)(pre + 2 * n); }
void launch_precompute(const float4* shp, int n, float4* pre, hipStream_t st);
// FP32 cost of edges [0, m) (m clamped to the device count *d_mcount when
// that is given); edges needing FP64 are appended to fb_list.  Edges with an
// end outside [0, n) get a NaN cost.  orient: the end with the smaller
// logical index (cen[].w) is the mixture's first component; otherwise ea[e]
// is.  adj.akey nullable.
void launch_edge_cost(const float4* cen, const float4* pre, const float* sh, int app_dims,
                      const int* ea, const int* eb, int m, int n, bool orient, const CrnTab& crn,
                      float fb_ratio, float* cost, float* dgeo, int* fb_list, int* fb_count,
                      AdjOut adj, hipStream_t st, const int* d_mcount = nullptr);
// FP64 cost of the listed edges (list nullable: all edges [0, count_host)).
void launch_edge_cost_fp64(const float4* cen, const float4* shp, const float* sh, int app_dims,
                           const int* ea, const int* eb, int n, bool orient, const int* list,
                           const int* d_count, int count_cap, const CrnTab& crn, float* cost,
                           float* dgeo, AdjOut adj, hipStream_t st);

// select.hip -- greedy disjoint pairs by locally-dominant matching
struct Adjacency {
  int* aoff;                 // [n+1]
  unsigned long long* akey;  // [aoff[n]]
  int* au;                   // [aoff[n]]
};
size_t select_temp_bytes(long long n, long long m, int nseg);
size_t select_adj_bytes(long long n, long long m);
// Adjacency of an arbitrary edge list (cost per edge, caller numbering);
// m is clamped to the device count *d_mcount when that is given.
void build_adjacency(const int* ea, const int* eb, const float* cost, long long m, int n,
                     Adjacency* adj, void* ws, hipStream_t st, const int* d_mcount = nullptr);
struct SelectResult {
  long long pairs;
  int iters;
};
// partner[n] (physical); pair tie-break on lg (nullable: identity).  Each of
// the nseg segments (row -> segment in sg, nullable when nseg = 1) keeps at
// most hP[s] pairs (host array); hM (host, nullable) receives the pairs kept
// per segment, d_npairs (device int64, nullable) segment 0's count.
// Synchronises st, unless dP is given: then (nseg = 1) the budget is the
// device int64 *dP, hP and hM are unused, nothing is read back and the
// result's fields are -1.
SelectResult select_pairs(const Adjacency& adj, int n, const int* lg, const int* sg, int nseg,
                          const long long* hP, int* partner, void* temp, hipStream_t st,
                          long long* d_npairs, long long* hM, const long long* dP = nullptr);
// As select_pairs with nothing read back and no synchronisation: budgets
// in device memory (dP, nseg), the pairs kept per segment left in device
// memory (*d_mseg, nseg ints), the finishing workgroup's iteration count in
// *d_tail_iters (device).  Returns the grid-wide iterations launched.
int select_pairs_async(const Adjacency& adj, int n, const int* lg, const int* sg, int nseg,
                       const long long* dP, int* partner, void* temp, hipStream_t st,
                       const int** d_mseg, const int** d_tail_iters);

// merge.hip -- MPMM merge + stable compaction in working layout
size_t merge_temp_bytes(long long n);
// Returns the new count.  lg nullable (identity).  seg nullable: when given
// (segments of the rows in sg), rows of segments with next < 0 are dropped,
// sg_o receives each row's new segment position, and the output rows are
// placed by (segment, Morton key of the output centre over the segment's
// box): the physical order of the working set is free, the logical
// numbering is unaffected.  Without seg, survivors keep their relative
// order.  Writes the provenance pairs
// (min origin, max origin) of the merges to trace (nullable) in the order of
// the lower logical index.
// parent (nullable, indexed by logical index) receives the logical index of
// the output splat each input splat becomes (both ends of a pair the same).
// Synchronises st, unless host_count is false (only without seg): then
// nothing is read back, the new count is left in *d_nout_i32 (required) and
// the result is -1.
long long merge_compact(const float4* cen, const int* lg, const float4* shp, const float* sh,
                        const int* org, int n, const int* partner, float4* cen_o, int* lg_o,
                        float4* shp_o, float* sh_o, int* org_o, int* trace, void* temp,
                        hipStream_t st, int* d_nout_i32, const int* sg, int* sg_o,
                        const SegInfo* seg, int nseg, int* parent = nullptr, bool host_count = true);

// prune.hip -- opacity pre-filter (tau' = min(tau, median alpha), keep alpha >= tau')
size_t prune_temp_bytes(long long n);
// Activated plain arrays -> their survivors (origin nullable); the count goes
// to the device int64 *d_nout.  Asynchronous.
void prune_splats(const float* mu, const float* scale, const float* quat, const float* alpha,
                  const float* sh, const int* origin, int n, float tau, float* mu_o,
                  float* scale_o, float* quat_o, float* alpha_o, float* sh_o, int* origin_o,
                  long long* d_nout, void* temp, hipStream_t st);
// Stored-form arrays -> their survivors; kept[o] = input index of survivor o.
// Returns the survivors' count; *nonfinite is set when an opacity is not
// finite.  Synchronises st.
long long prune_stored(const float* pos, const float* ls, const float* rot, const float* op,
                       const float* sh, int n, float tau, float* pos_o, float* ls_o,
                       float* rot_o, float* op_o, float* sh_o, int* kept, bool* nonfinite,
                       void* temp, hipStream_t st);
// v[i] = map[v[i]] for i < count (entries < 0 kept).
void remap_indices(int* v, long long count, const int* map, hipStream_t st);

// crn.cpp
void crn_host(uint64_t seed, int round, int S, float* out);

// Stage timing with HIP events recorded on the working stream.
// Per-stage HIP event timing of one call.  The events come from a pool that
// the timer keeps (per thread, for the device it was last used on; they are
// not released before the thread ends), created without the system-scope
// fence a default event record makes: a timing event needs no cache
// writeback, and one at every stage boundary would stall the stream.
struct StageTimer {
  static constexpr int kMax = 4096;
  bool on = false;
  unsigned mask = 0;  // bit s: stage s is timed
  hipStream_t st = nullptr;
  int used = 0;
  int created = 0;  // events in the pool
  int dev = -1;     // device of the pool
  int stage[kMax / 2];
  hipEvent_t ev[kMax];
  // timing: options.timing (0 off, 1 every stage, NANOGS_TIME_SOME | bits)
  void begin_call(int timing, hipStream_t s) {
    on = timing != 0;
    mask = timing == 1 ? ~0u : (unsigned)timing & 0x3fffffffu;  // (bits below the flag)
    st = s;
    used = 0;
    if (!on) return;
    int d = 0;
    NG_HIP(hipGetDevice(&d));
    if (d != dev) {  // a pool of another device's events: start a new one
      created = 0;
      dev = d;
    }
  }
  int start(int which) {
    if (!on || !((mask >> which) & 1u) || used + 2 > kMax) return -1;
    const int i = used;
    used += 2;
    for (; created < used; ++created)
      NG_HIP(hipEventCreateWithFlags(&ev[created], hipEventDisableSystemFence));
    stage[i / 2] = which;
    NG_HIP(hipEventRecord(ev[i], st));
    return i;
  }
  void stop(int i) {
    if (i >= 0) NG_HIP(hipEventRecord(ev[i + 1], st));
  }
  // after the stream is synchronised: accumulate (the events stay pooled)
  void collect(double* ms, int* launches) {
    for (int i = 0; i < used; i += 2) {
      float t = 0.f;
      NG_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
      ms[stage[i / 2]] += t;
      launches[stage[i / 2]] += 1;
    }
    used = 0;
  }
};

}  // namespace ng
