// Exact k-nearest-neighbour graph over splat centres (Sec. 3.1).
//
// Spatial structure: the working array is kept sorted by the level-8 cell of
// the 30-bit Morton key of the centres (quantised on a 1024^3 grid over the
// bounding cube), so every octree cell of level 8 or coarser is a contiguous
// range of rows; a table of cell starts at one level gives the range of any
// cell at that level or coarser.
//
// Query, in three kernels.  The block gather (four lanes per query) screens
// the rows of the 3x3x3 block of cells around the query at a level chosen by
// the block's row count, plus the cells of the k-th ball outside the block,
// and buffers every row that may enter the list.  The exact pass gives the
// buffered rows the exact key and keeps the k best.  Queries the gather gives
// up on (heavy blocks, wide or full balls, full buffers) are finished one
// wave each.
// Candidates are screened in float against bounds widened for rounding (never
// rejecting a point the exact key would keep); survivors get the exact key
// (d2, logical index) with d2 = ((dx*dx + dy*dy) + dz*dz) in double without
// contraction.  The result is the exact kNN with ties broken by index.
#include <algorithm>
#include <cstring>
#include <climits>

#include "../../include/nanogs.h"
#include "internal.h"

namespace ng {
namespace {


// ---- Morton keys -----------------------------------------------------------
__global__ void __launch_bounds__(256)
k_bbox(const float* __restrict__ xyz3, const float4* __restrict__ cen4, int n,
       unsigned* __restrict__ box) {
  __shared__ float red[4][6];
  float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float v[3];
    if (cen4) {
      float4 c = cen4[i];
      v[0] = c.x;
      v[1] = c.y;
      v[2] = c.z;
    } else {
      v[0] = xyz3[3 * (long long)i];
      v[1] = xyz3[3 * (long long)i + 1];
      v[2] = xyz3[3 * (long long)i + 2];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      mn[a] = fminf(mn[a], v[a]);
      mx[a] = fmaxf(mx[a], v[a]);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    for (int d = 32; d > 0; d >>= 1) {
      mn[a] = fminf(mn[a], __shfl_xor(mn[a], d, 64));
      mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], d, 64));
    }
  }
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      red[w][a] = mn[a];
      red[w][3 + a] = mx[a];
    }
  }
  __syncthreads();
  // one atomic per block and bound (the per-wave values are combined first)
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    float v = red[0][a];
    for (int j = 1; j < 4; ++j) v = a < 3 ? fminf(v, red[j][a]) : fmaxf(v, red[j][a]);
    if (a < 3)
      atomicMin(&box[a], f2ord(v));
    else
      atomicMax(&box[a], f2ord(v));
  }
}

__global__ void k_morton(const float* __restrict__ xyz3, const float4* __restrict__ cen4, int n,
                         const unsigned* __restrict__ box, unsigned* __restrict__ keys) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v[3];
  if (cen4) {
    float4 c = cen4[i];
    v[0] = c.x;
    v[1] = c.y;
    v[2] = c.z;
  } else {
    v[0] = xyz3[3 * (long long)i];
    v[1] = xyz3[3 * (long long)i + 1];
    v[2] = xyz3[3 * (long long)i + 2];
  }
  keys[i] = morton_key(v[0], v[1], v[2], box) >> kSortKeyShift;
}

__global__ void k_iota(int* v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// ---- cell table ------------------------------------------------------------
// The working array is sorted by level-8 cell of the 30-bit Morton key of the
// centres, so every octree cell of level L <= 8 (a Morton prefix of 3L bits)
// is a contiguous range of rows.  A segment's table holds, for every cell c
// of level LT, the first row whose level-LT cell is >= c (cstart[8^LT] = the
// segment's end); a cell of a coarser level L is the range
// [cstart[c << 3(LT-L)], cstart[(c+1) << 3(LT-L)]).
//
// Built without a histogram: every row gets the global code toff + cell (rows
// of segments without a table take their successor's toff - 1), which does
// not decrease along the rows because the segments' tables follow their rows'
// order; then entry e of the concatenated tables is the first row whose code
// is >= e.

// code[i] as above, inv[logical] = i, and *unsorted |= 1 if a row's cell is
// smaller than its predecessor's in the same segment.
__global__ void k_cell_codes(const float4* __restrict__ cen, int n, const int* __restrict__ sg,
                             const SegInfo* __restrict__ seg, int* __restrict__ code,
                             int* __restrict__ inv, int* __restrict__ unsorted) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 c = cen[i];
  inv[__float_as_int(c.w)] = i;
  const SegInfo& S = seg[sg ? sg[i] : 0];
  if (S.LT <= 0) {
    code[i] = S.toff - 1;
    return;
  }
  const int shift = 3 * (10 - S.LT);
  const unsigned cell = morton_key(c.x, c.y, c.z, S.box) >> shift;
  code[i] = S.toff + (int)cell;
  if (i != S.row0) {
    const float4 a = cen[i - 1];
    if ((morton_key(a.x, a.y, a.z, S.box) >> shift) > cell) atomicOr(unsorted, 1);
  }
}

// First indices r0, r1 whose code is >= k0 and >= k1 (code sorted, n if
// none; a wave-uniform call).  A 64-way search: each step samples 64 evenly
// spaced positions of a range and keeps the gap where the predicate turns, so
// the range shrinks 64-fold; the two searches share the steps so that their
// loads overlap.
NG_DEV void lower_bound_wave2(const int* __restrict__ code, int n, int k0, int k1, int& r0,
                              int& r1) {
  const int lane = lane_id();
  int lo[2] = {0, 0}, hi[2] = {n, n};
  const int key[2] = {k0, k1};
  while (lo[0] < hi[0] || lo[1] < hi[1]) {
    unsigned long long below[2];
    int step[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      step[s] = (hi[s] - lo[s] + 63) >> 6;
      const long long p = lo[s] + (long long)lane * step[s];
      below[s] = __ballot(lo[s] < hi[s] && p < hi[s] && code[p] < key[s]);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (lo[s] >= hi[s]) continue;
      if (!below[s]) {
        hi[s] = lo[s];
        continue;
      }
      const int t = 63 - __clzll((long long)below[s]);  // last sample below the key
      const long long pt = lo[s] + (long long)t * step[s];
      lo[s] = (int)pt + 1;
      if (t < 63 && pt + step[s] < hi[s]) hi[s] = (int)(pt + step[s]);
    }
  }
  r0 = lo[0];
  r1 = lo[1];
}

// table[e] = first row i with code[i] >= e, for e in [0, m].  One wave per
// chunk of kFillChunk entries [E, E + kFillChunk): the rows [r0, r1) whose
// codes fall in the chunk come from one two-key search.  With at most
// kFillRows of them, each row that starts its code marks that code's slot in
// LDS with its index, and entry e is the smallest mark at or after e (r1 when
// none): a suffix minimum, 32 entries per lane and across the lanes.  Denser
// chunks search every entry among [r0, r1) (32 interleaved binary searches
// per lane).  The table goes out in coalesced 16-byte stores.
constexpr int kFillChunk = 2048;
constexpr int kFillPer = kFillChunk / 64;
constexpr int kFillRows = 1024;

__global__ void __launch_bounds__(64)
k_table_fill(const int* __restrict__ code, int n, int m, int* __restrict__ table) {
  __shared__ __align__(16) int mark[kFillChunk];
  const int lane = threadIdx.x;
  const int E = blockIdx.x * kFillChunk;  // <= m (grid)
  int r0, r1;
  lower_bound_wave2(code, n, E, E + kFillChunk, r0, r1);
  const int cnt = r1 - r0;
  if (cnt > kFillRows) {
    int b[kFillPer];
#pragma unroll
    for (int q = 0; q < kFillPer; ++q) b[q] = r0;
    for (int len = cnt; len > 1;) {
      const int half = len >> 1;
#pragma unroll
      for (int q = 0; q < kFillPer; ++q)
        if (code[b[q] + half] < E + 64 * q + lane) b[q] += half;
      len -= half;
    }
#pragma unroll
    for (int q = 0; q < kFillPer; ++q) {
      const int e = E + 64 * q + lane;
      if (e <= m) table[e] = b[q] + (code[b[q]] < e ? 1 : 0);
    }
    return;
  }
  int4* m4 = reinterpret_cast<int4*>(mark);
  const int4 none = make_int4(INT_MAX, INT_MAX, INT_MAX, INT_MAX);
#pragma unroll
  for (int k = 0; k < kFillChunk / 256; ++k) m4[k * 64 + lane] = none;
  __syncthreads();
  // four loads in flight per lane; a row's predecessor comes from the lane
  // below (lane 0: from lane 63 of the previous load, or none at r0)
  int above = INT_MIN;
  for (int base = r0; base < r1; base += 256) {
    int c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = base + 64 * k + lane;
      c[k] = j < r1 ? code[j] : INT_MAX;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = base + 64 * k + lane;
      int prev = __shfl_up(c[k], 1, 64);
      if (lane == 0) prev = above;
      above = __shfl(c[k], 63, 64);
      // (the range test only matters for unsorted rows, which the order flag reports)
      if (j < r1 && c[k] != prev && c[k] >= E && c[k] - E < kFillChunk) mark[c[k] - E] = j;
    }
  }
  __syncthreads();
  int v[kFillPer];
#pragma unroll
  for (int k = 0; k < kFillPer / 4; ++k) {
    const int4 t = m4[lane * (kFillPer / 4) + k];
    v[4 * k] = t.x;
    v[4 * k + 1] = t.y;
    v[4 * k + 2] = t.z;
    v[4 * k + 3] = t.w;
  }
  int x = v[0];
#pragma unroll
  for (int q = 1; q < kFillPer; ++q) x = min(x, v[q]);
  // suffix minimum over the lanes, then the carry from the lanes above
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_down(x, d, 64);
    if (lane + d < 64) x = min(x, y);
  }
  int carry = __shfl_down(x, 1, 64);
  carry = lane < 63 ? min(carry, r1) : r1;
#pragma unroll
  for (int q = kFillPer - 1; q >= 0; --q) {
    carry = min(carry, v[q]);
    v[q] = carry;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kFillPer / 4; ++k)
    m4[lane * (kFillPer / 4) + k] = make_int4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kFillChunk / 256; ++k) {
    const int e = E + k * 256 + 4 * lane;
    const int4 t = m4[k * 64 + lane];
    if (e + 3 <= m) {
      *reinterpret_cast<int4*>(table + e) = t;
    } else {
      if (e <= m) table[e] = t.x;
      if (e + 1 <= m) table[e + 1] = t.y;
      if (e + 2 <= m) table[e + 2] = t.z;
    }
  }
}

// Rows of segments without a search (inert): empty lists.
// Also zeroes the query counters (zero[0, nzero)).
__global__ void k_knn_prefill(int n, const int* __restrict__ sg, const SegInfo* __restrict__ seg,
                              int k_out, int* __restrict__ nbr, int* __restrict__ zero,
                              int nzero) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nzero) zero[p] = 0;
  if (p >= n) return;
  if (seg[sg ? sg[p] : 0].kclass == 0)
    for (int t = 0; t < k_out; ++t) nbr[(long long)p * k_out + t] = -1;
}

// ---- query -----------------------------------------------------------------
NG_DEV double dist2(double qx, double qy, double qz, float x, float y, float z) {
#pragma clang fp contract(off)
  double dx = qx - (double)x;
  double dy = qy - (double)y;
  double dz = qz - (double)z;
  return (dx * dx + dy * dy) + dz * dz;
}

// Float admission bound from the exact k-th key: every point whose double
// distance is <= d has a float distance <= the returned value.  The float
// evaluation rounds at most five times (relative 5 * 2^-24 on a squared
// distance), the conversion once more; 1.0000025 (about 42 * 2^-24) covers it.
NG_DEV float admit_bound(double d) {
  const float t = (float)d;
  return t * 1.0000025f;
}

template <int K>
struct Best {
  double d[K];
  int l[K];

  NG_DEV void init() {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      d[t] = INFINITY;
      l[t] = INT_MAX;
    }
  }
  NG_DEV static bool less(double da, int la, double db, int lb) {
    return da < db || (da == db && la < lb);
  }
  // sorted insertion; the caller checked that (dc, lc) beats entry K-1
  NG_DEV void insert(double dc, int lc) {
    bool lt_next = true;
#pragma unroll
    for (int t = K - 1; t > 0; --t) {
      const bool lt_prev = less(dc, lc, d[t - 1], l[t - 1]);
      // shift the previous entry down, or drop the candidate here
      const double nd = lt_prev ? d[t - 1] : (lt_next ? dc : d[t]);
      const int nl = lt_prev ? l[t - 1] : (lt_next ? lc : l[t]);
      d[t] = nd;
      l[t] = nl;
      lt_next = lt_prev;
    }
    if (lt_next) {
      d[0] = dc;
      l[0] = lc;
    }
  }
  NG_DEV void consider(double dc, int lc) {
    if (less(dc, lc, d[K - 1], l[K - 1])) insert(dc, lc);
  }
  // the kk-th smallest distance (kk <= K): the entries are sorted, so it is
  // the largest of the first kk (written as a reduction, which keeps the
  // entries in registers; an indexed read would move them to memory)
  NG_DEV double kth(int kk) const {
    double v = d[0];
#pragma unroll
    for (int q = 1; q < K; ++q) v = q < kk ? fmax(v, d[q]) : v;
    return v;
  }
};

// Geometry of the quantisation grid shared with morton_key: a point v lies in
// fine cell floor((v - lo) * sc) (clamped to [0, 1023]) per axis.
struct Grid {
  double lo[3];
  double inv_sc;  // real length of one fine cell
  double margin;  // slack for the float rounding of the quantisation
};

NG_DEV Grid grid_from_box(const unsigned* box) {
  Grid g;
  float lof[3], hif[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lof[a] = ord2f(box[a]);
    hif[a] = ord2f(box[3 + a]);
    g.lo[a] = lof[a];
  }
  const float ext = fmaxf(fmaxf(hif[0] - lof[0], hif[1] - lof[1]), hif[2] - lof[2]);
  const float sc = ext > 0.f ? 1023.0f / ext : 0.f;
  g.inv_sc = sc > 0.f ? 1.0 / (double)sc : 0.0;
  // the quantised coordinate of a point is within 3 float roundings
  // (relative) of the exact one: a few 1e-7 of a cell span; 1e-5 of the
  // extent (plus an absolute floor) covers it
  g.margin = 1e-5 * (double)ext + 1e-30;
  return g;
}

NG_DEV unsigned quant(float v, float lo, float sc) {
  float t = (v - lo) * sc;
  t = fminf(fmaxf(t, 0.f), 1023.f);
  return (unsigned)t;
}

// ---- block search, Q lanes per query -------------------------------------------
// A query takes the finest level L whose 3x3x3 block of level-L cells around
// its own cell holds at least `block_min` rows (or the segment's rows, if
// fewer), and selects its k best within that block in three passes over the
// block's rows, none of which inserts into a sorted list per candidate:
//   A. a histogram of the float squared distances, 64 bins of an eighth of
//      an octave each from (side/8)^2 to (2 side)^2 (side = cell side),
//      giving tau = the upper edge of the bin holding the keff-th distance;
//   B. the rows whose float distance is within tau (widened for rounding) go
//      to a buffer (about keff of them);
//   C. the buffered rows get the exact key (d2 in double, logical index) and
//      their rank among the buffered keys.
// Pass A scans every cell of the block; pass B skips the cells whose box is
// beyond tau (their rows fall in bins above tau, so the buffer does not
// change).
// Rows outside the block that may still enter the list lie in the cells of
// the k-th ball's range [q - r, q + r] outside the block; those are screened
// in pass B too.  A block over the scan cap, a range too wide or too full,
// or a buffer overflow sends the query to the wave search.

// the 3x3x3 block: own cell, 6 faces, 12 edges, 8 corners; the offsets are
// packed two bits per cell and axis (offset + 1), so a lane decodes cell c
// without a memory access
constexpr signed char kBlk[27][3] = {
    {0, 0, 0},    {-1, 0, 0},  {1, 0, 0},   {0, -1, 0},   {0, 1, 0},    {0, 0, -1},  {0, 0, 1},
    {-1, -1, 0},  {-1, 1, 0},  {1, -1, 0},  {1, 1, 0},    {-1, 0, -1},  {-1, 0, 1},  {1, 0, -1},
    {1, 0, 1},    {0, -1, -1}, {0, -1, 1},  {0, 1, -1},   {0, 1, 1},    {-1, -1, -1}, {-1, -1, 1},
    {-1, 1, -1},  {-1, 1, 1},  {1, -1, -1}, {1, -1, 1},   {1, 1, -1},   {1, 1, 1}};
constexpr unsigned long long pack_blk_axis(int a) {
  unsigned long long v = 0;
  for (int c = 0; c < 27; ++c) v |= (unsigned long long)(kBlk[c][a] + 1) << (2 * c);
  return v;
}
constexpr unsigned long long kBlkX = pack_blk_axis(0), kBlkY = pack_blk_axis(1),
                             kBlkZ = pack_blk_axis(2);
NG_DEV int blk(unsigned long long packed, int c) { return (int)((packed >> (2 * c)) & 3ull) - 1; }

// Dilated coordinates (spread10 form, bit i at bit 3i): the neighbours' codes
// follow from the centre's by dilated increment and decrement, without
// re-spreading every neighbour.
constexpr unsigned kDil = 0x09249249u;
struct Dil3 {
  unsigned m, c, p;  // spread10(v - 1), spread10(v), spread10(v + 1)
};
NG_DEV Dil3 dil3(unsigned v) {
  const unsigned d = spread10(v);
  return {(d - 1u) & kDil, d, ((d | ~kDil) + 1u) & kDil};
}
NG_DEV unsigned dil_pick(const Dil3& d, int off) { return off < 0 ? d.m : (off > 0 ? d.p : d.c); }

constexpr int kKnnLanes = 4;     // lanes per query of the block search
constexpr int kExactLanes = 8;   // lanes per query of the exact pass (4 and 8 measured)
constexpr int kHistWords = 32;   // its histogram: 64 eighth-octave bins, two per word
constexpr int kExtCells = 64;
constexpr int kExtRows = 128;  // rows of those cells a query scans itself   // cells of the k-th ball's range a lane may screen itself
// float screen: a point whose exact d2 is <= B has float d2 <= B * kScreen
// (the float evaluation rounds at most five times, about 3e-7 relative)
constexpr float kScreen = 1.000005f;
constexpr float kPrune = 1.00001f;  // same, for the float box distance of a cell

NG_DEV float d2_screen(float qx, float qy, float qz, float4 c) {
  const float dx = qx - c.x, dy = qy - c.y, dz = qz - c.z;
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// Query geometry shared by the block gather and the exact pass.  tq is the
// query in grid units (fine cells of the quantisation, unclamped): cell
// boxes are tested in that frame, where cell faces are exact integers and
// the rounding of a coordinate does not grow with its distance from the
// origin.
struct QueryGeo {
  float qxf, qyf, qzf;
  float lof[3];
  float ext, sc;
  float tq[3];
  unsigned qi[3];
};

// Slack of a cell face in grid units: the grid coordinate of a point is
// within about 1e-4 grid units of its exact value (one rounding of v - lo,
// whose magnitude is at most the extent, and one of the product with the
// scale), for the query and for the candidate alike.
constexpr float kGridSlack = 1.0f / 64.0f;

NG_DEV QueryGeo query_geo(const float4& cq, const SegInfo& S) {
  QueryGeo q;
  q.qxf = cq.x;
  q.qyf = cq.y;
  q.qzf = cq.z;
  float hif[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.lof[a] = ord2f(S.box[a]);
    hif[a] = ord2f(S.box[3 + a]);
  }
  q.ext = fmaxf(fmaxf(hif[0] - q.lof[0], hif[1] - q.lof[1]), hif[2] - q.lof[2]);
  q.sc = q.ext > 0.f ? 1023.0f / q.ext : 0.f;
  q.tq[0] = (q.qxf - q.lof[0]) * q.sc;
  q.tq[1] = (q.qyf - q.lof[1]) * q.sc;
  q.tq[2] = (q.qzf - q.lof[2]) * q.sc;
  q.qi[0] = quant(q.qxf, q.lof[0], q.sc);
  q.qi[1] = quant(q.qyf, q.lof[1], q.sc);
  q.qi[2] = quant(q.qzf, q.lof[2], q.sc);
  return q;
}

// Passes A and B for query p with Q lanes (Q = 2, 4 or 8, consecutive lanes
// of one wave).  The lanes split the 27 level lookups, then the cells: lane
// r scans the block's non-empty cells r, r + Q, ... (in block order) and the
// same share of the k-th ball's range, so a query's chain of dependent loads
// (a cell's range, then its rows) is about Q times shorter than with one
// lane.  The Q lanes share one histogram; a lane refreshes its pruning bound
// from it after each of its cells among the own cell and the faces (counts
// only grow, so a bound read early is still an upper bound of the k-th
// distance), and pass B starts once every lane is through pass A.  Pass B
// takes buffer slots from a counter in LDS, so the order of the buffered rows
// varies; the exact pass does not depend on it.  The query itself is not
// counted in pass A (it is buffered in pass B and skipped by the exact pass).
// Returns the number of buffered rows (written to gbuf[i * n + p]), or -1 when
// the query goes to the wave search; *level = the block's level.
template <int Q>
NG_DEV int qsum(int v) {
#pragma unroll
  for (int d = 1; d < Q; d <<= 1) v += __shfl_xor(v, d, 64);
  return v;
}
template <int Q>
NG_DEV unsigned long long qor64(unsigned long long v) {
#pragma unroll
  for (int d = 1; d < Q; d <<= 1) {
    const unsigned lo = __shfl_xor((unsigned)v, d, 64);
    const unsigned hi = __shfl_xor((unsigned)(v >> 32), d, 64);
    v |= ((unsigned long long)hi << 32) | lo;
  }
  return v;
}
// drops the lowest set bits of m, `count` of them
NG_DEV unsigned long long drop_bits(unsigned long long m, int count) {
  for (int i = 0; i < count && m; ++i) m &= m - 1ull;
  return m;
}

template <int K, int Q>
NG_DEV int block_gather_q(const float4* __restrict__ cen, int p, int n, const SegInfo& S,
                          const int* __restrict__ table, int block_min, int lane_rows,
                          unsigned* __restrict__ hist, int bs, int* __restrict__ slot,
                          int* __restrict__ gbuf, int* level, int* screens) {
  constexpr int CAP = 2 * K;
  const int r = lane_id() & (Q - 1);
  const int keff = S.keff;
  const int LT = S.LT;
  const int* cstart = table + S.toff;
  const QueryGeo q = query_geo(cen[p], S);
  const float qxf = q.qxf, qyf = q.qyf, qzf = q.qzf;

  int bmin = block_min > keff + 1 ? block_min : keff + 1;
  if (bmin > S.nrows) bmin = S.nrows;
  int L = LT;
  int rows = 0;
  unsigned mask = 0u;
  // two levels per step (L and L - 1): their table loads issue together
  auto level_counts = [&](int Lv, int& rw, unsigned& mk) {
    const int sl = 10 - Lv, G = 1 << Lv, sub = 3 * (LT - Lv);
    const int cx = (int)(q.qi[0] >> sl), cy = (int)(q.qi[1] >> sl), cz = (int)(q.qi[2] >> sl);
    const Dil3 dx = dil3((unsigned)cx), dy = dil3((unsigned)cy), dz = dil3((unsigned)cz);
    int a[(27 + Q - 1) / Q], bb[(27 + Q - 1) / Q];
#pragma unroll
    for (int i = 0; i < (27 + Q - 1) / Q; ++i) {
      a[i] = bb[i] = 0;
      const int c = i * Q + r;
      if (c >= 27) continue;
      const int ox = blk(kBlkX, c), oy = blk(kBlkY, c), oz = blk(kBlkZ, c);
      const int x = cx + ox, y = cy + oy, z = cz + oz;
      if (x < 0 || x >= G || y < 0 || y >= G || z < 0 || z >= G) continue;
      const unsigned f = ((dil_pick(dx, ox) << 2) | (dil_pick(dy, oy) << 1) | dil_pick(dz, oz))
                         << sub;
      a[i] = cstart[f];
      bb[i] = cstart[f + (1u << sub)];
    }
    rw = 0;
    mk = 0u;
#pragma unroll
    for (int i = 0; i < (27 + Q - 1) / Q; ++i) {
      const int cnt = bb[i] - a[i];
      rw += cnt;
      if (cnt > 0) mk |= 1u << (i * Q + r);
    }
  };
  for (;; L -= 2) {
    int r0, r1 = 0;
    unsigned m0, m1 = 0u;
    level_counts(L, r0, m0);
    if (L > 1) level_counts(L - 1, r1, m1);
    r0 = qsum<Q>(r0);
    m0 = (unsigned)qor64<Q>(m0);
    if (r0 >= bmin || L <= 1) {
      rows = r0;
      mask = m0;
      break;
    }
    r1 = qsum<Q>(r1);
    m1 = (unsigned)qor64<Q>(m1);
    if (r1 >= bmin || L - 1 <= 1) {
      rows = r1;
      mask = m1;
      L = L - 1;
      break;
    }
  }
  *level = L;
  *screens = 0;
  if (rows > lane_rows) return -1;
  int nscreen = 0;

  const int sl = 10 - L, sub = 3 * (LT - L);
  const int cx = (int)(q.qi[0] >> sl), cy = (int)(q.qi[1] >> sl), cz = (int)(q.qi[2] >> sl);
  const float side = q.sc > 0.f ? (float)(1 << sl) / q.sc : 0.f;
  const float side_g = (float)(1 << sl);
  const float sc2 = q.sc * q.sc;
  // eighth-octave bins: the float bits >> 20 (exponent and 3 mantissa bits)
  int base = (int)(__float_as_uint(side * side) >> 20) - 48;
  if (base < 0) base = 0;
  const Dil3 dx = dil3((unsigned)cx), dy = dil3((unsigned)cy), dz = dil3((unsigned)cz);
  auto gaps = [&](int cc, float ta, float* g2) {
#pragma unroll
    for (int o = -1; o <= 1; ++o) {
      const float lo = (float)(cc + o) * side_g - kGridSlack;
      const float hi = (float)(cc + o + 1) * side_g + kGridSlack;
      const float gg = fmaxf(fmaxf(lo - ta, ta - hi), 0.f);
      g2[o + 1] = gg * gg;
    }
  };
  float gx2[3], gy2[3], gz2[3];
  gaps(cx, q.tq[0], gx2);
  gaps(cy, q.tq[1], gy2);
  gaps(cz, q.tq[2], gz2);
  auto pick3 = [](const float* v, int off) { return off < 0 ? v[0] : (off > 0 ? v[2] : v[1]); };
  auto box_d2 = [&](int c) {
    return pick3(gx2, blk(kBlkX, c)) + pick3(gy2, blk(kBlkY, c)) + pick3(gz2, blk(kBlkZ, c));
  };
  auto range = [&](int c, int& a, int& b) {
    const unsigned f = ((dil_pick(dx, blk(kBlkX, c)) << 2) | (dil_pick(dy, blk(kBlkY, c)) << 1) |
                        dil_pick(dz, blk(kBlkZ, c))) << sub;
    a = cstart[f];
    b = cstart[f + (1u << sub)];
  };
  // (the histogram words in chunks of 8 whose loads issue together, no
  // further chunk once the bin is found)
  auto kth_edge = [&]() {
    int cum = 0, bstar = -1;
#pragma unroll
    for (int w0 = 0; w0 < kHistWords; w0 += 8) {
      unsigned v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = hist[(w0 + u) * bs];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        cum += (int)(v[u] & 0xffffu);
        if (bstar < 0 && cum >= keff) bstar = 2 * (w0 + u);
        cum += (int)(v[u] >> 16);
        if (bstar < 0 && cum >= keff) bstar = 2 * (w0 + u) + 1;
      }
      if (bstar >= 0) break;
    }
    if (bstar < 0 || bstar == 2 * kHistWords - 1 || base + bstar + 1 >= 2040) return INFINITY;
    return __uint_as_float((unsigned)(base + bstar + 1) << 20);
  };
  // this lane's cells of a mask (every Q-th set bit from its r-th), the
  // range of the next one loaded before the current one is scanned
  auto for_my_cells = [&](unsigned long long msk, auto&& rng, auto&& f) {
    unsigned long long rem = drop_bits(msk, r);
    int c = rem ? __ffsll((long long)rem) - 1 : -1;
    int a = 0, b = 0;
    if (c >= 0) rng(c, a, b);
    while (c >= 0) {
      rem = drop_bits(rem, Q);
      const int cn = rem ? __ffsll((long long)rem) - 1 : -1;
      int an = 0, bn = 0;
      if (cn >= 0) rng(cn, an, bn);
      f(c, a, b);
      c = cn;
      a = an;
      b = bn;
    }
  };

  // pass A
  for (int w = r; w < kHistWords; w += Q) hist[w * bs] = 0u;
  if (r == 0) *slot = 0;
  auto count = [&](const float4& cj, int j) {
    const float d2 = d2_screen(qxf, qyf, qzf, cj);
    int bin = (int)(__float_as_uint(d2) >> 20) - base;
    bin = bin < 0 ? 0 : (bin > 2 * kHistWords - 1 ? 2 * kHistWords - 1 : bin);
    // (the query itself adds nothing; a select, not a branch, so that the
    // row loads of a batch issue together)
    atomicAdd(&hist[(bin >> 1) * bs], j == p ? 0u : 1u << ((bin & 1) << 4));
  };
  // this lane's cells of the block (every Q-th set bit from its r-th, at
  // most kMyCells) and their ranges, loaded together and kept for pass B
  constexpr int kMyCells = (27 + Q - 1) / Q;
  int my_c[kMyCells], my_a[kMyCells], my_b[kMyCells];
  {
    unsigned long long rem = drop_bits(mask, r);
#pragma unroll
    for (int i = 0; i < kMyCells; ++i) {
      my_c[i] = rem ? __ffsll((long long)rem) - 1 : -1;
      my_a[i] = my_b[i] = 0;
      if (my_c[i] >= 0) range(my_c[i], my_a[i], my_b[i]);
      rem = drop_bits(rem, Q);
    }
  }
  auto for_block_cells = [&](auto&& f) {
#pragma unroll
    for (int i = 0; i < kMyCells; ++i)
      if (my_c[i] >= 0) f(my_c[i], my_a[i], my_b[i]);
  };
  // (every cell of the block: a bound read from the histogram after the own
  // and face cells, to skip the cells beyond it, costs more than it saves)
  for_block_cells([&](int, int a, int b) {
    nscreen += b - a;
    int j = a;
    for (; j + 4 <= b; j += 4) {
      const float4 c0 = cen[j], c1 = cen[j + 1], c2 = cen[j + 2], c3 = cen[j + 3];
      count(c0, j);
      count(c1, j + 1);
      count(c2, j + 2);
      count(c3, j + 3);
    }
    for (; j < b; ++j) count(cen[j], j);
  });
  const float tau = kth_edge();  // (every lane of the query is through pass A here)

  // pass B: rows within tau into the buffer, slots from the counter
  const float adm = tau * kScreen;
  auto keep = [&](const float4& cj, int j) {
    if (d2_screen(qxf, qyf, qzf, cj) <= adm) {
      const int pos = atomicAdd(slot, 1);
      if (pos < CAP) gbuf[(long long)pos * n + p] = j;
    }
  };
  auto scan_rows = [&](int a, int b) {
    nscreen += b - a;
    int j = a;
    for (; j + 4 <= b; j += 4) {
      const float4 c0 = cen[j], c1 = cen[j + 1], c2 = cen[j + 2], c3 = cen[j + 3];
      keep(c0, j);
      keep(c1, j + 1);
      keep(c2, j + 2);
      keep(c3, j + 3);
    }
    for (; j < b; ++j) keep(cen[j], j);
  };
  for_block_cells([&](int c, int a, int b) {
    if (c > 0 && box_d2(c) > tau * sc2 * kPrune) return;
    scan_rows(a, b);
  });

  // Rows outside the block: the block's keff-th float distance bounds the
  // true k-th one (times the rounding factor), so every row that may enter
  // the list lies within r of the query, in a level-L cell whose box (widened
  // by the margin) meets that ball.  The cells of that range outside the
  // block are screened here too, unless the range spans more than kExtCells
  // cells or holds more than kExtRows rows (then the wave search takes the
  // query).
  bool gave_up = false;
  if (q.sc > 0.f) {
    const int G = 1 << L;
    const float rg = sqrtf(adm) * q.sc * 1.000002f + 2.f * kGridSlack;
    const int c3[3] = {cx, cy, cz};
    int lo3[3], hi3[3];
    bool inside = true;
    int vol = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float f0 = floorf((q.tq[a] - rg) / side_g);
      const float f1 = floorf((q.tq[a] + rg) / side_g);
      lo3[a] = f0 < 0.f ? 0 : (f0 > (float)(G - 1) ? G - 1 : (int)f0);
      hi3[a] = f1 < 0.f ? 0 : (f1 > (float)(G - 1) ? G - 1 : (int)f1);
      inside = inside && lo3[a] >= c3[a] - 1 && hi3[a] <= c3[a] + 1;
      vol *= hi3[a] - lo3[a] + 1;
    }
    if (!inside) {
      if (!(tau < INFINITY) || vol > kExtCells) {
        gave_up = true;
      } else {
        const int nx = hi3[0] - lo3[0] + 1, ny = hi3[1] - lo3[1] + 1;
        unsigned long long emask = 0ull;
        for (int i = r; i < vol; i += Q) {
          const int x = lo3[0] + i % nx, y = lo3[1] + (i / nx) % ny, z = lo3[2] + i / (nx * ny);
          if (abs(x - cx) <= 1 && abs(y - cy) <= 1 && abs(z - cz) <= 1) continue;
          auto gap = [&](int c, float ta) {
            return fmaxf(fmaxf((float)c * side_g - kGridSlack - ta,
                               ta - ((float)(c + 1) * side_g + kGridSlack)), 0.f);
          };
          const float gx = gap(x, q.tq[0]), gy = gap(y, q.tq[1]), gz = gap(z, q.tq[2]);
          if (!(fmaf(gz, gz, fmaf(gy, gy, gx * gx)) > tau * sc2 * kPrune)) emask |= 1ull << i;
        }
        emask = qor64<Q>(emask);
        auto erange = [&](int i, int& a, int& b) {
          const int x = lo3[0] + i % nx, y = lo3[1] + (i / nx) % ny, z = lo3[2] + i / (nx * ny);
          const unsigned f = ((spread10((unsigned)x) << 2) | (spread10((unsigned)y) << 1) |
                              spread10((unsigned)z)) << sub;
          a = cstart[f];
          b = cstart[f + (1u << sub)];
        };
        int erows = 0;
        for_my_cells(emask, erange, [&](int, int a, int b) { erows += b - a; });
        erows = qsum<Q>(erows);
        if (erows > kExtRows)
          gave_up = true;
        else
          for_my_cells(emask, erange, [&](int, int a, int b) { scan_rows(a, b); });
      }
    }
  }
  *screens = nscreen;
  if (gave_up) return -1;
  const int nb = *slot;  // (every lane of the query is through pass B here)
  if (nb > CAP || nb < keff + 1) return -1;
  return nb;
}

// list (nullable): query only the rows list[0, *d_count)
// (Q lanes per query: the queries of a block are its threads / Q)
template <int K, int Q>
__global__ void __launch_bounds__(256)
k_knn_block(const float4* __restrict__ cen, int n, const int* __restrict__ sg,
            const SegInfo* __restrict__ seg, const int* __restrict__ table, int block_min,
            int lane_rows, int* __restrict__ gbuf, int2* __restrict__ ginfo,
            unsigned long long* __restrict__ screens, const int* __restrict__ list,
            const int* __restrict__ d_count) {
  // [kHistWords][bs / Q]: two 16-bit bin counts per word, then [bs / Q] slot
  // counters
  extern __shared__ unsigned s_hist[];
  const int idx = (xcd_block() * blockDim.x + threadIdx.x) / Q;
  const int cnt = list ? *d_count : n;
  const int p = idx < cnt ? (list ? list[idx] : idx) : n;
  int ns = 0;
  if (p < n) {
    const SegInfo& S = seg[sg ? sg[p] : 0];
    if (S.kclass == K) {
      int L = 0;
      const int nb = block_gather_q<K, Q>(cen, p, n, S, table, block_min, lane_rows,
                                          s_hist + threadIdx.x / Q, blockDim.x / Q,
                                          (int*)s_hist + kHistWords * (blockDim.x / Q) + threadIdx.x / Q,
                                          gbuf, &L, &ns);
      if ((threadIdx.x & (Q - 1)) == 0) ginfo[p] = make_int2(nb, L);
    }
  }
  // the screens of the wave, one atomic on the block's slot
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) ns += __shfl_xor(ns, d, 64);
  if (lane_id() == 0 && ns)
    atomicAdd(screens + (blockIdx.x % kScreenSlots) * (kScreenStride / 2),
              (unsigned long long)ns);
}

// Pass C with Q lanes per query (consecutive lanes): lane r takes the
// buffered rows r, r + Q, ... (their loads issue together), gives them the
// exact key, and ranks each against all buffered rows (keys broadcast from
// the other lanes); a row of rank t < keff is entry t of the list (as its
// working row when inv is given: the buffer holds working rows).  The keys
// are distinct (logical indices are), so the ranks are the sorted order.
constexpr int kExactWaves = 4;  // waves per workgroup of the exact pass
template <int K, int Q>
__global__ void __launch_bounds__(64 * kExactWaves)
k_knn_exact(const float4* __restrict__ cen, int n, int k_out, const int* __restrict__ sg,
            const SegInfo* __restrict__ seg, const int* __restrict__ table,
            const int* __restrict__ inv, int rows_logical, int* __restrict__ nbr,
            const int* __restrict__ gbuf, const int2* __restrict__ ginfo,
            int2* __restrict__ retry, int* __restrict__ n_retry, const int* __restrict__ list,
            const int* __restrict__ d_count) {
  constexpr int CAP = 2 * K;
  constexpr int PER = CAP / Q;  // buffer slots per lane
  const int lane = lane_id();
  const int r = lane & (Q - 1), qb = lane & ~(Q - 1);
  const int idx = (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) / Q);
  const int cnt = list ? *d_count : n;
  const int p = idx < cnt ? (list ? list[idx] : idx) : n;
  bool need = false;
  if (p < n) {
    const SegInfo& S = seg[sg ? sg[p] : 0];
    const int nb = S.kclass == K ? ginfo[p].x : -2;
    if (nb == -1 || (nb >= 0 && nb > CAP)) {
      need = r == 0;  // the gather gave up: retry from scratch
    } else if (nb >= 0) {
      const int keff = S.keff;
      const float4 cq = cen[p];
      const double qx = cq.x, qy = cq.y, qz = cq.z;
      int jj[PER];
#pragma unroll
      for (int t = 0; t < PER; ++t) {
        const int i = t * Q + r;
        jj[t] = i < nb ? gbuf[(long long)i * n + p] : -1;
      }
      double d[PER];
      int l[PER];
#pragma unroll
      for (int t = 0; t < PER; ++t) {
        d[t] = INFINITY;
        l[t] = INT_MAX;
        if (jj[t] >= 0 && jj[t] != p) {
          const float4 c = cen[jj[t]];
          d[t] = dist2(qx, qy, qz, c.x, c.y, c.z);
          l[t] = __float_as_int(c.w);
        }
      }
      int rank[PER];
#pragma unroll
      for (int t = 0; t < PER; ++t) rank[t] = 0;
      // every buffered key against this lane's keys
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        if (u * Q >= nb) break;  // (the same for the Q lanes)
#pragma unroll
        for (int s = 0; s < Q; ++s) {
          const double dy = __shfl(d[u], qb + s, 64);
          const int ly = __shfl(l[u], qb + s, 64);
#pragma unroll
          for (int t = 0; t < PER; ++t)
            rank[t] += (dy < d[t] || (dy == d[t] && ly < l[t])) ? 1 : 0;
        }
      }
      const long long row = rows_logical ? (long long)__float_as_int(cq.w) : (long long)p;
      int* out = nbr + row * k_out;
#pragma unroll
      for (int t = 0; t < PER; ++t)
        if (l[t] != INT_MAX && rank[t] < keff) out[rank[t]] = inv ? jj[t] : l[t];
      for (int t = keff + r; t < k_out; t += Q) out[t] = -1;
    }
  }
  // retries, appended with one atomic per workgroup (atomics of every wave
  // on one address serialise)
  __shared__ int s_cnt[kExactWaves + 1];
  const int w = (int)threadIdx.x >> 6;
  const unsigned long long m = __ballot(need);
  if (lane == 0) s_cnt[w] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int q = 0; q < kExactWaves; ++q) {
      const int c = s_cnt[q];
      s_cnt[q] = tot;
      tot += c;
    }
    s_cnt[kExactWaves] = tot ? atomicAdd(n_retry, tot) : 0;
  }
  __syncthreads();
  if (need) {
    const unsigned long long below = lane == 0 ? 0ull : (m & (~0ull >> (64 - lane)));
    retry[s_cnt[kExactWaves] + s_cnt[w] + __popcll(below)] = make_int2(p, 0);
  }
}

// ---- retries: one wave per query ---------------------------------------------
// Queries the block gather gave up on (a block over knn_lane_rows rows, a
// buffer overflow, or a k-th ball spanning too many cells), one wave each.
// The lanes share the work: cells are looked up one per lane, their rows are
// dealt out 64 at a time, and the k best live one entry per lane (lanes
// 0..K-1, sorted).  First the block
// search at the finest level whose 3x3x3 block holds bmin rows; if its k-th
// key reaches beyond the block, a ball search over the cells of the range
// [q - r, q + r] (r: that k-th distance) at the finest level where it spans at
// most 8 cells per axis.
template <int K>
struct WaveBest {
  double d;  // entry of this lane (lanes >= K hold +inf)
  int l;

  NG_DEV void init() {
    d = INFINITY;
    l = INT_MAX;
  }
  // entry kk - 1 (kk = the segment's k_eff, wave-uniform)
  NG_DEV double kth(int kk) const {
    const int lo = __shfl(__double2loint(d), kk - 1, 64);
    const int hi = __shfl(__double2hiint(d), kk - 1, 64);
    return __hiloint2double(hi, lo);
  }
  // insert (dc, lc) (wave-uniform); no-op if it does not beat entry K-1
  NG_DEV void insert(double dc, int lc) {
    const int lane = lane_id();
    const bool lt = dc < d || (dc == d && lc < l);
    // position = number of entries smaller than the candidate
    const unsigned long long ge = __ballot(lt) & ((1ull << K) - 1ull);
    if (ge == 0ull) return;
    const int pos = __ffsll((long long)ge) - 1;
    const int plo = __shfl_up(__double2loint(d), 1, 64);
    const int phi = __shfl_up(__double2hiint(d), 1, 64);
    const int pl = __shfl_up(l, 1, 64);
    if (lane < K) {
      if (lane == pos) {
        d = dc;
        l = lc;
      } else if (lane > pos) {
        d = __hiloint2double(phi, plo);
        l = pl;
      }
    }
  }
};

template <int K>
__global__ void __launch_bounds__(64)
k_knn_wave(const float4* __restrict__ cen, int n, int k_out, const int* __restrict__ sg,
           const SegInfo* __restrict__ seg, const int* __restrict__ table,
           const int* __restrict__ inv, int rows_logical, int block_min,
           int* __restrict__ nbr, const int2* __restrict__ list,
           const int* __restrict__ d_count) {
  constexpr int MAXC = 1024;  // cells one search may list
  constexpr int kRefine = 64;  // rows above which a listed cell is split
  __shared__ int s_start[MAXC];
  __shared__ int s_pref[MAXC + 1];
  __shared__ int s_hist[32];
  __shared__ int s_cand[64];
  const int lane = threadIdx.x;
  const int count = *d_count;
  for (int qidx = blockIdx.x; qidx < count; qidx += gridDim.x) {
    const int p = list[qidx].x;
    const SegInfo& S = seg[sg ? sg[p] : 0];
    if (S.kclass != K) continue;  // wave-uniform: one query per wave
    const int keff = S.keff;
    const int LT = S.LT;
    const int* cstart = table + S.toff;
    const Grid g = grid_from_box(S.box);
    float lof[3], hif[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lof[a] = ord2f(S.box[a]);
      hif[a] = ord2f(S.box[3 + a]);
    }
    const float ext = fmaxf(fmaxf(hif[0] - lof[0], hif[1] - lof[1]), hif[2] - lof[2]);
    const float sc = ext > 0.f ? 1023.0f / ext : 0.f;
    const float4 cq = cen[p];
    const double qx = cq.x, qy = cq.y, qz = cq.z;
    const float qxf = cq.x, qyf = cq.y, qzf = cq.z;
    const unsigned qi[3] = {quant(qxf, lof[0], sc), quant(qyf, lof[1], sc),
                            quant(qzf, lof[2], sc)};
    const long long row = rows_logical ? (long long)__float_as_int(cq.w) : (long long)p;
    int* out = nbr + row * k_out;
    WaveBest<K> best;

    // appends the lanes' non-empty ranges [a, b) to the cell list (ncell
    // cells so far, prefix sums of their rows in s_pref)
    int ncell = 0;
    auto add_cells = [&](int a, int b) {
      const bool has = b > a;
      const unsigned long long hm = __ballot(has);
      const int rank = __popcll(hm & (lane == 0 ? 0ull : (~0ull >> (64 - lane))));
      const int cnt = has ? b - a : 0;
      int incl = cnt;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
      }
      const int base = s_pref[ncell];
      if (has) {
        s_start[ncell + rank] = a;
        s_pref[ncell + rank] = base + incl - cnt;
      }
      const int added = __popcll(hm);
      __syncthreads();
      if (lane == 63) s_pref[ncell + added] = base + incl;
      ncell += added;
      __syncthreads();
    };
    // f(j, c) for the lanes' rows j (centre c) of the listed cells, 256 per
    // step, four per lane with their loads issued together (j = -1: no row).
    // A lane's rows advance 64 at a time, so its cell (the last one with
    // s_pref <= t) is usually the one it had or the next; a binary search
    // over the rest of the list covers longer jumps.
    auto for_rows = [&](auto&& f) {
      const int total = s_pref[ncell];
      int cur = 0;
      for (int t0 = 0; t0 < total; t0 += 256) {
        int jj[4];
        float4 cc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = t0 + 64 * u + lane;
          jj[u] = -1;
          if (t < total) {
            if (s_pref[cur + 1] <= t) {  // then cur + 1 < ncell (s_pref[ncell] = total)
              int lo = cur + 1, hi = ncell - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pref[mid] <= t) lo = mid; else hi = mid - 1;
              }
              cur = lo;
            }
            jj[u] = s_start[cur] + (t - s_pref[cur]);
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) cc[u] = jj[u] >= 0 ? cen[jj[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < 4; ++u) f(jj[u], cc[u]);
      }
    };
    // exact k best among the listed cells' rows.  A histogram of the float
    // distances (32 quarter-octave bins from 2^base) gives a bound tau (the
    // upper edge of the bin holding the keff-th distance); while the rows up
    // to that bin outnumber the lanes, the bin is split 32 ways by the next 5
    // bits of the float distance (another pass) and the bound moves to the
    // upper edge of the sub-bin holding the keff-th.  Every row that can be
    // among the k best has a float distance within the bound (widened for
    // rounding).  Up to 64 such rows get one lane each, the exact key, and
    // their rank by counting; more are inserted one after another.
    auto search = [&](int base) {
      best.init();
      if (lane < 32) s_hist[lane] = 0;
      __syncthreads();
      for_rows([&](int j, const float4& cj) {
        if (j >= 0 && j != p) {
          const float d2 = d2_screen(qxf, qyf, qzf, cj);
          int bin = (int)(__float_as_uint(d2) >> 21) - base;
          bin = bin < 0 ? 0 : (bin > 31 ? 31 : bin);
          atomicAdd(&s_hist[bin], 1);
        }
      });
      __syncthreads();
      int h = 0, cum = 0, bstar = -1;
      auto scan_hist = [&]() {
        h = lane < 32 ? s_hist[lane] : 0;
        cum = h;
#pragma unroll
        for (int d = 1; d < 32; d <<= 1) {
          const int y = __shfl_up(cum, d, 64);
          if (lane >= d) cum += y;
        }
        const unsigned long long reach = __ballot(lane < 32 && cum >= keff);
        bstar = reach ? __ffsll((long long)reach) - 1 : -1;
      };
      scan_hist();
      // the keff-th in a crowded bin 0 (rows closer than the window's floor):
      // the window moves down over those rows, 31 quarter octaves at a time;
      // its top bin then ends where bin 0 did
      bool closed = false;  // the top bin has an upper edge
      while (bstar == 0 && __shfl(h, 0, 64) > 64 && base > 0) {
        const int top = base, nbase = base > 31 ? base - 31 : 0;
        __syncthreads();
        if (lane < 32) s_hist[lane] = 0;
        __syncthreads();
        for_rows([&](int j, const float4& cj) {
          if (j >= 0 && j != p) {
            const int b21 = (int)(__float_as_uint(d2_screen(qxf, qyf, qzf, cj)) >> 21);
            if (b21 <= top) {
              const int bin = b21 - nbase;
              atomicAdd(&s_hist[bin < 0 ? 0 : bin], 1);
            }
          }
        });
        __syncthreads();
        base = nbase;
        closed = true;
        scan_hist();
      }
      float tau = INFINITY;
      if (bstar >= 0 && (bstar < 31 || closed) && base + bstar + 1 < 1020)
        tau = __uint_as_float((unsigned)(base + bstar + 1) << 21);
      // (bin 0 also holds every row below 2^base, so it is not split)
      if (bstar > 0 && tau < INFINITY) {
        int below = __shfl(cum - h, bstar, 64);  // rows in the bins before
        int inbin = __shfl(h, bstar, 64);
        unsigned key = (unsigned)(base + bstar);  // float bits >> sh of the bin
        int sh = 21;
        while (below + inbin > 64 && sh > 11) {
          const int sh2 = sh - 5;
          __syncthreads();
          if (lane < 32) s_hist[lane] = 0;
          __syncthreads();
          for_rows([&](int j, const float4& cj) {
            if (j >= 0 && j != p) {
              const unsigned bits = __float_as_uint(d2_screen(qxf, qyf, qzf, cj));
              if ((bits >> sh) == key) atomicAdd(&s_hist[(bits >> sh2) & 31], 1);
            }
          });
          __syncthreads();
          h = lane < 32 ? s_hist[lane] : 0;
          cum = h;
#pragma unroll
          for (int d = 1; d < 32; d <<= 1) {
            const int y = __shfl_up(cum, d, 64);
            if (lane >= d) cum += y;
          }
          // the sub-bins hold the bin's rows, so the keff-th is among them
          const unsigned long long r2 = __ballot(lane < 32 && below + cum >= keff);
          if (!r2) break;  // (not reached: keep the bound found so far)
          const int sb = __ffsll((long long)r2) - 1;
          below += __shfl(cum - h, sb, 64);
          inbin = __shfl(h, sb, 64);
          key = (key << 5) | (unsigned)sb;
          sh = sh2;
          tau = __uint_as_float((key + 1u) << sh);
        }
      }
      const float adm = tau * kScreen;
      int nc = 0;
      for_rows([&](int j, const float4& c) {
        const bool pass = j >= 0 && j != p && d2_screen(qxf, qyf, qzf, c) <= adm;
        const unsigned long long m = __ballot(pass);
        const int pos = nc + __popcll(m & (lane == 0 ? 0ull : (~0ull >> (64 - lane))));
        if (pass && pos < 64) s_cand[pos] = j;
        nc += __popcll(m);
      });
      __syncthreads();
      if (nc <= 64) {
        const int jme = lane < nc ? s_cand[lane] : -1;
        double dme = INFINITY;
        int lme = INT_MAX;
        if (jme >= 0) {
          const float4 c = cen[jme];
          dme = dist2(qx, qy, qz, c.x, c.y, c.z);
          lme = __float_as_int(c.w);
        }
        int rank = 0;
        for (int t = 0; t < nc; ++t) {
          const double dt = __shfl(dme, t, 64);
          const int lt = __shfl(lme, t, 64);
          rank += (dt < dme || (dt == dme && lt < lme)) ? 1 : 0;
        }
        if (lane >= nc) rank = lane;  // the ranks are then a permutation
        const int dlo = __builtin_amdgcn_ds_permute(rank << 2, __double2loint(dme));
        const int dhi = __builtin_amdgcn_ds_permute(rank << 2, __double2hiint(dme));
        const int lr = __builtin_amdgcn_ds_permute(rank << 2, lme);
        if (lane < K) {
          best.d = __hiloint2double(dhi, dlo);
          best.l = lr;
        }
      } else {
        for_rows([&](int j, const float4& c) {
          bool pass = false;
          double dme = 0.0;
          int lme = 0;
          if (j >= 0 && j != p) {
            if (d2_screen(qxf, qyf, qzf, c) <= adm) {
              pass = true;
              dme = dist2(qx, qy, qz, c.x, c.y, c.z);
              lme = __float_as_int(c.w);
            }
          }
          unsigned long long m = __ballot(pass);
          while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int dlo = __shfl(__double2loint(dme), src, 64);
            const int dhi = __shfl(__double2hiint(dme), src, 64);
            const int ls = __shfl(lme, src, 64);
            best.insert(__hiloint2double(dhi, dlo), ls);
          }
        });
      }
      __syncthreads();
    };
    auto bin_base = [](double len2) {
      const int b = (int)(__float_as_uint((float)len2) >> 21);
      return b > 0 ? b : 0;
    };

    double kd = INFINITY;  // an upper bound of the k-th key once known
    bool done = false;
    {
      // block search: the finest level whose 3x3x3 block holds bmin rows
      int bmin = block_min > keff + 1 ? block_min : keff + 1;
      if (bmin > S.nrows) bmin = S.nrows;
      // two levels per step: lanes 0..26 look up level L, lanes 32..58
      // level L - 1 (their loads issue together)
      int L, a = 0, b = 0;
      const int half = lane >> 5, li = lane & 31;
      for (L = LT;; L -= 2) {
        const int Lh = L - half;
        a = b = 0;
        if (li < 27 && Lh >= 1) {
          const int sl = 10 - Lh, G = 1 << Lh, sub = 3 * (LT - Lh);
          const int cx = (int)(qi[0] >> sl), cy = (int)(qi[1] >> sl), cz = (int)(qi[2] >> sl);
          const int x = cx + blk(kBlkX, li), y = cy + blk(kBlkY, li), z = cz + blk(kBlkZ, li);
          if (x >= 0 && x < G && y >= 0 && y < G && z >= 0 && z < G) {
            const unsigned f = ((spread10((unsigned)x) << 2) | (spread10((unsigned)y) << 1) |
                                spread10((unsigned)z)) << sub;
            a = cstart[f];
            b = cstart[f + (1u << sub)];
          }
        }
        int rows = b - a;
#pragma unroll
        for (int d = 16; d > 0; d >>= 1) rows += __shfl_xor(rows, d, 64);
        const int rows0 = __shfl(rows, 0, 64), rows1 = __shfl(rows, 32, 64);
        if (rows0 >= bmin || L <= 1) {
          if (half) a = b = 0;  // (the ranges of level L)
          break;
        }
        if (rows1 >= bmin || L - 1 <= 1) {
          if (!half) a = b = 0;
          L = L - 1;
          break;
        }
      }
      if (lane == 0) s_pref[0] = 0;
      __syncthreads();
      ncell = 0;
      add_cells(a, b);
      const int sl = 10 - L, G = 1 << L;
      const double sd = (double)(1 << sl) * g.inv_sc;
      // (bins from (side/5.7)^2 up to 8 side^2, past the block's farthest row)
      search(bin_base(sd * sd) - 20);
      kd = best.kth(keff);
      // exact if the k-th key is closer than the block's faces
      const int cx = (int)(qi[0] >> sl), cy = (int)(qi[1] >> sl), cz = (int)(qi[2] >> sl);
      double rho = INFINITY;
      if (cx - 1 > 0) rho = fmin(rho, qx - (g.lo[0] + (cx - 1) * sd + g.margin));
      if (cx + 2 < G) rho = fmin(rho, (g.lo[0] + (cx + 2) * sd - g.margin) - qx);
      if (cy - 1 > 0) rho = fmin(rho, qy - (g.lo[1] + (cy - 1) * sd + g.margin));
      if (cy + 2 < G) rho = fmin(rho, (g.lo[1] + (cy + 2) * sd - g.margin) - qy);
      if (cz - 1 > 0) rho = fmin(rho, qz - (g.lo[2] + (cz - 1) * sd + g.margin));
      if (cz + 2 < G) rho = fmin(rho, (g.lo[2] + (cz + 2) * sd - g.margin) - qz);
      done = !(sc > 0.f) || !(rho < INFINITY) || (rho > 0.0 && rho * rho * (1.0 - 1e-9) > kd);
    }
    if (!done) {
      // ball search: every row within the bound lies in a cell of the
      // range [q - r, q + r] (boxes widened by the margin); the range is
      // taken at the finest level where it spans at most 8 cells per axis,
      // and its cells whose box is beyond the bound are skipped
      const double r = sqrt(kd) + 2.0 * g.margin;
      const double q3[3] = {qx, qy, qz};
      int L = LT, lo3[3], hi3[3];
      for (;; --L) {
        const double sd = (double)(1 << (10 - L)) * g.inv_sc;
        const int G = 1 << L;
        bool fits = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double f0 = floor((q3[a] - r - g.lo[a]) / sd);
          const double f1 = floor((q3[a] + r - g.lo[a]) / sd);
          lo3[a] = f0 < 0.0 ? 0 : (f0 > G - 1 ? G - 1 : (int)f0);
          hi3[a] = f1 < 0.0 ? 0 : (f1 > G - 1 ? G - 1 : (int)f1);
          fits = fits && hi3[a] - lo3[a] < 8;
        }
        if (fits || L <= 1) break;
      }
      const int sub = 3 * (LT - L);
      const double sd = (double)(1 << (10 - L)) * g.inv_sc;
      const int nx = hi3[0] - lo3[0] + 1, ny = hi3[1] - lo3[1] + 1;
      const int ncube = nx * ny * (hi3[2] - lo3[2] + 1);
      if (lane == 0) s_pref[0] = 0;
      __syncthreads();
      ncell = 0;
      // a cell of more than kRefine rows (and above LT) is replaced by its
      // eight children whose boxes meet the ball, while the list has room
      const double sdc = sd * 0.5;
      for (int c0 = 0; c0 < ncube; c0 += 64) {
        const int ci = c0 + lane;
        int a = 0, b = 0, x = 0, y = 0, z = 0;
        if (ci < ncube) {
          x = lo3[0] + ci % nx;
          y = lo3[1] + (ci / nx) % ny;
          z = lo3[2] + ci / (nx * ny);
          const double gx = fmax(fmax(g.lo[0] + x * sd - g.margin - qx, qx - (g.lo[0] + (x + 1) * sd + g.margin)), 0.0);
          const double gy = fmax(fmax(g.lo[1] + y * sd - g.margin - qy, qy - (g.lo[1] + (y + 1) * sd + g.margin)), 0.0);
          const double gz = fmax(fmax(g.lo[2] + z * sd - g.margin - qz, qz - (g.lo[2] + (z + 1) * sd + g.margin)), 0.0);
          if (!((gx * gx + gy * gy) + gz * gz > kd * (1.0 + 1e-12))) {
            const unsigned f = ((spread10((unsigned)x) << 2) | (spread10((unsigned)y) << 1) |
                                spread10((unsigned)z)) << sub;
            a = cstart[f];
            b = cstart[f + (1u << sub)];
          }
        }
        const bool heavy = L < LT && b - a > kRefine;
        const unsigned long long hm = __ballot(heavy);
        // room: this step's cells and children plus every cell still to come
        const int later = ncube - c0 - 64 > 0 ? ncube - c0 - 64 : 0;
        const bool refine = hm && ncell + 64 + 7 * __popcll(hm) + later <= MAXC;
        add_cells(refine && heavy ? 0 : a, refine && heavy ? 0 : b);
        if (refine) {
          const int subc = sub - 3;
#pragma unroll 1
          for (int ch = 0; ch < 8; ++ch) {
            int ca = 0, cb = 0;
            if (heavy) {
              const int xc = 2 * x + (ch >> 2 & 1), yc = 2 * y + (ch >> 1 & 1), zc = 2 * z + (ch & 1);
              const double gx = fmax(fmax(g.lo[0] + xc * sdc - g.margin - qx, qx - (g.lo[0] + (xc + 1) * sdc + g.margin)), 0.0);
              const double gy = fmax(fmax(g.lo[1] + yc * sdc - g.margin - qy, qy - (g.lo[1] + (yc + 1) * sdc + g.margin)), 0.0);
              const double gz = fmax(fmax(g.lo[2] + zc * sdc - g.margin - qz, qz - (g.lo[2] + (zc + 1) * sdc + g.margin)), 0.0);
              if (!((gx * gx + gy * gy) + gz * gz > kd * (1.0 + 1e-12))) {
                const unsigned f = ((spread10((unsigned)xc) << 2) | (spread10((unsigned)yc) << 1) |
                                    spread10((unsigned)zc)) << subc;
                ca = cstart[f];
                cb = cstart[f + (1u << subc)];
              }
            }
            add_cells(ca, cb);
          }
        }
      }
      search(bin_base(kd) - 30);
    }
    // row out: lane t < keff holds entry t
    if (lane < k_out) {
      int o = -1;
      if (lane < keff) o = inv ? inv[best.l] : best.l;
      out[lane] = o;
    }
    __syncthreads();
  }
}

// ---- local neighbourhood refresh (Sec. 3.4) -----------------------------------
// After a pass, parent[o] is the new logical index of old logical index o (both
// ends of a merged pair name the merged splat), nbr_log[o][t] the old list in
// old logical indices.  A new splat is dirty when it was formed by a merge or
// when its old list names a splat that merged; every other splat takes its
// old list carried to the new indices (nothing it listed moved, and the
// entries keep their order, since surviving indices keep theirs).

__global__ void k_refresh_count(const int* __restrict__ parent, int n_old,
                                int* __restrict__ pcount) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o < n_old) atomicAdd(&pcount[parent[o]], 1);
}

// append row to list (one atomic per wave)
NG_DEV void append_row(bool take, int row, int* __restrict__ list, int* __restrict__ count) {
  const unsigned long long m = __ballot(take);
  if (!m) return;
  const int lane = lane_id();
  const int leader = __ffsll((long long)m) - 1;
  int at = 0;
  if (lane == leader) at = atomicAdd(count, __popcll(m));
  at = __shfl(at, leader, 64);
  if (take) list[at + __popcll(m & ((1ull << lane) - 1ull))] = row;
}

// pcount[v] & 3 = old splats that became v (1 or 2); the bits above count
// the ends of a merged pair that have been seen, so that one lists it.
__global__ void k_refresh_rows(const int* __restrict__ parent, int n_old,
                               int* __restrict__ pcount, const int* __restrict__ nbr_log,
                               int k_out, int keff, const int* __restrict__ inv,
                               int* __restrict__ nbr, int* __restrict__ dlist,
                               int* __restrict__ dcount) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  bool dirty = false;
  int row = 0;
  if (o < n_old) {
    const int v = parent[o];
    row = inv[v];
    if ((pcount[v] & 3) == 1) {
      const int* old = nbr_log + (long long)o * k_out;
      for (int t = 0; t < keff; ++t) dirty = dirty || (pcount[parent[old[t]]] & 3) != 1;
      if (!dirty) {
        int* out = nbr + (long long)row * k_out;
        for (int t = 0; t < k_out; ++t) out[t] = t < keff ? inv[parent[old[t]]] : -1;
      }
    } else {
      dirty = atomicAdd(&pcount[v], 4) < 4;  // the first end seen lists it
    }
  }
  append_row(dirty, row, dlist, dcount);
}

// nbr_log[lg[p]][t] = lg[nbr[p][t]] (t < keff), -1 after
__global__ void k_save_log(const int* __restrict__ lg, const int* __restrict__ nbr, int n,
                           int k_out, int keff, int* __restrict__ nbr_log) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * k_out) return;
  const int p = (int)(i / k_out), t = (int)(i % k_out);
  const int e = nbr[i];
  nbr_log[(long long)lg[p] * k_out + t] = t < keff && e >= 0 ? lg[e] : -1;
}

// The one-segment descriptor of the plain entry, written on the device (its
// box from the bounds kernel), so the entry reads nothing back.
__global__ void k_plain_seg(SegInfo* __restrict__ s, const unsigned* __restrict__ box, int n,
                            int LT, int keff, int kclass) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    for (int a = 0; a < 6; ++a) s->box[a] = box[a];
    s->row0 = 0;
    s->nrows = n;
    s->LT = LT;
    s->toff = 0;
    s->keff = keff;
    s->kclass = kclass;
    s->crn = 0;
    s->next = 0;
  }
}

__global__ void k_gather_cen(const float* __restrict__ xyz3, const int* __restrict__ perm, int n,
                             float4* __restrict__ cen) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int i = perm[p];
  cen[p] = make_float4(xyz3[3 * (long long)i], xyz3[3 * (long long)i + 1],
                       xyz3[3 * (long long)i + 2], __int_as_float(i));
}

}  // namespace

// Finest table level of a segment of n rows: one above the smallest level L
// with 8^L >= n (about 1/8 row per cell: surfaces crowd their cells, and a
// query takes coarser levels where it needs them), moved down by the tuned
// bias, between 1 and 8.  8^LT < 64 n bounds the table.
int table_level(long long n) {
  int L = 1;
  while (L < 8 && (1ll << (3 * L)) < n) ++L;
  int LT = L + 1 + tuning_for(n).knn_level_bias;
  if (LT > L + 1) LT = L + 1;
  return LT < 1 ? 1 : (LT > 8 ? 8 : LT);
}

// Upper bound of table_level(n) over every allowed bias (workspace sizing).
int table_level_max(long long n) {
  int L = 1;
  while (L < 8 && (1ll << (3 * L)) < n) ++L;
  return L + 1 > 8 ? 8 : L + 1;
}

int kclass_of(int keff) {
  if (keff <= 0) return 0;
  return keff <= 8 ? 8 : keff <= 16 ? 16 : keff <= 24 ? 24 : 32;
}

long long table_entries(int LT) { return LT > 0 ? (1ll << (3 * LT)) + 1 : 0; }

KnnMem carve_knn(void* base, long long n, long long entries, int kmax, size_t* bytes) {
  Carver c(base);
  KnnMem m;
  m.table = c.take<int>(entries + 1);
  m.inv = c.take<int>(n);
  m.retry = c.take<int2>(n);
  m.ginfo = c.take<int2>(n);
  m.counters = c.take<int>(kKnnCounters);
  // last: its size depends on kmax (builds carve with kmax = 0)
  m.gbuf = c.take<int>(n * (2 * (long long)kclass_of(kmax) + 1));
  if (bytes) *bytes = c.bytes();
  return m;
}

void knn_build(const float4* cen, int n, const int* sg, const SegInfo* dseg, long long entries,
               void* mem, int* d_unsorted, hipStream_t st) {
  KnnMem m = carve_knn(mem, n, entries, 0, nullptr);
  if (n <= 0) return;
  if (entries >= INT_MAX - 2 * kFillChunk)
    throw std::runtime_error("internal: cell tables exceed 2^31 entries");
  // the codes live in the gather buffer (n ints at least), which the
  // queries overwrite later
  int* code = m.gbuf;
  k_cell_codes<<<blocks_for(n, 256), 256, 0, st>>>(cen, n, sg, dseg, code, m.inv, d_unsorted);
  NG_LAUNCH_CHECK();
  k_table_fill<<<(unsigned)(entries / kFillChunk + 1), 64, 0, st>>>(code, n, (int)entries,
                                                                    m.table);
  NG_LAUNCH_CHECK();
}

// list (device, nullable): query only the rows list[0, *d_count) (the grids
// cover n rows)
template <int K>
void query_k(const float4* cen, int n, int k_out, const int* sg, const SegInfo* dseg,
             const KnnMem& m, const int* inv, int rows_logical, int* nbr, StageTimer* T,
             hipStream_t st, const int* list = nullptr, const int* d_count = nullptr) {
  const Tuning& t = tuning_for(n);
  const int bs = t.knn_block;
  int tk = T ? T->start(NANOGS_T_KNN_QUERY) : -1;
  constexpr int Q = kKnnLanes;
  k_knn_block<K, Q><<<blocks_for((long long)n * Q, bs), bs, (size_t)(kHistWords + 1) * (bs / Q) * sizeof(unsigned),
                      st>>>(cen, n, sg, dseg, m.table, t.knn_block_min, t.knn_lane_rows, m.gbuf,
                            m.ginfo, (unsigned long long*)(m.counters + kScreenBase), list,
                            d_count);
  NG_LAUNCH_CHECK();
  if (T) T->stop(tk);
  tk = T ? T->start(NANOGS_T_KNN_EXACT) : -1;
  constexpr int QE = kExactLanes;
  static_assert(2 * K % QE == 0, "exact-pass lanes must divide the buffer");
  k_knn_exact<K, QE><<<blocks_for((long long)n * QE, 64 * kExactWaves), 64 * kExactWaves, 0, st>>>(
      cen, n, k_out, sg, dseg, m.table, inv, rows_logical, nbr, m.gbuf, m.ginfo, m.retry,
      m.counters + 1, list, d_count);
  NG_LAUNCH_CHECK();
  if (T) T->stop(tk);
}

template <int K>
void query_wave_k(const float4* cen, int n, int k_out, const int* sg, const SegInfo* dseg,
                  const KnnMem& m, const int* inv, int rows_logical, int* nbr, StageTimer* T,
                  hipStream_t st) {
  const int tk = T ? T->start(NANOGS_T_KNN_WAVE) : -1;
  // the retry count stays on the device: a grid of fixed size strides over it
  const int cap = tuning_for(n).knn_wave_grid;
  unsigned g = (unsigned)(n < cap ? n : cap);
  if (g < 1) g = 1;
  k_knn_wave<K><<<g, 64, 0, st>>>(cen, n, k_out, sg, dseg, m.table, inv, rows_logical,
                                  tuning_for(n).knn_block_min, nbr, m.retry, m.counters + 1);
  NG_LAUNCH_CHECK();
  if (T) T->stop(tk);
}

void knn_query(const float4* cen, int n, int k_out, const int* sg, const SegInfo* dseg,
               unsigned class_mask, long long entries, void* mem, bool use_inv, int rows_logical,
               int* nbr, StageTimer* T, hipStream_t st) {
  KnnMem m = carve_knn(mem, n, entries, k_out, nullptr);
  const int* inv = use_inv ? m.inv : nullptr;
  if (n <= 0) return;
  // (counters: [1] retries, the screen slots from kScreenBase)
  k_knn_prefill<<<blocks_for(std::max(n, kKnnCounters), 256), 256, 0, st>>>(
      n, sg, dseg, k_out, nbr, m.counters + 1, kKnnCounters - 1);
  NG_LAUNCH_CHECK();
  if (class_mask & 1u) query_k<8>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, T, st);
  if (class_mask & 2u) query_k<16>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, T, st);
  if (class_mask & 4u) query_k<24>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, T, st);
  if (class_mask & 8u) query_k<32>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, T, st);
  // retries (unordered: each query's result does not depend on the order)
  if (class_mask & 1u) query_wave_k<8>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, T, st);
  if (class_mask & 2u) query_wave_k<16>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, T, st);
  if (class_mask & 4u) query_wave_k<24>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, T, st);
  if (class_mask & 8u) query_wave_k<32>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, T, st);
}

void knn_refresh(const float4* cen, int n_new, int n_old, int k_out, int keff, const int* sg,
                 const SegInfo* dseg, long long entries, void* mem, const int* parent,
                 int* pcount, const int* nbr_log, int* dlist, int* dcount, int* nbr, StageTimer* T,
                 hipStream_t st) {
  KnnMem m = carve_knn(mem, n_new, entries, k_out, nullptr);
  fill_i32(pcount, 0, n_new, st);
  fill_i32(dcount, 0, 1, st);
  fill_i32(m.counters + 1, 0, 1, st);
  fill_i32(m.counters + kScreenBase, 0, kScreenSlots * kScreenStride, st);
  if (n_old > 0) {
    k_refresh_count<<<blocks_for(n_old, 256), 256, 0, st>>>(parent, n_old, pcount);
    NG_LAUNCH_CHECK();
    k_refresh_rows<<<blocks_for(n_old, 256), 256, 0, st>>>(parent, n_old, pcount, nbr_log, k_out,
                                                          keff, m.inv, nbr, dlist, dcount);
    NG_LAUNCH_CHECK();
  }
  switch (kclass_of(keff)) {
    case 8: query_k<8>(cen, n_new, k_out, sg, dseg, m, m.inv, 0, nbr, T, st, dlist, dcount);
            query_wave_k<8>(cen, n_new, k_out, sg, dseg, m, m.inv, 0, nbr, T, st); break;
    case 16: query_k<16>(cen, n_new, k_out, sg, dseg, m, m.inv, 0, nbr, T, st, dlist, dcount);
             query_wave_k<16>(cen, n_new, k_out, sg, dseg, m, m.inv, 0, nbr, T, st); break;
    case 24: query_k<24>(cen, n_new, k_out, sg, dseg, m, m.inv, 0, nbr, T, st, dlist, dcount);
             query_wave_k<24>(cen, n_new, k_out, sg, dseg, m, m.inv, 0, nbr, T, st); break;
    default: query_k<32>(cen, n_new, k_out, sg, dseg, m, m.inv, 0, nbr, T, st, dlist, dcount);
             query_wave_k<32>(cen, n_new, k_out, sg, dseg, m, m.inv, 0, nbr, T, st); break;
  }
}

void knn_save_log(const int* lg, const int* nbr, int n, int k_out, int keff, int* nbr_log,
                  hipStream_t st) {
  if (n <= 0) return;
  k_save_log<<<blocks_for((long long)n * k_out, 256), 256, 0, st>>>(lg, nbr, n, k_out, keff,
                                                                     nbr_log);
  NG_LAUNCH_CHECK();
}

unsigned class_bit(int kclass) {
  return kclass == 8 ? 1u : kclass == 16 ? 2u : kclass == 24 ? 4u : kclass == 32 ? 8u : 0u;
}

void launch_morton_keys(const float* pos_xyz3, const float4* cen4, int n, unsigned* keys,
                        void* temp, hipStream_t st) {
  unsigned* box = (unsigned*)temp;
  // mins start at the largest key, maxima at the smallest
  fill_i32((int*)box, -1, 3, st);
  fill_i32((int*)box + 3, 0, 3, st);
  unsigned b = blocks_for(n, 256);
  if (b > 256) b = 256;
  k_bbox<<<b, 256, 0, st>>>(pos_xyz3, cen4, n, box);
  NG_LAUNCH_CHECK();
  k_morton<<<blocks_for(n, 256), 256, 0, st>>>(pos_xyz3, cen4, n, box, keys);
  NG_LAUNCH_CHECK();
}

// Plain entry: centres in caller order -> Morton-sorted copy -> one-segment
// table -> rows by caller index.
size_t knn_plain_bytes(long long n, int k) {
  Carver c(nullptr);
  c.take<unsigned>(64);
  c.take<unsigned>(n);
  c.take<int>(n);
  c.take<float4>(n);
  c.take<SegInfo>(1);
  size_t kb = 0;
  carve_knn(nullptr, n, table_entries(table_level_max(n)), k, &kb);
  return c.bytes() + std::max(kb, sort_temp_bytes(n));
}

void knn_plain(const float* mu, int n, int k, int keff, int* nbr, void* ws, hipStream_t st) {
  Carver c(ws);
  unsigned* boxmem = c.take<unsigned>(64);
  unsigned* keys = c.take<unsigned>(n);
  int* perm = c.take<int>(n);
  float4* cen = c.take<float4>(n);
  SegInfo* dseg = c.take<SegInfo>(1);
  void* rest = (char*)ws + c.bytes();
  launch_morton_keys(mu, nullptr, n, keys, boxmem, st);
  k_iota<<<blocks_for(n, 256), 256, 0, st>>>(perm, n);
  NG_LAUNCH_CHECK();
  sort_pairs_u32(keys, perm, n, kSortKeyBits, rest, st);
  k_gather_cen<<<blocks_for(n, 256), 256, 0, st>>>(mu, perm, n, cen);
  NG_LAUNCH_CHECK();
  const int LT = table_level(n);
  const int kclass = kclass_of(keff);
  k_plain_seg<<<1, 64, 0, st>>>(dseg, boxmem, n, LT, keff, kclass);
  NG_LAUNCH_CHECK();
  const long long entries = table_entries(LT);
  KnnMem m = carve_knn(rest, n, entries, k, nullptr);
  fill_i32(m.counters, 0, 1, st);  // order check: sorted above by the same keys
  knn_build(cen, n, nullptr, dseg, entries, rest, m.counters, st);
  knn_query(cen, n, k, nullptr, dseg, class_bit(kclass), entries, rest, false, 1, nbr, nullptr, st);
}

}  // namespace ng
