// Exact k-nearest-neighbour graph over splat centres (Sec. 3.1).
//
// Spatial structure: the working array is kept sorted by the 30-bit Morton
// key of the centres (quantised on a 1024^3 grid over the bounding cube), so
// every octree cell is a contiguous range of rows; a table of cell starts at
// one level gives the range of any cell at that level or coarser.
//
// Query, in two kernels.  A query whose own finest-level cell holds at least
// k+1 rows (dense surroundings) is served by one lane: it scans that cell,
// then rings of neighbouring cells, skipping cells beyond the current k-th
// distance, and stops when the k-th distance is inside the searched block
// (cells are disjoint, so every unseen row is farther).  The other queries
// are served by a whole wave each, at a coarser level: the lanes share the
// cells and rows and hold the k best one entry per lane, so a query near a
// dense surface costs its rows / 64 steps instead of stalling 63 idle lanes.
// Candidates are screened in float against a bound derived from the current
// k-th key (never rejecting a point that the exact key would keep); survivors
// get the exact key (d2, logical index) with d2 = ((dx*dx + dy*dy) + dz*dz)
// in double without contraction.  The result is the exact kNN with ties
// broken by index.
#include <algorithm>
#include <cstring>
#include <climits>

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
  keys[i] = morton_key(v[0], v[1], v[2], box);
}

__global__ void k_iota(int* v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// ---- cell table ------------------------------------------------------------
// The working array is sorted by the 30-bit Morton key of the centres, so
// every octree cell (a Morton prefix of 3L bits at level L) is a contiguous
// range of rows.  The table holds, for every cell c of level LT, the first row
// whose level-LT cell is >= c (cstart[ncells] = n); a cell of a coarser level
// L is the range [cstart[c << 3(LT-L)], cstart[(c+1) << 3(LT-L)]).

// hist[toff + c] = rows of segment sid in its level-LT cell c, from the run
// boundaries of the sorted keys (each run adds its end and subtracts its
// start); flags a key that is smaller than its predecessor in the segment.
// Segments without a table (LT = 0) are skipped.
__global__ void k_cell_runs(const float4* __restrict__ cen, int n, const int* __restrict__ sg,
                            const SegInfo* __restrict__ seg, int* __restrict__ hist,
                            int* __restrict__ unsorted) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const SegInfo& S = seg[sg ? sg[i] : 0];
  if (S.LT <= 0) return;
  const int shift = 3 * (10 - S.LT);
  const float4 c = cen[i];
  const unsigned key = morton_key(c.x, c.y, c.z, S.box);
  const unsigned cell = key >> shift;
  const bool first = i == S.row0;
  const bool last = i + 1 == S.row0 + S.nrows;
  unsigned prev_key = 0u, next_cell = ~0u;
  if (!first) {
    const float4 a = cen[i - 1];
    prev_key = morton_key(a.x, a.y, a.z, S.box);
  }
  if (!last) {
    const float4 b = cen[i + 1];
    next_cell = morton_key(b.x, b.y, b.z, S.box) >> shift;
  }
  if (!first && prev_key > key) atomicOr(unsorted, 1);
  if (first || (prev_key >> shift) != cell) atomicAdd(&hist[S.toff + cell], -(i - S.row0));
  if (last || next_cell != cell) atomicAdd(&hist[S.toff + cell], i - S.row0 + 1);
}

// Rows of segments without a search (inert): empty lists.  Every row starts
// as not sparse.
__global__ void k_knn_prefill(int n, const int* __restrict__ sg, const SegInfo* __restrict__ seg,
                              int k_out, int* __restrict__ nbr, int* __restrict__ sparse_flag) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  sparse_flag[p] = 0;
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

// Exact k-NN of one query over the cell table at the finest level LT, for
// queries whose own cell holds at least K + 1 rows (so the own cell alone
// fills the list and the k-th distance is at most the cell's diagonal: the
// search never needs more than rings 1 and 2); the others are flagged in
// sparse_flag for k_knn_wave.  Search:
// the query's own cell, then rings R = 1, 2, ... of level-L cells (the cells
// at Chebyshev distance R), skipping cells whose box (widened by the
// quantisation margin) is beyond the current k-th key.  After ring R the
// block of (2R+1)^3 cells around the query's cell has been searched; the
// search stops once the k-th key is closer than the block's boundary (faces
// on the grid's outer boundary do not count: no row lies beyond them), since
// every row outside the block is then farther.  Cells are disjoint, so no row
// is seen twice.
template <int K>
__global__ void __launch_bounds__(256)
k_knn_grid(const float4* __restrict__ cen, int n, int k_out, const int* __restrict__ sg,
           const SegInfo* __restrict__ seg, const int* __restrict__ table,
           const int* __restrict__ inv, int rows_logical, int* __restrict__ nbr,
           int* __restrict__ sparse_flag) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const SegInfo& S = seg[sg ? sg[p] : 0];
  if (S.kclass != K) return;  // another launch (or none: inert) serves it
  const int keff = S.keff;
  const int LT = S.LT;
  const unsigned* box = S.box;
  const int* cstart = table + S.toff;
  const int rb = S.row0 - cstart[0];  // table values -> rows
  const float4 cq = cen[p];
  const double qx = cq.x, qy = cq.y, qz = cq.z;
  const float qxf = cq.x, qyf = cq.y, qzf = cq.z;
  const Grid g = grid_from_box(box);
  float lof[3], hif[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lof[a] = ord2f(box[a]);
    hif[a] = ord2f(box[3 + a]);
  }
  const float ext = fmaxf(fmaxf(hif[0] - lof[0], hif[1] - lof[1]), hif[2] - lof[2]);
  const float sc = ext > 0.f ? 1023.0f / ext : 0.f;
  const unsigned qi[3] = {quant(qxf, lof[0], sc), quant(qyf, lof[1], sc), quant(qzf, lof[2], sc)};

  // Queries whose own finest-level cell holds fewer than K + 1 rows (sparse
  // surroundings) are flagged for k_knn_wave instead.
  const int L = LT;
  {
    const unsigned mc = (spread10(qi[0] >> (10 - L)) << 2) | (spread10(qi[1] >> (10 - L)) << 1) |
                        spread10(qi[2] >> (10 - L));
    const int cnt = cstart[mc + 1] - cstart[mc];
    const bool sparse = cnt < K + 1 && sc > 0.f;
    sparse_flag[p] = sparse ? 1 : 0;
    if (sparse) return;
  }
  const int s = 10 - L;
  const int G = 1 << L;
  const int sub = 3 * (LT - L);
  const double side = (double)(1 << s) * g.inv_sc;
  const int cx = (int)(qi[0] >> s), cy = (int)(qi[1] >> s), cz = (int)(qi[2] >> s);

  Best<K> best;
  best.init();
  float thr = INFINITY;
  auto scan = [&](int a, int b) {
    for (int j = a; j < b; ++j) {
      const float4 c = cen[j];
      const float dx = qxf - c.x, dy = qyf - c.y, dz = qzf - c.z;
      if (dx * dx + dy * dy + dz * dz <= thr && j != p)
        best.consider(dist2(qx, qy, qz, c.x, c.y, c.z), __float_as_int(c.w));
    }
    thr = admit_bound(best.d[K - 1]);
  };
  auto cell_range = [&](int x, int y, int z, int& a, int& b) {
    const unsigned mc = (spread10((unsigned)x) << 2) | (spread10((unsigned)y) << 1) |
                        spread10((unsigned)z);
    const unsigned f = mc << sub;
    a = cstart[f] + rb;
    b = cstart[f + (1u << sub)] + rb;
  };
  {
    int a, b;
    cell_range(cx, cy, cz, a, b);
    scan(a, b);
  }
  // a zero-extent grid has every row in one cell: the own cell was all
  for (int R = 1; sc > 0.f; ++R) {
    for (int dx = -R; dx <= R; ++dx) {
      const int x = cx + dx;
      if (x < 0 || x >= G) continue;
      for (int dy = -R; dy <= R; ++dy) {
        const int y = cy + dy;
        if (y < 0 || y >= G) continue;
        const bool edge_xy = dx == -R || dx == R || dy == -R || dy == R;
        for (int dz = -R; dz <= R; dz += (edge_xy ? 1 : 2 * R)) {
          const int z = cz + dz;
          if (z < 0 || z >= G) continue;
          // distance from the query to the cell's widened box, in double
          const double bx0 = g.lo[0] + x * side - g.margin, bx1 = g.lo[0] + (x + 1) * side + g.margin;
          const double by0 = g.lo[1] + y * side - g.margin, by1 = g.lo[1] + (y + 1) * side + g.margin;
          const double bz0 = g.lo[2] + z * side - g.margin, bz1 = g.lo[2] + (z + 1) * side + g.margin;
          const double gx = fmax(fmax(bx0 - qx, qx - bx1), 0.0);
          const double gy = fmax(fmax(by0 - qy, qy - by1), 0.0);
          const double gz = fmax(fmax(bz0 - qz, qz - bz1), 0.0);
          const double bd = (gx * gx + gy * gy) + gz * gz;
          if (bd > best.d[K - 1] * (1.0 + 1e-12)) continue;
          int a, b;
          cell_range(x, y, z, a, b);
          if (b > a) scan(a, b);
        }
      }
    }
    // distance from the query to the boundary of the searched block (shrunk
    // by the margin); faces on the grid boundary are open
    double rho = INFINITY;
    if (cx - R > 0) rho = fmin(rho, qx - (g.lo[0] + (cx - R) * side + g.margin));
    if (cx + R + 1 < G) rho = fmin(rho, (g.lo[0] + (cx + R + 1) * side - g.margin) - qx);
    if (cy - R > 0) rho = fmin(rho, qy - (g.lo[1] + (cy - R) * side + g.margin));
    if (cy + R + 1 < G) rho = fmin(rho, (g.lo[1] + (cy + R + 1) * side - g.margin) - qy);
    if (cz - R > 0) rho = fmin(rho, qz - (g.lo[2] + (cz - R) * side + g.margin));
    if (cz + R + 1 < G) rho = fmin(rho, (g.lo[2] + (cz + R + 1) * side - g.margin) - qz);
    if (!(rho < INFINITY)) break;  // the block covers the whole grid
    if (rho > 0.0 && rho * rho * (1.0 - 1e-9) > best.d[K - 1]) break;
  }

  const long long row = rows_logical ? (long long)__float_as_int(cq.w) : (long long)p;
  int* out = nbr + row * k_out;
#pragma unroll
  for (int t = 0; t < K; ++t) {
    if (t < k_out) {
      int o = -1;
      if (t < keff) o = inv ? inv[best.l[t]] : best.l[t];
      out[t] = o;
    }
  }
  for (int t = K; t < k_out; ++t) out[t] = -1;
}

// ---- sparse queries ------------------------------------------------------------
// Exact k-NN of the sparse queries, one wave per query.  Level: the finest
// L < LT whose cell around the query holds at least K + 1 rows (or level 1),
// so rings 1 and 2 suffice as in k_knn_grid.  The lanes share the work: the
// cells of a ring are tested one per lane (box against the current k-th
// distance), the rows of the cells that pass are dealt out 64 at a time, and
// the k best live one entry per lane (lanes 0..K-1, sorted), so an insertion
// is a ballot and a shift.  The own cell is scanned first.
template <int K>
struct WaveBest {
  double d;  // entry of this lane (lanes >= K hold +inf)
  int l;

  NG_DEV void init() {
    d = INFINITY;
    l = INT_MAX;
  }
  NG_DEV double kth() const {
    const int lo = __shfl(__double2loint(d), K - 1, 64);
    const int hi = __shfl(__double2hiint(d), K - 1, 64);
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
           const int* __restrict__ inv, int rows_logical, int* __restrict__ nbr,
           const int* __restrict__ list, const int* __restrict__ d_count) {
  __shared__ int s_start[128];
  __shared__ int s_pref[129];
  const int lane = threadIdx.x;
  const int count = *d_count;
  for (int qidx = blockIdx.x; qidx < count; qidx += gridDim.x) {
    const int p = list[qidx];
    const SegInfo& S = seg[sg ? sg[p] : 0];
    if (S.kclass != K) continue;  // wave-uniform: one query per wave
    const int keff = S.keff;
    const int LT = S.LT;
    const unsigned* box = S.box;
    const int* cstart = table + S.toff;
    const int rb = S.row0 - cstart[0];
    const Grid g = grid_from_box(box);
    float lof[3], hif[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lof[a] = ord2f(box[a]);
      hif[a] = ord2f(box[3 + a]);
    }
    const float ext = fmaxf(fmaxf(hif[0] - lof[0], hif[1] - lof[1]), hif[2] - lof[2]);
    const float sc = ext > 0.f ? 1023.0f / ext : 0.f;
    const float4 cq = cen[p];
    const double qx = cq.x, qy = cq.y, qz = cq.z;
    const float qxf = cq.x, qyf = cq.y, qzf = cq.z;
    const unsigned qi[3] = {quant(qxf, lof[0], sc), quant(qyf, lof[1], sc),
                            quant(qzf, lof[2], sc)};
    int L = LT - 1 >= 1 ? LT - 1 : 1;
    while (L > 1) {
      const int sl = 10 - L;
      const unsigned mc = (spread10(qi[0] >> sl) << 2) | (spread10(qi[1] >> sl) << 1) |
                          spread10(qi[2] >> sl);
      const unsigned f = mc << (3 * (LT - L));
      if (cstart[f + (1u << (3 * (LT - L)))] - cstart[f] >= K + 1) break;
      --L;
    }
    const int sl = 10 - L;
    const int G = 1 << L;
    const int sub = 3 * (LT - L);
    const double side = (double)(1 << sl) * g.inv_sc;
    const int cx = (int)(qi[0] >> sl), cy = (int)(qi[1] >> sl), cz = (int)(qi[2] >> sl);
    WaveBest<K> best;
    best.init();

    // scans the rows of the cells listed in s_start / s_pref (ncell cells)
    auto scan_cells = [&](int ncell) {
      const int total = s_pref[ncell];
      for (int t0 = 0; t0 < total; t0 += 64) {
        const int t = t0 + lane;
        bool pass = false;
        int j = -1;
        float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
        const float thr = admit_bound(best.kth());
        if (t < total) {
          int lo = 0, hi = ncell - 1;  // last cell with s_pref <= t
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pref[mid] <= t) lo = mid; else hi = mid - 1;
          }
          j = s_start[lo] + (t - s_pref[lo]);
          c = cen[j];
          const float dx = qxf - c.x, dy = qyf - c.y, dz = qzf - c.z;
          pass = dx * dx + dy * dy + dz * dz <= thr && j != p;
        }
        unsigned long long m = __ballot(pass);
        const double dme = pass ? dist2(qx, qy, qz, c.x, c.y, c.z) : 0.0;
        const int lme = __float_as_int(c.w);
        while (m) {
          const int src = __ffsll((long long)m) - 1;
          m &= m - 1;
          const int dlo = __shfl(__double2loint(dme), src, 64);
          const int dhi = __shfl(__double2hiint(dme), src, 64);
          const int ls = __shfl(lme, src, 64);
          best.insert(__hiloint2double(dhi, dlo), ls);
        }
      }
    };
    // own cell
    {
      const unsigned mc = (spread10((unsigned)cx) << 2) | (spread10((unsigned)cy) << 1) |
                          spread10((unsigned)cz);
      const unsigned f = mc << sub;
      if (lane == 0) {
        s_start[0] = cstart[f] + rb;
        s_pref[0] = 0;
        s_pref[1] = cstart[f + (1u << sub)] - cstart[f];
      }
      __syncthreads();
      scan_cells(1);
      __syncthreads();
    }
    for (int R = 1; sc > 0.f; ++R) {
      // cells of ring R, enumerated over the (2R+1)^3 cube, 64 per step
      const int side_n = 2 * R + 1;
      const int ncube = side_n * side_n * side_n;
      for (int c0 = 0; c0 < ncube; c0 += 64) {
        const int ci = c0 + lane;
        const double kd = best.kth();  // wave-uniform, read before any branch
        int a = 0, b = 0;
        if (ci < ncube) {
          const int dx = ci % side_n - R, dy = (ci / side_n) % side_n - R, dz = ci / (side_n * side_n) - R;
          const int x = cx + dx, y = cy + dy, z = cz + dz;
          const bool on_ring = max(max(abs(dx), abs(dy)), abs(dz)) == R;
          if (on_ring && x >= 0 && x < G && y >= 0 && y < G && z >= 0 && z < G) {
            const double bx0 = g.lo[0] + x * side - g.margin, bx1 = g.lo[0] + (x + 1) * side + g.margin;
            const double by0 = g.lo[1] + y * side - g.margin, by1 = g.lo[1] + (y + 1) * side + g.margin;
            const double bz0 = g.lo[2] + z * side - g.margin, bz1 = g.lo[2] + (z + 1) * side + g.margin;
            const double gx = fmax(fmax(bx0 - qx, qx - bx1), 0.0);
            const double gy = fmax(fmax(by0 - qy, qy - by1), 0.0);
            const double gz = fmax(fmax(bz0 - qz, qz - bz1), 0.0);
            const double bd = (gx * gx + gy * gy) + gz * gz;
            if (!(bd > kd * (1.0 + 1e-12))) {
              const unsigned mc = (spread10((unsigned)x) << 2) | (spread10((unsigned)y) << 1) |
                                  spread10((unsigned)z);
              const unsigned f = mc << sub;
              a = cstart[f] + rb;
              b = cstart[f + (1u << sub)] + rb;
            }
          }
        }
        // compact the non-empty cells of this step into s_start / s_pref
        const bool has = b > a;
        const unsigned long long hm = __ballot(has);
        const int rank = __popcll(hm & (lane == 0 ? 0ull : (~0ull >> (64 - lane))));
        int cnt = has ? b - a : 0;
        int incl = cnt;  // inclusive prefix of counts over the non-empty cells
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const int y = __shfl_up(incl, d, 64);
          if (lane >= d) incl += y;
        }
        if (has) {
          s_start[rank] = a;
          s_pref[rank] = incl - cnt;
        }
        const int ncell = __popcll(hm);
        if (lane == 63) s_pref[ncell] = incl;
        __syncthreads();
        if (ncell > 0) scan_cells(ncell);
        __syncthreads();
      }
      double rho = INFINITY;
      if (cx - R > 0) rho = fmin(rho, qx - (g.lo[0] + (cx - R) * side + g.margin));
      if (cx + R + 1 < G) rho = fmin(rho, (g.lo[0] + (cx + R + 1) * side - g.margin) - qx);
      if (cy - R > 0) rho = fmin(rho, qy - (g.lo[1] + (cy - R) * side + g.margin));
      if (cy + R + 1 < G) rho = fmin(rho, (g.lo[1] + (cy + R + 1) * side - g.margin) - qy);
      if (cz - R > 0) rho = fmin(rho, qz - (g.lo[2] + (cz - R) * side + g.margin));
      if (cz + R + 1 < G) rho = fmin(rho, (g.lo[2] + (cz + R + 1) * side - g.margin) - qz);
      if (!(rho < INFINITY)) break;
      if (rho > 0.0 && rho * rho * (1.0 - 1e-9) > best.kth()) break;
    }
    // row out: lane t < keff holds entry t
    const long long row = rows_logical ? (long long)__float_as_int(cq.w) : (long long)p;
    int* out = nbr + row * k_out;
    if (lane < k_out) {
      int o = -1;
      if (lane < keff) o = inv ? inv[best.l] : best.l;
      out[lane] = o;
    }
    __syncthreads();
  }
}

__global__ void k_scatter_flagged(const int* __restrict__ flag, const int* __restrict__ pos, int n,
                                  int* __restrict__ list) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n && flag[p]) list[pos[p]] = p;
}

__global__ void k_invert(const float4* __restrict__ cen, int n, int* __restrict__ inv) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) inv[__float_as_int(cen[p].w)] = p;
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

// Finest table level of a segment of n rows: about 8^L >= n (moved by the
// tuned bias), between 1 and 7.
int table_level(long long n) {
  int L = 1;
  while (L < 7 && (1ll << (3 * L)) < n) ++L;
  L += tuning_for(n).knn_level_bias;
  return L < 1 ? 1 : (L > 7 ? 7 : L);
}

// Upper bound of table_level(n) over every allowed bias (workspace sizing).
int table_level_max(long long n) {
  int L = 1;
  while (L < 7 && (1ll << (3 * L)) < n) ++L;
  return L + 1 > 7 ? 7 : L + 1;
}

int kclass_of(int keff) {
  if (keff <= 0) return 0;
  return keff <= 8 ? 8 : keff <= 16 ? 16 : keff <= 24 ? 24 : 32;
}

long long table_entries(int LT) { return LT > 0 ? (1ll << (3 * LT)) + 1 : 0; }

KnnMem carve_knn(void* base, long long n, long long entries, size_t* bytes) {
  Carver c(base);
  KnnMem m;
  m.hist = c.take<int>(entries + 1);
  m.table = c.take<int>(entries + 1);
  m.inv = c.take<int>(n);
  m.sflag = c.take<int>(n);
  m.spos = c.take<int>(n);
  m.sparse = c.take<int>(n);
  m.counters = c.take<int>(64);
  const size_t scan = std::max(scan_temp_bytes(entries + 1), scan_temp_bytes(n));
  m.scan_temp = base ? (char*)base + c.bytes() : nullptr;
  if (bytes) *bytes = c.bytes() + scan;
  return m;
}

void knn_build(const float4* cen, int n, const int* sg, const SegInfo* dseg, long long entries,
               void* mem, int* d_unsorted, bool invert, hipStream_t st) {
  KnnMem m = carve_knn(mem, n, entries, nullptr);
  fill_i32(m.hist, 0, entries + 1, st);
  k_cell_runs<<<blocks_for(n, 256), 256, 0, st>>>(cen, n, sg, dseg, m.hist, d_unsorted);
  NG_LAUNCH_CHECK();
  scan_exclusive_i32(m.hist, m.table, entries + 1, nullptr, m.scan_temp, st);
  if (invert) {
    k_invert<<<blocks_for(n, 256), 256, 0, st>>>(cen, n, m.inv);
    NG_LAUNCH_CHECK();
  }
}

template <int K>
void query_k(const float4* cen, int n, int k_out, const int* sg, const SegInfo* dseg,
             const KnnMem& m, const int* inv, int rows_logical, int* nbr, hipStream_t st) {
  const int bs = tuning_for(n).knn_block;
  k_knn_grid<K><<<blocks_for(n, bs), bs, 0, st>>>(cen, n, k_out, sg, dseg, m.table, inv,
                                                  rows_logical, nbr, m.sflag);
  NG_LAUNCH_CHECK();
}

template <int K>
void query_wave_k(const float4* cen, int n, int k_out, const int* sg, const SegInfo* dseg,
                  const KnnMem& m, const int* inv, int rows_logical, int* nbr, hipStream_t st) {
  // the sparse count stays on the device: a grid of fixed size strides over it
  const int cap = tuning_for(n).knn_wave_grid;
  unsigned g = (unsigned)(n < cap ? n : cap);
  if (g < 1) g = 1;
  k_knn_wave<K><<<g, 64, 0, st>>>(cen, n, k_out, sg, dseg, m.table, inv, rows_logical, nbr,
                                  m.sparse, m.counters + 1);
  NG_LAUNCH_CHECK();
}

void knn_query(const float4* cen, int n, int k_out, const int* sg, const SegInfo* dseg,
               unsigned class_mask, long long entries, void* mem, bool use_inv, int rows_logical,
               int* nbr, hipStream_t st) {
  KnnMem m = carve_knn(mem, n, entries, nullptr);
  const int* inv = use_inv ? m.inv : nullptr;
  k_knn_prefill<<<blocks_for(n, 256), 256, 0, st>>>(n, sg, dseg, k_out, nbr, m.sflag);
  NG_LAUNCH_CHECK();
  if (class_mask & 1u) query_k<8>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, st);
  if (class_mask & 2u) query_k<16>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, st);
  if (class_mask & 4u) query_k<24>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, st);
  if (class_mask & 8u) query_k<32>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, st);
  // sparse queries, compacted in working (Morton) order
  scan_exclusive_i32(m.sflag, m.spos, n, m.counters + 1, m.scan_temp, st);
  k_scatter_flagged<<<blocks_for(n, 256), 256, 0, st>>>(m.sflag, m.spos, n, m.sparse);
  NG_LAUNCH_CHECK();
  if (class_mask & 1u) query_wave_k<8>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, st);
  if (class_mask & 2u) query_wave_k<16>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, st);
  if (class_mask & 4u) query_wave_k<24>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, st);
  if (class_mask & 8u) query_wave_k<32>(cen, n, k_out, sg, dseg, m, inv, rows_logical, nbr, st);
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
size_t knn_plain_bytes(long long n) {
  Carver c(nullptr);
  c.take<unsigned>(64);
  c.take<unsigned>(n);
  c.take<int>(n);
  c.take<float4>(n);
  c.take<SegInfo>(1);
  size_t kb = 0;
  carve_knn(nullptr, n, table_entries(table_level_max(n)), &kb);
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
  sort_pairs_u32(keys, perm, n, 30, rest, st);
  k_gather_cen<<<blocks_for(n, 256), 256, 0, st>>>(mu, perm, n, cen);
  NG_LAUNCH_CHECK();
  SegInfo h;
  std::memset(&h, 0, sizeof(h));
  h.row0 = 0;
  h.nrows = n;
  h.LT = table_level(n);
  h.toff = 0;
  h.keff = keff;
  h.kclass = kclass_of(keff);
  NG_HIP(hipMemcpyAsync(dseg, &h, sizeof(h), hipMemcpyHostToDevice, st));
  NG_HIP(hipMemcpyAsync(dseg->box, boxmem, 6 * sizeof(unsigned), hipMemcpyDeviceToDevice, st));
  const long long entries = table_entries(h.LT);
  KnnMem m = carve_knn(rest, n, entries, nullptr);
  fill_i32(m.counters, 0, 1, st);  // order check: sorted above by the same keys
  knn_build(cen, n, nullptr, dseg, entries, rest, m.counters, false, st);
  knn_query(cen, n, k, nullptr, dseg, class_bit(h.kclass), entries, rest, false, 1, nbr, st);
  // the host copy of h must outlive the async copy
  NG_HIP(hipStreamSynchronize(st));
}

}  // namespace ng
