// Exact k-nearest-neighbour graph over splat centres (Sec. 3.1).
//
// Spatial structure: the splats sit in the working array in (near) Morton
// order; consecutive runs of 16 form leaf buckets, and a complete binary tree
// over the buckets (heap numbering: root 1, children 2i and 2i+1, leaves from
// nb2) stores an axis-aligned box per node.  The tree is correct for ANY
// order of the array (boxes are computed from the points); Morton order only
// keeps the boxes tight.  Rebuilding it costs one pass over the centres, so it
// is rebuilt every round without re-sorting.
//
// Query: one thread per query splat, consecutive threads = neighbouring
// splats, so the lanes of a wave walk nearly the same nodes.  The k best
// (d2, logical index) pairs live in registers, sorted.  The query's own
// bucket and its two neighbours in the array seed the list, then a stackless
// left-first walk visits every node whose box is within the current k-th
// distance (<=, so exact ties are still resolved by index).  Distances and
// box bounds are double, evaluated as ((dx*dx + dy*dy) + dz*dz) without
// contraction: the box bound never exceeds the distance of a point inside the
// box (rounding is monotone), so pruning is exact.
#include <climits>

#include "internal.h"

namespace ng {
namespace {

constexpr int LEAF = 16;

// ---- Morton keys -----------------------------------------------------------
__global__ void k_bbox(const float* __restrict__ xyz3, const float4* __restrict__ cen4, int n,
                       unsigned* __restrict__ box) {
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
  if (lane_id() == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      atomicMin(&box[a], f2ord(mn[a]));
      atomicMax(&box[3 + a], f2ord(mx[a]));
    }
  }
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

__global__ void k_morton(const float* __restrict__ xyz3, const float4* __restrict__ cen4, int n,
                         const unsigned* __restrict__ box, unsigned* __restrict__ keys) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = ord2f(box[a]);
    hi[a] = ord2f(box[3 + a]);
  }
  float ext = fmaxf(fmaxf(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
  float sc = ext > 0.f ? 1023.0f / ext : 0.f;
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
  unsigned q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float t = (v[a] - lo[a]) * sc;
    t = fminf(fmaxf(t, 0.f), 1023.f);
    q[a] = (unsigned)t;
  }
  keys[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
}

__global__ void k_iota(int* v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// ---- tree ------------------------------------------------------------------
struct Box {
  float lx, ly, lz, hx, hy, hz;
};

NG_DEV Box box_empty() { return {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY}; }

NG_DEV Box box_join(const Box& a, const Box& b) {
  return {fminf(a.lx, b.lx), fminf(a.ly, b.ly), fminf(a.lz, b.lz),
          fmaxf(a.hx, b.hx), fmaxf(a.hy, b.hy), fmaxf(a.hz, b.hz)};
}

NG_DEV void box_store(float4* bmin, float4* bmax, long long node, const Box& b) {
  bmin[node] = make_float4(b.lx, b.ly, b.lz, 0.f);
  bmax[node] = make_float4(b.hx, b.hy, b.hz, 0.f);
}

// Builds up to 8 levels of the tree per block, from 256 consecutive nodes of
// level `lc` (leaf level when cen != nullptr: the leaf boxes come from points).
__global__ void __launch_bounds__(256)
k_tree_levels(const float4* __restrict__ cen, int n, int lc, int levels,
              float4* __restrict__ bmin, float4* __restrict__ bmax) {
  __shared__ Box sb[256];
  const long long first = 1ll << lc;
  const long long cnt = first;  // nodes on level lc
  const long long li = (long long)blockIdx.x * 256 + threadIdx.x;
  const bool valid = li < cnt;
  Box b = box_empty();
  if (valid) {
    if (cen) {
      long long p0 = li * LEAF;
      for (int j = 0; j < LEAF; ++j) {
        long long p = p0 + j;
        if (p < n) {
          float4 c = cen[p];
          b.lx = fminf(b.lx, c.x);
          b.ly = fminf(b.ly, c.y);
          b.lz = fminf(b.lz, c.z);
          b.hx = fmaxf(b.hx, c.x);
          b.hy = fmaxf(b.hy, c.y);
          b.hz = fmaxf(b.hz, c.z);
        }
      }
      box_store(bmin, bmax, first + li, b);
    } else {
      float4 a = bmin[first + li], c = bmax[first + li];
      b = {a.x, a.y, a.z, c.x, c.y, c.z};
    }
  }
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int s = 1; s <= levels; ++s) {
    const int step = 1 << s;
    if (valid && (threadIdx.x & (step - 1)) == 0) {
      Box j = box_join(sb[threadIdx.x], sb[threadIdx.x + (step >> 1)]);
      sb[threadIdx.x] = j;
      box_store(bmin, bmax, (first + li) >> s, j);
    }
    __syncthreads();
  }
}

// ---- query -----------------------------------------------------------------
NG_DEV double dist2(double qx, double qy, double qz, float x, float y, float z) {
#pragma clang fp contract(off)
  double dx = qx - (double)x;
  double dy = qy - (double)y;
  double dz = qz - (double)z;
  return (dx * dx + dy * dy) + dz * dz;
}

NG_DEV double box_dist2(double qx, double qy, double qz, float4 lo, float4 hi) {
#pragma clang fp contract(off)
  double gx = fmax(fmax((double)lo.x - qx, qx - (double)hi.x), 0.0);
  double gy = fmax(fmax((double)lo.y - qy, qy - (double)hi.y), 0.0);
  double gz = fmax(fmax((double)lo.z - qz, qz - (double)hi.z), 0.0);
  return (gx * gx + gy * gy) + gz * gz;
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
    bool lt_next = less(dc, lc, d[K - 1], l[K - 1]);  // == true
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

template <int K>
__global__ void __launch_bounds__(256)
k_knn_query(const float4* __restrict__ cen, int n, int keff, int k_out, int nb, int nb2,
            const float4* __restrict__ bmin, const float4* __restrict__ bmax,
            const int* __restrict__ inv, int rows_logical, int* __restrict__ nbr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float4 cq = cen[p];
  const double qx = cq.x, qy = cq.y, qz = cq.z;
  const int ql = __float_as_int(cq.w);
  Best<K> best;
  best.init();

  const int myleaf = p / LEAF;
  const int lo_leaf = myleaf > 0 ? myleaf - 1 : 0;
  const int hi_leaf = myleaf + 1 < nb ? myleaf + 1 : nb - 1;
  {
    const int j1 = min((hi_leaf + 1) * LEAF, n);
    for (int j = lo_leaf * LEAF; j < j1; ++j) {
      if (j == p) continue;
      float4 c = cen[j];
      best.consider(dist2(qx, qy, qz, c.x, c.y, c.z), __float_as_int(c.w));
    }
  }

  unsigned node = 1;
  while (true) {
    bool descend = false;
    const float4 lo = bmin[node], hi = bmax[node];
    if (lo.x <= hi.x && box_dist2(qx, qy, qz, lo, hi) <= best.d[K - 1]) {
      if (node >= (unsigned)nb2) {
        const int leaf = (int)(node - (unsigned)nb2);
        if (leaf < lo_leaf || leaf > hi_leaf) {
          const int j0 = leaf * LEAF;
          const int j1 = min(j0 + LEAF, n);
          for (int j = j0; j < j1; ++j) {
            float4 c = cen[j];
            best.consider(dist2(qx, qy, qz, c.x, c.y, c.z), __float_as_int(c.w));
          }
        }
      } else {
        descend = true;
      }
    }
    if (descend) {
      node = 2 * node;
    } else {
      const unsigned t = __builtin_ctz(node + 1);
      const unsigned anc = node >> t;
      if (anc == 0) break;
      node = anc + 1;
    }
  }

  const long long row = rows_logical ? (long long)ql : (long long)p;
  int* out = nbr + row * k_out;
#pragma unroll
  for (int t = 0; t < K; ++t) {
    if (t < k_out) {
      int v = -1;
      if (t < keff) v = inv ? inv[best.l[t]] : best.l[t];
      out[t] = v;
    }
  }
  for (int t = K; t < k_out; ++t) out[t] = -1;
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

struct TreeShape {
  int nb, nb2, H;
};

TreeShape tree_shape(long long n) {
  TreeShape s;
  s.nb = (int)((n + LEAF - 1) / LEAF);
  if (s.nb < 1) s.nb = 1;
  s.H = 0;
  while ((1ll << s.H) < s.nb) ++s.H;
  s.nb2 = 1 << s.H;
  return s;
}

void build_tree(const float4* cen, int n, const TreeShape& ts, float4* bmin, float4* bmax,
                hipStream_t st) {
  int lc = ts.H;
  int levels = lc < 8 ? lc : 8;
  k_tree_levels<<<blocks_for(1ll << lc, 256), 256, 0, st>>>(cen, n, lc, levels, bmin, bmax);
  NG_LAUNCH_CHECK();
  lc -= levels;
  while (lc > 0) {
    levels = lc < 8 ? lc : 8;
    k_tree_levels<<<blocks_for(1ll << lc, 256), 256, 0, st>>>(nullptr, n, lc, levels, bmin, bmax);
    NG_LAUNCH_CHECK();
    lc -= levels;
  }
}

void query(const float4* cen, int n, int keff, int k_out, const TreeShape& ts, const float4* bmin,
           const float4* bmax, const int* inv, int rows_logical, int* nbr, hipStream_t st) {
  dim3 g(blocks_for(n, 256)), b(256);
  if (keff <= 8)
    k_knn_query<8><<<g, b, 0, st>>>(cen, n, keff, k_out, ts.nb, ts.nb2, bmin, bmax, inv,
                                    rows_logical, nbr);
  else if (keff <= 16)
    k_knn_query<16><<<g, b, 0, st>>>(cen, n, keff, k_out, ts.nb, ts.nb2, bmin, bmax, inv,
                                     rows_logical, nbr);
  else if (keff <= 24)
    k_knn_query<24><<<g, b, 0, st>>>(cen, n, keff, k_out, ts.nb, ts.nb2, bmin, bmax, inv,
                                     rows_logical, nbr);
  else
    k_knn_query<32><<<g, b, 0, st>>>(cen, n, keff, k_out, ts.nb, ts.nb2, bmin, bmax, inv,
                                     rows_logical, nbr);
  NG_LAUNCH_CHECK();
}

}  // namespace

size_t knn_tree_bytes(long long n) {
  TreeShape ts = tree_shape(n);
  Carver c(nullptr);
  c.take<float4>(2ll * ts.nb2);
  c.take<float4>(2ll * ts.nb2);
  c.take<int>(n);
  return c.bytes();
}

void launch_morton_keys(const float* pos_xyz3, const float4* cen4, int n, unsigned* keys,
                        void* temp, hipStream_t st) {
  unsigned* box = (unsigned*)temp;
  // mins start at the largest key, maxima at the smallest
  fill_i32((int*)box, -1, 3, st);
  fill_i32((int*)box + 3, 0, 3, st);
  unsigned b = blocks_for(n, 256);
  if (b > 1024) b = 1024;
  k_bbox<<<b, 256, 0, st>>>(pos_xyz3, cen4, n, box);
  NG_LAUNCH_CHECK();
  k_morton<<<blocks_for(n, 256), 256, 0, st>>>(pos_xyz3, cen4, n, box, keys);
  NG_LAUNCH_CHECK();
}

void knn_working_tree(const float4* cen, int n, void* tree_mem, hipStream_t st) {
  TreeShape ts = tree_shape(n);
  Carver c(tree_mem);
  float4* bmin = c.take<float4>(2ll * ts.nb2);
  float4* bmax = c.take<float4>(2ll * ts.nb2);
  int* inv = c.take<int>(n);
  build_tree(cen, n, ts, bmin, bmax, st);
  k_invert<<<blocks_for(n, 256), 256, 0, st>>>(cen, n, inv);
  NG_LAUNCH_CHECK();
}

void knn_working_query(const float4* cen, int n, int k, int keff, int* nbr, void* tree_mem,
                       hipStream_t st) {
  TreeShape ts = tree_shape(n);
  Carver c(tree_mem);
  float4* bmin = c.take<float4>(2ll * ts.nb2);
  float4* bmax = c.take<float4>(2ll * ts.nb2);
  int* inv = c.take<int>(n);
  query(cen, n, keff, k, ts, bmin, bmax, inv, 0, nbr, st);
}

// Plain entry: centres in caller order -> sorted copy -> tree -> rows by
// caller index.
size_t knn_plain_bytes(long long n) {
  Carver c(nullptr);
  c.take<unsigned>(64);
  c.take<unsigned>(n);
  c.take<int>(n);
  c.take<float4>(n);
  return c.bytes() + knn_tree_bytes(n) + sort_temp_bytes(n);
}

void knn_plain(const float* mu, int n, int k, int keff, int* nbr, void* ws, hipStream_t st) {
  Carver c(ws);
  unsigned* boxmem = c.take<unsigned>(64);
  unsigned* keys = c.take<unsigned>(n);
  int* perm = c.take<int>(n);
  float4* cen = c.take<float4>(n);
  char* rest = (char*)ws + c.bytes();
  void* tree_mem = rest;
  void* sort_mem = rest + knn_tree_bytes(n);
  launch_morton_keys(mu, nullptr, n, keys, boxmem, st);
  k_iota<<<blocks_for(n, 256), 256, 0, st>>>(perm, n);
  NG_LAUNCH_CHECK();
  sort_pairs_u32(keys, perm, n, 30, sort_mem, st);
  k_gather_cen<<<blocks_for(n, 256), 256, 0, st>>>(mu, perm, n, cen);
  NG_LAUNCH_CHECK();
  TreeShape ts = tree_shape(n);
  Carver t(tree_mem);
  float4* bmin = t.take<float4>(2ll * ts.nb2);
  float4* bmax = t.take<float4>(2ll * ts.nb2);
  build_tree(cen, n, ts, bmin, bmax, st);
  query(cen, n, keff, k, ts, bmin, bmax, nullptr, 1, nbr, st);
}

}  // namespace ng
