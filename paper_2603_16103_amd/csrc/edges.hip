// Undirected union of the directed kNN lists (Algorithm 1,
// UndirectedUnionEdges): row p emits its neighbour j unless j also lists p
// and j comes first in the logical order, so every unordered pair appears
// exactly once.  Edges are numbered in emission order (by row, then slot);
// edge e is stored as (src[e] = emitting row, tgt[e] = the neighbour).
//
// The same pass builds the incidence structure the pair selection reads:
//   eoff[p]  first edge emitted by row p (eoff[n] = m): row p's own edges
//            are the contiguous range [eoff[p], eoff[p+1]);
//   ioff[p]  start of p's incoming edges in a second numbering (ioff[n] = m);
//   islot[e] rank of edge e among the edges whose tgt is tgt[e].
// With aoff[p] = eoff[p] + ioff[p], every splat p owns the adjacency range
// [aoff[p], aoff[p+1]) holding first its emitted edges, then its incoming
// ones: each edge has exactly one entry at each of its two ends.
#include "internal.h"

namespace ng {
namespace {

NG_DEV int logical(const int* lg, int p) { return lg ? lg[p] : p; }

// thread per directed slot (p, t): 1 if the slot emits an edge.  When k
// divides 64 a row's slots are k consecutive lanes of one wave (the grid is a
// multiple of 64), and with cnt given the row's first lane also writes its
// emitted count and zeroes its incoming counter (what k_edge_count does
// otherwise).
__global__ void __launch_bounds__(256)
k_edge_flags(const int* __restrict__ nbr, const int* __restrict__ lg, int n, int k, int vec4,
             unsigned char* __restrict__ flag, int* __restrict__ cnt, int* __restrict__ ideg) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cnt && s == 0) {
    cnt[n] = 0;  // so the scan's entry n is the total
    if (ideg) ideg[n] = 0;
  }
  if (s >= (long long)n * k) return;
  const int p = (int)(s / k);
  const int j = nbr[s];
  bool emit = false;
  if (j >= 0 && j < n && j != p) {
    if (logical(lg, p) < logical(lg, j)) {
      emit = true;
    } else {
      const int* rj = nbr + (long long)j * k;
      bool mutual = false;
      if (vec4) {
        const int4* r4 = (const int4*)rj;
        for (int u = 0; u < (k >> 2); ++u) {
          const int4 v = r4[u];
          mutual |= (v.x == p) | (v.y == p) | (v.z == p) | (v.w == p);
        }
      } else {
        for (int u = 0; u < k; ++u) mutual |= (rj[u] == p);
      }
      emit = !mutual;
    }
  }
  flag[s] = emit ? 1 : 0;
  if (cnt) {  // (64 % k == 0 here)
    const unsigned long long m = __ballot(emit);
    const int t = (int)(s - (long long)p * k);
    if (t == 0) {
      const int first = lane_id();
      const unsigned long long row = k == 64 ? ~0ull : (((1ull << k) - 1ull) << first);
      cnt[p] = __popcll(m & row);
      if (ideg) ideg[p] = 0;
    }
  }
}

// thread per row: emitted count (the row's flags are contiguous bytes)
__global__ void __launch_bounds__(256)
k_edge_count(const unsigned char* __restrict__ flag, int n, int k, int* __restrict__ cnt,
             int* __restrict__ ideg) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > n) return;
  if (ideg) ideg[p] = 0;  // the incoming counters of the emit pass
  int c = 0;
  if (p < n) {
    const unsigned char* f = flag + (long long)p * k;
    for (int t = 0; t < k; ++t) c += f[t];
  }
  cnt[p] = c;  // cnt[n] = 0, so the scan's entry n is the total
}

// thread per directed slot: an emitting slot writes its edge at eoff[p] +
// (emitting slots before it in row p); its rank among the edges into its
// target comes from an atomic counter per target (each slot's atomic is
// independent of the others, so none waits for another's result)
__global__ void __launch_bounds__(256)
k_edge_emit(const int* __restrict__ nbr, int n, int k, const unsigned char* __restrict__ flag,
            const int* __restrict__ eoff, int* __restrict__ src, int* __restrict__ tgt,
            int* __restrict__ indeg, int* __restrict__ islot) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = s < (long long)n * k;
  const bool emit = in && flag[s];
  int rank = 0;  // emitting slots before this one in its row
  if (64 % k == 0) {
    // a row's slots are k consecutive lanes of one wave (the grid is a
    // multiple of 64 and k divides 64): the rank is a ballot
    const unsigned long long m = __ballot(emit);
    const int lane = lane_id();
    const int first = lane - (int)(s % k);  // lane of the row's first slot
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const unsigned long long row = first == 0 ? ~0ull : ~(~0ull >> (64 - first));
    rank = __popcll(m & below & row);
  }
  if (!emit) return;
  const int p = (int)(s / k);
  const int t = (int)(s - (long long)p * k);
  if (64 % k != 0) {
    const unsigned char* f = flag + (long long)p * k;
    for (int u = 0; u < t; ++u) rank += f[u];
  }
  const int o = eoff[p] + rank;
  const int j = nbr[s];
  src[o] = p;
  tgt[o] = j;
  if (islot) islot[o] = atomicAdd(&indeg[j], 1);
}

__global__ void k_to_i64(const int* __restrict__ v, long long* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = (long long)*v;
}

// (src, tgt) -> (smaller, larger) in the caller's numbering
__global__ void k_edge_minmax(const int* __restrict__ src, const int* __restrict__ tgt,
                              const int* __restrict__ d_m, int* __restrict__ ei,
                              int* __restrict__ ej) {
  const int m = *d_m;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
    const int a = src[e], b = tgt[e];
    ei[e] = a < b ? a : b;
    ej[e] = a < b ? b : a;
  }
}

// Sort keys of the lexicographic order: pass 0 keys each edge position by
// its larger end, pass 1 (after a stable sort by that) by its smaller end;
// positions at and past the count get `pad`, above every index.
__global__ void k_lex_keys(const int* __restrict__ lo, const int* __restrict__ hi,
                           const int* __restrict__ d_m, long long cap, unsigned pad, int pass,
                           unsigned* __restrict__ key, int* __restrict__ val) {
  const int m = *d_m;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < cap;
       p += (long long)gridDim.x * blockDim.x) {
    if (pass == 0) {
      val[p] = (int)p;
      key[p] = p < m ? (unsigned)hi[p] : pad;
    } else {
      const int e = val[p];
      key[p] = e < m ? (unsigned)lo[e] : pad;
    }
  }
}

__global__ void k_lex_gather(const int* __restrict__ lo, const int* __restrict__ hi,
                             const int* __restrict__ d_m, const int* __restrict__ order,
                             int* __restrict__ ei, int* __restrict__ ej) {
  const int m = *d_m;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
    const int e = order[p];
    ei[p] = lo[e];
    ej[p] = hi[e];
  }
}

__global__ void k_add_offsets(const int* __restrict__ a, const int* __restrict__ b, int n1,
                              int* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n1) out[p] = a[p] + b[p];
}

}  // namespace

size_t edges_temp_bytes(long long n, int k) {
  Carver c(nullptr);
  c.take<unsigned char>(n * k);
  c.take<int>(n + 1);
  c.take<int>(n + 1);
  c.take<int>(4);
  return c.bytes() + scan_temp_bytes(n + 1);
}

size_t edges_public_bytes(long long n, int k) {
  Carver c(nullptr);
  c.take<int>(n * k);
  c.take<int>(n * k);
  c.take<int>(n + 1);
  c.take<int>(n * k);       // smaller ends
  c.take<int>(n * k);       // larger ends
  c.take<unsigned>(n * k);  // sort keys
  c.take<int>(n * k);       // sort values
  return c.bytes() + std::max(edges_temp_bytes(n, k), sort_temp_bytes(n * k));
}

void launch_union_edges(const int* nbr, const int* lg, int n, int k, EdgeSet es, long long* d_m,
                        void* temp, hipStream_t st) {
  Carver c(temp);
  unsigned char* flag = c.take<unsigned char>((long long)n * k);
  int* cnt = c.take<int>(n + 1);
  int* tot = c.take<int>(4);
  int* ideg = c.take<int>(n + 1);
  void* stemp = (char*)temp + c.bytes();
  const long long slots = (long long)n * k;
  // rows read as int4 when every row start is 16-byte aligned
  const int vec4 = (k % 4 == 0) && ((uintptr_t)nbr % 16 == 0);
  const bool fused = k > 0 && 64 % k == 0;  // the flags kernel counts the rows
  k_edge_flags<<<blocks_for(slots, 256), 256, 0, st>>>(nbr, lg, n, k, vec4, flag,
                                                       fused ? cnt : nullptr,
                                                       es.ioff ? ideg : nullptr);
  NG_LAUNCH_CHECK();
  if (!fused) {
    k_edge_count<<<blocks_for(n + 1, 256), 256, 0, st>>>(flag, n, k, cnt,
                                                         es.ioff ? ideg : nullptr);
    NG_LAUNCH_CHECK();
  }
  scan_exclusive_i32(cnt, es.eoff, n + 1, tot, stemp, st);
  k_edge_emit<<<blocks_for(slots, 256), 256, 0, st>>>(nbr, n, k, flag, es.eoff, es.src, es.tgt,
                                                  ideg, es.ioff ? es.islot : nullptr);
  NG_LAUNCH_CHECK();
  if (es.ioff) {
    scan_exclusive_i32(ideg, es.ioff, n + 1, nullptr, stemp, st);
    k_add_offsets<<<blocks_for(n + 1, 256), 256, 0, st>>>(es.eoff, es.ioff, n + 1, es.aoff);
    NG_LAUNCH_CHECK();
  }
  if (d_m) {
    k_to_i64<<<1, 64, 0, st>>>(tot, d_m);
    NG_LAUNCH_CHECK();
  }
}

void union_edges_public(const int* nbr, int n, int k, int* ei, int* ej, long long* d_m,
                        void* ws, hipStream_t st) {
  const long long cap = (long long)n * k;
  Carver c(ws);
  EdgeSet es{};
  es.src = c.take<int>(cap);
  es.tgt = c.take<int>(cap);
  es.eoff = c.take<int>(n + 1);
  int* lo = c.take<int>(cap);
  int* hi = c.take<int>(cap);
  unsigned* key = c.take<unsigned>(cap);
  int* val = c.take<int>(cap);
  void* temp = (char*)ws + c.bytes();
  launch_union_edges(nbr, nullptr, n, k, es, d_m, temp, st);
  // the total sits at eoff[n]
  const int* tot = es.eoff + n;
  unsigned b = blocks_for(cap, 256);
  if (b > 4096) b = 4096;
  k_edge_minmax<<<b, 256, 0, st>>>(es.src, es.tgt, tot, lo, hi);
  NG_LAUNCH_CHECK();
  // lexicographic (smaller, larger) order by two stable sorts over the
  // capacity (no host read of the count)
  int bits = 1;
  while ((1ll << bits) <= (long long)n) ++bits;
  for (int pass = 0; pass < 2; ++pass) {
    k_lex_keys<<<b, 256, 0, st>>>(lo, hi, tot, cap, (unsigned)n, pass, key, val);
    NG_LAUNCH_CHECK();
    sort_pairs_u32(key, val, cap, bits, temp, st);
  }
  k_lex_gather<<<b, 256, 0, st>>>(lo, hi, tot, val, ei, ej);
  NG_LAUNCH_CHECK();
}

}  // namespace ng
