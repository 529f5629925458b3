// Undirected union of the directed kNN lists (Algorithm 1,
// UndirectedUnionEdges): row i emits its neighbour j unless j also lists i
// and j comes first in the logical order, so every unordered pair appears
// exactly once.  Count per row, exclusive scan, emit: the output order is
// deterministic (by row, then slot).
#include "internal.h"

namespace ng {
namespace {

NG_DEV int logical(const int* lg, int p) { return lg ? lg[p] : p; }

__global__ void k_edge_flags(const int* __restrict__ nbr, const int* __restrict__ lg, int n, int k,
                             unsigned char* __restrict__ flag, int* __restrict__ cnt) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int* row = nbr + (long long)p * k;
  const int lp = logical(lg, p);
  int c = 0;
  for (int t = 0; t < k; ++t) {
    const int j = row[t];
    bool emit = false;
    if (j >= 0 && j < n && j != p) {
      if (lp < logical(lg, j)) {
        emit = true;
      } else {
        const int* rj = nbr + (long long)j * k;
        bool mutual = false;
        for (int u = 0; u < k; ++u) mutual |= (rj[u] == p);
        emit = !mutual;
      }
    }
    flag[(long long)p * k + t] = emit ? 1 : 0;
    c += emit ? 1 : 0;
  }
  cnt[p] = c;
}

__global__ void k_edge_emit(const int* __restrict__ nbr, const int* __restrict__ lg, int n, int k,
                            const unsigned char* __restrict__ flag, const int* __restrict__ off,
                            int* __restrict__ ea, int* __restrict__ eb) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int* row = nbr + (long long)p * k;
  const int lp = logical(lg, p);
  int o = off[p];
  for (int t = 0; t < k; ++t) {
    if (flag[(long long)p * k + t]) {
      const int j = row[t];
      const bool first = lp < logical(lg, j);
      ea[o] = first ? p : j;
      eb[o] = first ? j : p;
      ++o;
    }
  }
}

__global__ void k_to_i64(const int* __restrict__ v, long long* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = (long long)*v;
}

}  // namespace

size_t edges_temp_bytes(long long n, int k) {
  Carver c(nullptr);
  c.take<unsigned char>(n * k);
  c.take<int>(n);
  c.take<int>(n);
  c.take<int>(4);
  return c.bytes() + scan_temp_bytes(n);
}

void launch_union_edges(const int* nbr, const int* lg, int n, int k, int* ea, int* eb,
                        long long* d_m, void* temp, hipStream_t st) {
  Carver c(temp);
  unsigned char* flag = c.take<unsigned char>((long long)n * k);
  int* cnt = c.take<int>(n);
  int* off = c.take<int>(n);
  int* tot = c.take<int>(4);
  void* stemp = (char*)temp + c.bytes();
  k_edge_flags<<<blocks_for(n, 256), 256, 0, st>>>(nbr, lg, n, k, flag, cnt);
  NG_LAUNCH_CHECK();
  scan_exclusive_i32(cnt, off, n, tot, stemp, st);
  k_edge_emit<<<blocks_for(n, 256), 256, 0, st>>>(nbr, lg, n, k, flag, off, ea, eb);
  NG_LAUNCH_CHECK();
  k_to_i64<<<1, 64, 0, st>>>(tot, d_m);
  NG_LAUNCH_CHECK();
}

}  // namespace ng
