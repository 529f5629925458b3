// Greedy disjoint pairs (Sec. 3.4; Algorithm 1 GreedyDisjointPairs): the
// result of scanning the edges in increasing key order (cost, i, j), i < j in
// the logical order, taking an edge when both ends are free, and stopping at
// the budget P.
//
// Without the budget, the scan's result is the unique locally-dominant
// matching under that strict total order: repeatedly take every live edge
// that is the smallest at both of its ends, then drop edges touching a taken
// vertex.  On the edges of one vertex v, the order (cost, i, j) equals the
// order (cost, other endpoint), so each vertex's minimum is a single 64-bit
// atomicMin of (orderable cost bits << 32 | logical index of the other end).
// With a budget the scan keeps exactly the P smallest keys of that matching
// (later scan decisions never change earlier ones), found by radix select.
#include "internal.h"

namespace ng {
namespace {

constexpr unsigned long long KEY_MAX = ~0ull;

NG_DEV int logical(const int* lg, int p) { return lg ? lg[p] : p; }

// Appends `value` for every lane with `flag`, one atomic per wave; slots at
// or beyond `cap` are counted but not written.
NG_DEV void append_wave(bool flag, int value, int* list, int* count, int cap) {
  const unsigned long long m = __ballot(flag);
  if (m == 0) return;
  const int lane = lane_id();
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(m));
  base = __shfl(base, leader, 64);
  if (flag) {
    const unsigned long long below = lane == 0 ? 0ull : (m & (~0ull >> (64 - lane)));
    const int slot = base + __popcll(below);
    if (slot < cap) list[slot] = value;
  }
}

// Filter the previous live list (or all edges when in_list is null), keep the
// edges whose ends are both free, and post their keys to both ends.
__global__ void __launch_bounds__(256)
k_ld_min(const int* __restrict__ ea, const int* __restrict__ eb, const float* __restrict__ cost,
         const int* __restrict__ lg, int n, int m_all, const int* __restrict__ in_list,
         const int* __restrict__ in_count, const int* __restrict__ partner,
         unsigned long long* __restrict__ best, int* __restrict__ out_list,
         int* __restrict__ out_count) {
  const int cnt = in_list ? *in_count : m_all;
  const int nb = (cnt + 255) / 256;
  for (int blk = blockIdx.x; blk < nb; blk += gridDim.x) {
    const int i = blk * 256 + threadIdx.x;
    bool keep = false;
    int e = 0;
    if (i < cnt) {
      e = in_list ? in_list[i] : i;
      const int a = ea[e], b = eb[e];
      const float c = cost[e];
      keep = a >= 0 && a < n && b >= 0 && b < n && a != b && isfinite(c) && partner[a] < 0 &&
             partner[b] < 0;
      if (keep) {
        const unsigned long long hi = (unsigned long long)f2ord(c) << 32;
        atomicMin(&best[a], hi | (unsigned)logical(lg, b));
        atomicMin(&best[b], hi | (unsigned)logical(lg, a));
      }
    }
    append_wave(keep, e, out_list, out_count, m_all);
  }
}

// Take the edges that are the minimum at both ends; clear the next round's
// minima at the ends of every live edge.
__global__ void __launch_bounds__(256)
k_ld_match(const int* __restrict__ ea, const int* __restrict__ eb, const float* __restrict__ cost,
           const int* __restrict__ lg, const int* __restrict__ list, const int* __restrict__ count,
           const unsigned long long* __restrict__ best, unsigned long long* __restrict__ best_next,
           int* __restrict__ partner, int* __restrict__ matched, int* __restrict__ n_matched,
           int matched_cap) {
  const int cnt = *count;
  const int nb = (cnt + 255) / 256;
  for (int blk = blockIdx.x; blk < nb; blk += gridDim.x) {
    const int i = blk * 256 + threadIdx.x;
    bool take = false;
    int e = 0;
    if (i < cnt) {
      e = list[i];
      const int a = ea[e], b = eb[e];
      const unsigned long long hi = (unsigned long long)f2ord(cost[e]) << 32;
      take = best[a] == (hi | (unsigned)logical(lg, b)) &&
             best[b] == (hi | (unsigned)logical(lg, a));
      if (take) {
        partner[a] = b;
        partner[b] = a;
      }
      best_next[a] = KEY_MAX;
      best_next[b] = KEY_MAX;
    }
    append_wave(take, e, matched, n_matched, matched_cap);
  }
}

// Single-workgroup radix select of the P smallest matched edges under
// (orderable cost, min logical, max logical); keep[i] = 1 for those.
__global__ void __launch_bounds__(1024)
k_topp(const int* __restrict__ matched, int M, const int* __restrict__ ea,
       const int* __restrict__ eb, const float* __restrict__ cost, const int* __restrict__ lg,
       int P, unsigned char* __restrict__ keep) {
  __shared__ int hist[256];
  __shared__ unsigned s_prefix;
  __shared__ int s_need, s_tie_count;
  __shared__ unsigned long long s_prefix2;
  if (threadIdx.x == 0) {
    s_prefix = 0u;
    s_need = P;
  }
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    const unsigned hi_mask = pass == 0 ? 0u : (0xffffffffu << (shift + 8));
    for (int d = threadIdx.x; d < 256; d += blockDim.x) hist[d] = 0;
    __syncthreads();
    const unsigned pref = s_prefix;
    for (int i = threadIdx.x; i < M; i += blockDim.x) {
      const unsigned k = f2ord(cost[matched[i]]);
      if ((k & hi_mask) == (pref & hi_mask)) atomicAdd(&hist[(k >> shift) & 255u], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int cum = 0, need = s_need, d = 0;
      for (; d < 255; ++d) {
        if (cum + hist[d] >= need) break;
        cum += hist[d];
      }
      s_need = need - cum;
      s_prefix = pref | ((unsigned)d << shift);
      s_tie_count = hist[d];
    }
    __syncthreads();
  }
  const unsigned T = s_prefix;
  const bool all_ties = s_tie_count == s_need;
  if (threadIdx.x == 0) s_prefix2 = all_ties ? ~0ull : 0ull;
  __syncthreads();
  if (!all_ties) {
    for (int pass = 0; pass < 8; ++pass) {
      const int shift = 56 - 8 * pass;
      const unsigned long long hi_mask = pass == 0 ? 0ull : (~0ull << (shift + 8));
      for (int d = threadIdx.x; d < 256; d += blockDim.x) hist[d] = 0;
      __syncthreads();
      const unsigned long long pref = s_prefix2;
      for (int i = threadIdx.x; i < M; i += blockDim.x) {
        const int e = matched[i];
        if (f2ord(cost[e]) != T) continue;
        const unsigned la = (unsigned)logical(lg, ea[e]), lb = (unsigned)logical(lg, eb[e]);
        const unsigned long long k2 =
            ((unsigned long long)min(la, lb) << 32) | (unsigned long long)max(la, lb);
        if ((k2 & hi_mask) == (pref & hi_mask)) atomicAdd(&hist[(k2 >> shift) & 255ull], 1);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int cum = 0, need = s_need, d = 0;
        for (; d < 255; ++d) {
          if (cum + hist[d] >= need) break;
          cum += hist[d];
        }
        s_need = need - cum;
        s_prefix2 = pref | ((unsigned long long)d << shift);
      }
      __syncthreads();
    }
  }
  const unsigned long long T2 = s_prefix2;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const int e = matched[i];
    const unsigned k = f2ord(cost[e]);
    bool kp = k < T;
    if (k == T) {
      const unsigned la = (unsigned)logical(lg, ea[e]), lb = (unsigned)logical(lg, eb[e]);
      const unsigned long long k2 =
          ((unsigned long long)min(la, lb) << 32) | (unsigned long long)max(la, lb);
      kp = k2 <= T2;
    }
    keep[i] = kp ? 1 : 0;
  }
}

__global__ void k_unmatch(const int* __restrict__ matched, int M, const int* __restrict__ ea,
                          const int* __restrict__ eb, const unsigned char* __restrict__ keep,
                          int* __restrict__ partner) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M || keep[i]) return;
  const int e = matched[i];
  partner[ea[e]] = -1;
  partner[eb[e]] = -1;
}

__global__ void k_store_i64(const int* __restrict__ v, long long cap, long long* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    long long x = *v;
    *out = x < cap ? x : cap;
  }
}

unsigned grid_for(long long m) {
  unsigned b = blocks_for(m, 256);
  return b > 4096 ? 4096 : b;
}

}  // namespace

size_t select_temp_bytes(long long n, long long m) {
  Carver c(nullptr);
  c.take<unsigned long long>(n);
  c.take<unsigned long long>(n);
  c.take<int>(m);
  c.take<int>(m);
  c.take<int>(n / 2 + 1);
  c.take<unsigned char>(n / 2 + 1);
  c.take<int>(64);
  return c.bytes();
}

SelectResult select_pairs(const int* ea, const int* eb, const float* cost, long long m, int n,
                          const int* lg, long long max_pairs, int* partner, void* temp,
                          hipStream_t st, long long* d_npairs) {
  Carver c(temp);
  unsigned long long* best[2] = {c.take<unsigned long long>(n), c.take<unsigned long long>(n)};
  int* list[2] = {c.take<int>(m), c.take<int>(m)};
  int* matched = c.take<int>(n / 2 + 1);
  unsigned char* keep = c.take<unsigned char>(n / 2 + 1);
  int* counters = c.take<int>(64);  // [0..1]: live counts, [2]: matched count
  long long* host = pinned_host();

  fill_i32(partner, -1, n, st);
  fill_u64(best[0], KEY_MAX, n, st);
  fill_i32(counters, 0, 64, st);
  SelectResult r{0, 0};
  int cur = 0;
  long long live = m;
  for (int it = 0; live > 0; ++it) {
    int* cnt_out = counters + (it & 1);
    fill_i32(cnt_out, 0, 1, st);
    k_ld_min<<<grid_for(live), 256, 0, st>>>(ea, eb, cost, lg, n, (int)m,
                                             it == 0 ? nullptr : list[cur ^ 1],
                                             counters + ((it & 1) ^ 1), partner, best[it & 1],
                                             list[cur], cnt_out);
    NG_LAUNCH_CHECK();
    NG_HIP(hipMemcpyAsync(host, cnt_out, sizeof(int), hipMemcpyDeviceToHost, st));
    NG_HIP(hipStreamSynchronize(st));
    live = *(int*)host;
    if (live == 0) break;
    k_ld_match<<<grid_for(live), 256, 0, st>>>(ea, eb, cost, lg, list[cur], cnt_out, best[it & 1],
                                               best[(it & 1) ^ 1], partner, matched,
                                               counters + 2, n / 2 + 1);
    NG_LAUNCH_CHECK();
    cur ^= 1;
    r.iters = it + 1;
  }
  NG_HIP(hipMemcpyAsync(host, counters + 2, sizeof(int), hipMemcpyDeviceToHost, st));
  NG_HIP(hipStreamSynchronize(st));
  long long M = *(int*)host;
  // duplicate edges in a caller's list can over-count; a matching has at
  // most n/2 edges
  if (M > n / 2 + 1) M = n / 2 + 1;
  if (M > max_pairs) {
    k_topp<<<1, 1024, 0, st>>>(matched, (int)M, ea, eb, cost, lg, (int)max_pairs, keep);
    NG_LAUNCH_CHECK();
    k_unmatch<<<blocks_for(M, 256), 256, 0, st>>>(matched, (int)M, ea, eb, keep, partner);
    NG_LAUNCH_CHECK();
    M = max_pairs;
  }
  if (d_npairs) {
    k_store_i64<<<1, 64, 0, st>>>(counters + 2, max_pairs, d_npairs);
    NG_LAUNCH_CHECK();
  }
  r.pairs = M;
  return r;
}

}  // namespace ng
