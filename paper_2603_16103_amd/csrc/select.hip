// Greedy disjoint pairs (Sec. 3.4; Algorithm 1 GreedyDisjointPairs): the
// result of scanning the edges in increasing key order (cost, i, j), i < j in
// the logical order, taking an edge when both ends are free, and stopping at
// the budget P.
//
// Without the budget, the scan's result is the unique locally-dominant
// matching under that strict total order: repeatedly take every live edge
// that is the smallest at both of its ends, then drop the taken vertices.
// On the edges of one vertex v the order (cost, i, j) equals the order
// (cost, logical index of the other end), so each adjacency entry carries the
// 64-bit key (orderable cost bits << 32 | logical index of the other end).
//
// Vertex-centric iterations over the incidence ranges (no atomics on keys):
//   pick : every active vertex takes the smallest key among its entries whose
//          other end is still free (pick[v] = that end, or -1 if none);
//   match: v with pick[pick[v]] == v is matched to it (each end writes only
//          its own partner entry); vertices with pick = -1 can never match and
//          leave; the rest form the next active list.
// A vertex picked by an active v is itself active (v is one of its free
// ends), so pick[] is never read stale.  With a budget the scan keeps exactly
// the P smallest keys of that matching (later scan decisions never change
// earlier ones), found by radix select over (cost, i, j).
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace ng {
namespace {

constexpr unsigned long long KEY_MAX = ~0ull;

NG_DEV int logical(const int* lg, int p) { return lg ? lg[p] : p; }

// ---- generic incidence from an arbitrary edge list (stage entry point) ----
NG_DEV bool edge_ok(int a, int b, int n) { return a >= 0 && a < n && b >= 0 && b < n && a != b; }

__global__ void k_deg_count(const int* __restrict__ ea, const int* __restrict__ eb, int m, int n,
                            int* __restrict__ deg, const int* __restrict__ d_mcount) {
  if (d_mcount) m = min(m, *d_mcount);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
    const int a = ea[e], b = eb[e];
    if (!edge_ok(a, b, n)) continue;
    atomicAdd(&deg[a], 1);
    atomicAdd(&deg[b], 1);
  }
}

NG_DEV unsigned long long entry_key(float c, int other_logical) {
  if (!isfinite(c)) return KEY_MAX;
  return ((unsigned long long)f2ord(c) << 32) | (unsigned)other_logical;
}

__global__ void k_adj_fill(const int* __restrict__ ea, const int* __restrict__ eb,
                           const float* __restrict__ cost, int m, int n,
                           const int* __restrict__ aoff, int* __restrict__ cursor,
                           unsigned long long* __restrict__ akey, int* __restrict__ au,
                           const int* __restrict__ d_mcount) {
  if (d_mcount) m = min(m, *d_mcount);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
    const int a = ea[e], b = eb[e];
    if (!edge_ok(a, b, n)) continue;
    const float c = cost[e];
    const int sa = aoff[a] + atomicAdd(&cursor[a], 1);
    const int sb = aoff[b] + atomicAdd(&cursor[b], 1);
    akey[sa] = entry_key(c, b);
    au[sa] = b;
    akey[sb] = entry_key(c, a);
    au[sb] = a;
  }
}

// ---- matching iterations ----------------------------------------------------
// act == nullptr: every vertex [0, n) is active, and (first iteration) every
// vertex is free.
//
// pick: each active vertex takes its smallest entry whose other end is free.
// Other ends only ever go from free to matched, so a vertex keeps its kTop
// smallest entries (sorted) from its last full scan: the first of them whose
// other end is still free is the smallest free entry of all, since every
// entry outside the cache has a larger key.  Only a vertex whose cached ends
// are all matched scans its whole range again (and refills the cache with
// the smallest entries whose other end is free, the only ones that can
// matter later).
constexpr int kTop = 2;  // (2, 4, 6 and 8 measured: 2 is fastest)

struct PickState {
  unsigned long long* tkey;  // [n][kTop] cached smallest keys, ascending
  int* tu;                   // [n][kTop] their other ends
  int* tn;                   // [n] cached entries (0: none cached yet)
};

// One vertex's pick; returns the other end (-1: no free entry) and the key.
NG_DEV int pick_vertex(int v, bool all_free, const int* __restrict__ aoff,
                       const unsigned long long* __restrict__ akey, const int* __restrict__ au,
                       const int* __restrict__ partner, const PickState& ps,
                       unsigned long long& bkey) {
  if (!all_free) {
    const int tn = ps.tn[v];
#pragma unroll
    for (int q = 0; q < kTop; ++q) {
      if (q < tn) {
        const int u = ps.tu[(long long)v * kTop + q];
        if (partner[u] < 0) {
          bkey = ps.tkey[(long long)v * kTop + q];
          return u;
        }
      }
    }
  }
  // full scan: the kTop smallest entries with a free other end, sorted
  unsigned long long k[kTop];
  int uu[kTop];
#pragma unroll
  for (int q = 0; q < kTop; ++q) {
    k[q] = KEY_MAX;
    uu[q] = -1;
  }
  auto consider = [&](unsigned long long key, int u) {
    if (!(key < k[kTop - 1])) return;
    // sorted insertion (registers, fully unrolled)
    bool lt_next = true;
#pragma unroll
    for (int q = kTop - 1; q > 0; --q) {
      const bool lt_prev = key < k[q - 1];
      const unsigned long long nk = lt_prev ? k[q - 1] : (lt_next ? key : k[q]);
      const int nu = lt_prev ? uu[q - 1] : (lt_next ? u : uu[q]);
      k[q] = nk;
      uu[q] = nu;
      lt_next = lt_prev;
    }
    if (lt_next) {
      k[0] = key;
      uu[0] = u;
    }
  };
  int t = aoff[v];
  const int t1 = aoff[v + 1];
  for (; t + 4 <= t1; t += 4) {
    unsigned long long kk[4];
    int u[4];
    bool f[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      kk[q] = akey[t + q];
      u[q] = au[t + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) f[q] = all_free || partner[u[q]] < 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (f[q] && kk[q] != KEY_MAX) consider(kk[q], u[q]);
  }
  for (; t < t1; ++t) {
    const unsigned long long key = akey[t];
    const int u = au[t];
    if (key != KEY_MAX && (all_free || partner[u] < 0)) consider(key, u);
  }
  int n_ok = 0;
#pragma unroll
  for (int q = 0; q < kTop; ++q) {
    ps.tkey[(long long)v * kTop + q] = k[q];
    ps.tu[(long long)v * kTop + q] = uu[q];
    n_ok += uu[q] >= 0 ? 1 : 0;
  }
  ps.tn[v] = n_ok;
  bkey = k[0];
  return uu[0];
}

__global__ void __launch_bounds__(256)
k_ld_pick(const int* __restrict__ aoff, const unsigned long long* __restrict__ akey,
          const int* __restrict__ au, const int* __restrict__ partner,
          const int* __restrict__ act, const int* __restrict__ act_count, int n,
          int* __restrict__ pick, unsigned* __restrict__ pcost, int* __restrict__ next_count,
          PickState ps) {
  const int cnt = act ? *act_count : n;
  if (blockIdx.x == 0 && threadIdx.x == 0) *next_count = 0;
  const bool all_free = act == nullptr;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    const int v = act ? act[i] : i;
    unsigned long long best = KEY_MAX;
    pick[v] = pick_vertex(v, all_free, aoff, akey, au, partner, ps, best);
    pcost[v] = (unsigned)(best >> 32);
  }
}

// The first pick of a matching (every end free): kPickLanes lanes per
// vertex.  Lane r loads the vertex's entries r, r + kPickLanes, ... (the
// group's loads are contiguous and issue together) and keeps its kTop
// smallest; kTop rounds of a minimum over the group then give the vertex's
// kTop smallest entries in order (the keys of one vertex are distinct: they
// end in the other end's logical index), the same cache and pick as a full
// scan by one lane.
constexpr int kPickLanes = 4;  // (4 and 8 measured)

__global__ void __launch_bounds__(256)
k_ld_pick_first(const int* __restrict__ aoff, const unsigned long long* __restrict__ akey,
                const int* __restrict__ au, int n, int* __restrict__ pick,
                unsigned* __restrict__ pcost, int* __restrict__ counters, int* __restrict__ partner,
                PickState ps) {
  constexpr int L = kPickLanes;
  // (the matching's counters and partner entries start here: no fills)
  if (blockIdx.x == 0 && threadIdx.x < 64) counters[threadIdx.x] = 0;
  const int lane = lane_id();
  const int r = lane & (L - 1), gb = lane & ~(L - 1);
  const long long stride = (long long)gridDim.x * blockDim.x / L;
  for (long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / L; i < n; i += stride) {
    const int v = (int)i;
    if (r == 0) partner[v] = -1;
    const int t0 = aoff[v], t1 = aoff[v + 1];
    unsigned long long k[kTop];
    int uu[kTop];
#pragma unroll
    for (int q = 0; q < kTop; ++q) {
      k[q] = KEY_MAX;
      uu[q] = -1;
    }
    auto consider = [&](unsigned long long key, int u) {
      if (!(key < k[kTop - 1])) return;
      bool lt_next = true;
#pragma unroll
      for (int q = kTop - 1; q > 0; --q) {
        const bool lt_prev = key < k[q - 1];
        const unsigned long long nk = lt_prev ? k[q - 1] : (lt_next ? key : k[q]);
        const int nu = lt_prev ? uu[q - 1] : (lt_next ? u : uu[q]);
        k[q] = nk;
        uu[q] = nu;
        lt_next = lt_prev;
      }
      if (lt_next) {
        k[0] = key;
        uu[0] = u;
      }
    };
    int t = t0 + r;
    for (; t + 2 * L < t1; t += 3 * L) {
      const unsigned long long a0 = akey[t], a1 = akey[t + L], a2 = akey[t + 2 * L];
      const int u0 = au[t], u1 = au[t + L], u2 = au[t + 2 * L];
      consider(a0, u0);
      consider(a1, u1);
      consider(a2, u2);
    }
    for (; t < t1; t += L) consider(akey[t], au[t]);
    // the group's kTop smallest, one per round (KEY_MAX: none left)
    int head = 0;
    unsigned long long gk[kTop];
    int gu[kTop];
#pragma unroll
    for (int q = 0; q < kTop; ++q) {
      unsigned long long mine = KEY_MAX;
      int mu = -1;
#pragma unroll
      for (int h = 0; h < kTop; ++h)
        if (h == head) {
          mine = k[h];
          mu = uu[h];
        }
      unsigned long long m = mine;
#pragma unroll
      for (int d = 1; d < L; d <<= 1) {
        const unsigned lo = __shfl_xor((unsigned)m, d, 64);
        const unsigned hi = __shfl_xor((unsigned)(m >> 32), d, 64);
        const unsigned long long o = ((unsigned long long)hi << 32) | lo;
        m = o < m ? o : m;
      }
      const unsigned long long own = (__ballot(mine == m && m != KEY_MAX) >> gb) & ((1ull << L) - 1);
      const int owner = own ? gb + __ffsll((long long)own) - 1 : gb;
      const int u = __shfl(mu, owner, 64);
      gk[q] = m;
      gu[q] = m != KEY_MAX ? u : -1;
      if (own && lane == owner) ++head;
    }
    if (r == 0) {
      int n_ok = 0;
#pragma unroll
      for (int q = 0; q < kTop; ++q) {
        ps.tkey[(long long)v * kTop + q] = gk[q];
        ps.tu[(long long)v * kTop + q] = gu[q];
        n_ok += gu[q] >= 0 ? 1 : 0;
      }
      ps.tn[v] = n_ok;
      pick[v] = gu[0];
      pcost[v] = (unsigned)(gk[0] >> 32);
    }
  }
}

// Block-wide append: every thread with `flag` gets a distinct slot of
// `list`, with one atomic on *count per block.  Every thread of the block
// must call it (it synchronises the block).
template <int NW>
NG_DEV int block_append(bool flag, int* s_cnt, int* count) {
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  if (lane == 0) s_cnt[w] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int q = 0; q < NW; ++q) {
      const int c = s_cnt[q];
      s_cnt[q] = tot;
      tot += c;
    }
    s_cnt[NW] = tot ? atomicAdd(count, tot) : 0;
  }
  __syncthreads();
  const unsigned long long below = lane == 0 ? 0ull : (m & (~0ull >> (64 - lane)));
  const int slot = s_cnt[NW] + s_cnt[w] + __popcll(below);
  __syncthreads();  // s_cnt is reused by the next call
  return slot;
}

// match step for active entry i (cnt entries): mutual picks are matched (each
// end writes only its own partner slot, the lower logical end records the
// pair); vertices whose pick was not returned stay active.
template <int NW>
NG_DEV void match_entry(int i, int cnt, const int* __restrict__ act, const int* __restrict__ pick,
                        const unsigned* __restrict__ pcost, const int* __restrict__ lg,
                        int* __restrict__ partner, int* __restrict__ next_act,
                        int* __restrict__ next_count, int* __restrict__ pair_a,
                        int* __restrict__ pair_b, unsigned* __restrict__ pair_c,
                        int* __restrict__ npairs, int* s_cnt) {
  bool keep = false, rec = false;
  int v = 0, u = -1;
  if (i < cnt) {
    v = act ? act[i] : i;
    u = pick[v];
    if (u >= 0) {
      if (pick[u] == v) {
        partner[v] = u;
        rec = logical(lg, v) < logical(lg, u);
      } else {
        keep = true;
      }
    }
  }
  const int ks = block_append<NW>(keep, s_cnt, next_count);
  if (keep) next_act[ks] = v;
  const int ps = block_append<NW>(rec, s_cnt, npairs);
  if (rec) {
    pair_a[ps] = v;
    pair_b[ps] = u;
    pair_c[ps] = pcost[v];
  }
}

// Appends use one atomic per block and list.
constexpr int kMatchBlock = 1024;
__global__ void __launch_bounds__(kMatchBlock)
k_ld_match(const int* __restrict__ act, const int* __restrict__ act_count, int n,
           const int* __restrict__ pick, const unsigned* __restrict__ pcost,
           const int* __restrict__ lg, int* __restrict__ partner, int* __restrict__ next_act,
           int* __restrict__ next_count, int* __restrict__ pair_a, int* __restrict__ pair_b,
           unsigned* __restrict__ pair_c, int* __restrict__ npairs) {
  constexpr int NW = kMatchBlock / 64;
  __shared__ int s_cnt[NW + 1];
  const int cnt = act ? *act_count : n;
  // whole blocks stay in the loop for the block-wide appends
  const int span = (cnt + kMatchBlock - 1) / kMatchBlock * kMatchBlock;
  for (int i0 = blockIdx.x * kMatchBlock; i0 < span; i0 += gridDim.x * kMatchBlock)
    match_entry<NW>(i0 + (int)threadIdx.x, cnt, act, pick, pcost, lg, partner, next_act,
                    next_count, pair_a, pair_b, pair_c, npairs, s_cnt);
}

// The remaining iterations in one workgroup: pick and match alternate over
// the active list (lists swap between A and B) until it is empty, with no
// launch or host round trip per iteration.  cnt[0] / cnt[1]: the counts of
// lists A / B; the list the last grid-wide match wrote is `in_sel`.
// iters (device) receives the number of iterations run here.  Every
// iteration retires at least one active vertex (the smallest live edge is
// both its ends' pick; a vertex with no free neighbour leaves), so more than
// (first count + 1) iterations mean a broken adjacency: the loop stops there
// and iters receives minus the count, which the callers report as an error.
__global__ void __launch_bounds__(kMatchBlock)
k_ld_tail(const int* __restrict__ aoff, const unsigned long long* __restrict__ akey,
          const int* __restrict__ au, int* __restrict__ partner, int* __restrict__ listA,
          int* __restrict__ listB, int* __restrict__ cnt, int in_sel, int* __restrict__ pick,
          unsigned* __restrict__ pcost, const int* __restrict__ lg, int* __restrict__ pair_a,
          int* __restrict__ pair_b, unsigned* __restrict__ pair_c, int* __restrict__ npairs,
          PickState ps, int* __restrict__ iters) {
  constexpr int NW = kMatchBlock / 64;
  __shared__ int s_cnt[NW + 1];
  __shared__ int s_n;
  int sel = in_sel;
  int it = 0;
  int limit = 0;
  bool broken = false;
  while (true) {
    int* in = sel == 0 ? listA : listB;
    int* out = sel == 0 ? listB : listA;
    int* in_cnt = cnt + sel;
    int* out_cnt = cnt + (sel ^ 1);
    if (threadIdx.x == 0) s_n = *in_cnt;
    __syncthreads();
    const int c = s_n;
    if (c == 0) break;
    if (it == 0) limit = c + 1;
    if (it > limit) {
      broken = true;
      break;
    }
    for (int i = threadIdx.x; i < c; i += kMatchBlock) {
      const int v = in[i];
      unsigned long long best = KEY_MAX;
      pick[v] = pick_vertex(v, false, aoff, akey, au, partner, ps, best);
      pcost[v] = (unsigned)(best >> 32);
    }
    if (threadIdx.x == 0) *out_cnt = 0;
    __threadfence_block();
    __syncthreads();
    const int span = (c + kMatchBlock - 1) / kMatchBlock * kMatchBlock;
    for (int i0 = 0; i0 < span; i0 += kMatchBlock)
      match_entry<NW>(i0 + (int)threadIdx.x, c, in, pick, pcost, lg, partner, out, out_cnt,
                      pair_a, pair_b, pair_c, npairs, s_cnt);
    __threadfence_block();
    __syncthreads();
    sel ^= 1;
    ++it;
  }
  if (threadIdx.x == 0) *iters = broken ? -it : it;
}

// ---- budget: keep the P smallest (cost, i, j) of each segment's matching --
// Adds the lanes' valid bins to an LDS histogram.  Matched costs crowd a few
// bins, and lanes of one instruction adding to one address serialise, so the
// bin of the first valid lane (twice) is added once for all its lanes.
NG_DEV void hist_add(int* hist, unsigned bin, bool valid) {
#pragma unroll
  for (int round = 0; round < 2; ++round) {
    const unsigned long long m = __ballot(valid);
    if (!m) return;
    const int leader = __ffsll((long long)m) - 1;
    const unsigned bl = (unsigned)__shfl((int)bin, leader, 64);
    const bool same = valid && bin == bl;
    const unsigned long long sm = __ballot(same);
    if (lane_id() == leader) atomicAdd(&hist[bl], __popcll(sm));
    valid = valid && !same;
  }
  if (valid) atomicAdd(&hist[bin], 1);
}

// The digit holding the need-th key of a 256-bin histogram (all threads of
// the block; blockDim.x >= 256): an inclusive scan over the bins, then the
// bin whose range of cumulative counts contains need.  Sets *s_digit,
// *s_need (the rank within that digit) and *s_count (its keys).
NG_DEV void pick_digit(const int* hist, int need, int* s_wsum, int* s_digit, int* s_need,
                       int* s_count) {
  const int t = threadIdx.x;
  const int h = t < 256 ? hist[t] : 0;
  int x = h;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane_id() >= d) x += y;
  }
  if (t < 256 && lane_id() == 63) s_wsum[t >> 6] = x;
  __syncthreads();
  if (t < 256) {
    int off = 0;
    for (int w = 0; w < (t >> 6); ++w) off += s_wsum[w];
    const int incl = off + x, excl = incl - h;
    // the last bin takes whatever is left (need never exceeds the keys)
    if (excl < need && (incl >= need || t == 255)) {
      *s_digit = t;
      *s_need = need - excl;
      *s_count = h;
    }
  }
  __syncthreads();
}

// Pairs of segment b: idx[pstart[b] .. pend[b]) (idx null: pairs [0, M)).
// One workgroup per segment runs a radix select when its matching exceeds
// its budget P[b] (the matching of a segment's last pass only); mseg[b]
// receives the pairs kept.
__global__ void __launch_bounds__(1024)
k_topp_seg(const int* __restrict__ pair_a, const int* __restrict__ pair_b,
           const unsigned* __restrict__ pair_c, const int* __restrict__ idx,
           const int* __restrict__ pstart, const int* __restrict__ pend,
           const int* __restrict__ d_M, const long long* __restrict__ Pseg,
           const int* __restrict__ lg, int* __restrict__ partner, int* __restrict__ mseg) {
  constexpr int kTieCap = 2048;
  __shared__ int hist[256];
  __shared__ int s_wsum[4];
  __shared__ int s_digit, s_need, s_count, s_ntie;
  __shared__ unsigned long long s_k2[kTieCap];
  const int b = blockIdx.x;
  const int i0 = idx ? pstart[b] : 0;
  const int M = idx ? pend[b] - pstart[b] : *d_M;
  const long long Pll = Pseg[b];
  if ((long long)M <= Pll) {
    if (threadIdx.x == 0) mseg[b] = M;
    return;
  }
  const int P = (int)(Pll > 0 ? Pll : 0);
  auto at = [&](int i) { return idx ? idx[i0 + i] : i; };
  if (threadIdx.x == 0) mseg[b] = P;
  if (P == 0) {
    for (int i = threadIdx.x; i < M; i += blockDim.x) {
      const int e = at(i);
      partner[pair_a[e]] = -1;
      partner[pair_b[e]] = -1;
    }
    return;
  }
  // (loops run over whole blocks of threads so that every lane of a wave
  // reaches the ballots; eight keys per thread and step, their loads issued
  // together)
  constexpr int U = 8;
  const int stride = U * (int)blockDim.x;
  const int span = (M + stride - 1) / stride * stride;
  unsigned prefix = 0u;
  int need = P, tie_count = 0;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    const unsigned hi_mask = pass == 0 ? 0u : (0xffffffffu << (shift + 8));
    for (int d = threadIdx.x; d < 256; d += blockDim.x) hist[d] = 0;
    __syncthreads();
    for (int i0 = threadIdx.x; i0 < span; i0 += stride) {
      unsigned k[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        k[u] = i < M ? pair_c[at(i)] : 0u;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        hist_add(hist, (k[u] >> shift) & 255u, i < M && (k[u] & hi_mask) == (prefix & hi_mask));
      }
    }
    __syncthreads();
    pick_digit(hist, need, s_wsum, &s_digit, &s_need, &s_count);
    prefix |= (unsigned)s_digit << shift;
    need = s_need;
    tie_count = s_count;
    __syncthreads();
  }
  const unsigned T = prefix;
  const bool all_ties = tie_count == need;
  unsigned long long prefix2 = all_ties ? ~0ull : 0ull;
  if (!all_ties) {
    // several pairs share the cost T: rank them by (i, j), from an LDS copy
    // of their keys when they fit (else straight from the pair arrays)
    const bool in_lds = tie_count <= kTieCap;
    if (in_lds) {
      if (threadIdx.x == 0) s_ntie = 0;
      __syncthreads();
      for (int i0 = threadIdx.x; i0 < span; i0 += stride) {
        int ee[U];
        unsigned kk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * (int)blockDim.x;
          ee[u] = i < M ? at(i) : -1;
          kk[u] = ee[u] >= 0 ? pair_c[ee[u]] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (ee[u] >= 0 && kk[u] == T)
            s_k2[atomicAdd(&s_ntie, 1)] =
                ((unsigned long long)(unsigned)logical(lg, pair_a[ee[u]]) << 32) |
                (unsigned long long)(unsigned)logical(lg, pair_b[ee[u]]);
      }
      __syncthreads();
    }
    const int tspan = (tie_count + (int)blockDim.x - 1) / (int)blockDim.x * (int)blockDim.x;
    for (int pass = 0; pass < 8; ++pass) {
      const int shift = 56 - 8 * pass;
      const unsigned long long hi_mask = pass == 0 ? 0ull : (~0ull << (shift + 8));
      for (int d = threadIdx.x; d < 256; d += blockDim.x) hist[d] = 0;
      __syncthreads();
      if (in_lds) {
        for (int i = threadIdx.x; i < tspan; i += blockDim.x) {
          const unsigned long long k2 = i < tie_count ? s_k2[i] : 0ull;
          hist_add(hist, (unsigned)((k2 >> shift) & 255ull),
                   i < tie_count && (k2 & hi_mask) == (prefix2 & hi_mask));
        }
      } else {
        for (int i = threadIdx.x; i < span; i += blockDim.x) {
          bool v = false;
          unsigned long long k2 = 0ull;
          if (i < M) {
            const int e = at(i);
            if (pair_c[e] == T) {
              k2 = ((unsigned long long)(unsigned)logical(lg, pair_a[e]) << 32) |
                   (unsigned long long)(unsigned)logical(lg, pair_b[e]);
              v = (k2 & hi_mask) == (prefix2 & hi_mask);
            }
          }
          hist_add(hist, (unsigned)((k2 >> shift) & 255ull), v);
        }
      }
      __syncthreads();
      pick_digit(hist, need, s_wsum, &s_digit, &s_need, &s_count);
      prefix2 |= (unsigned long long)s_digit << shift;
      need = s_need;
      __syncthreads();
    }
  }
  const unsigned long long T2 = prefix2;
  for (int i0 = threadIdx.x; i0 < span; i0 += stride) {
    int ee[U];
    unsigned kk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * (int)blockDim.x;
      ee[u] = i < M ? at(i) : -1;
      kk[u] = ee[u] >= 0 ? pair_c[ee[u]] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = ee[u];
      if (e < 0) continue;
      const unsigned k = kk[u];
      bool kp = k < T;
      if (k == T) {
        const unsigned long long k2 =
            ((unsigned long long)(unsigned)logical(lg, pair_a[e]) << 32) |
            (unsigned long long)(unsigned)logical(lg, pair_b[e]);
        kp = k2 <= T2;
      }
      if (!kp) {
        partner[pair_a[e]] = -1;
        partner[pair_b[e]] = -1;
      }
    }
  }
}

// segment of every pair (sort key) and the identity payload, over cap
// slots: slots at and past the pair count *d_M get key `pad` (sorted last)
__global__ void k_pair_seg(const int* __restrict__ pair_a, const int* __restrict__ sg,
                           const int* __restrict__ d_M, int cap, unsigned pad,
                           unsigned* __restrict__ key, int* __restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  key[i] = i < *d_M ? (unsigned)sg[pair_a[i]] : pad;
  idx[i] = i;
}

// [pstart[s], pend[s]) = run of segment s in the sorted keys
__global__ void k_seg_runs(const unsigned* __restrict__ key, const int* __restrict__ d_M,
                           int* __restrict__ pstart, int* __restrict__ pend) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int M = *d_M;
  if (i >= M) return;
  const unsigned s = key[i];
  if (i == 0 || key[i - 1] != s) pstart[s] = i;
  if (i == M - 1 || key[i + 1] != s) pend[s] = i + 1;
}

__global__ void k_store_npairs(const int* __restrict__ v, long long* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = (long long)*v;
}

unsigned grid_for(long long cnt) {
  unsigned b = blocks_for(cnt, 256);
  return b > 8192 ? 8192 : b;
}

}  // namespace

size_t select_temp_bytes(long long n, long long m, int nseg) {
  Carver c(nullptr);
  c.take<int>(n);                 // pick
  c.take<unsigned>(n);            // pcost
  c.take<int>(n);                 // act A
  c.take<int>(n);                 // act B
  c.take<int>(n / 2 + 1);         // pair_a
  c.take<int>(n / 2 + 1);         // pair_b
  c.take<unsigned>(n / 2 + 1);    // pair_c
  c.take<unsigned>(n / 2 + 1);    // pair segment keys
  c.take<int>(n / 2 + 1);         // pair order
  c.take<int>(nseg);              // pstart
  c.take<int>(nseg);              // pend
  c.take<long long>(nseg);        // budgets
  c.take<int>(nseg);              // pairs kept
  c.take<int>(64);                // counters
  c.take<unsigned long long>(n * kTop);  // cached smallest keys
  c.take<int>(n * kTop);          // their other ends
  c.take<int>(n);                 // cached counts
  (void)m;
  return c.bytes() + sort_temp_bytes(n / 2 + 1);
}

size_t select_adj_bytes(long long n, long long m) {
  Carver c(nullptr);
  c.take<int>(n + 1);
  c.take<int>(n + 1);
  c.take<int>(n + 1);
  c.take<unsigned long long>(2 * m);
  c.take<int>(2 * m);
  return c.bytes() + scan_temp_bytes(n + 1);
}

void build_adjacency(const int* ea, const int* eb, const float* cost, long long m, int n,
                     Adjacency* adj, void* ws, hipStream_t st, const int* d_mcount) {
  Carver c(ws);
  int* deg = c.take<int>(n + 1);
  int* cursor = c.take<int>(n + 1);
  adj->aoff = c.take<int>(n + 1);
  adj->akey = c.take<unsigned long long>(2 * m);
  adj->au = c.take<int>(2 * m);
  void* stemp = (char*)ws + c.bytes();
  fill_i32(deg, 0, n + 1, st);
  fill_i32(cursor, 0, n + 1, st);
  if (m > 0) {
    unsigned b = blocks_for(m, 256);
    if (b > 4096) b = 4096;
    k_deg_count<<<b, 256, 0, st>>>(ea, eb, (int)m, n, deg, d_mcount);
    NG_LAUNCH_CHECK();
  }
  scan_exclusive_i32(deg, adj->aoff, n + 1, nullptr, stemp, st);
  if (m > 0) {
    unsigned b = blocks_for(m, 256);
    if (b > 4096) b = 4096;
    k_adj_fill<<<b, 256, 0, st>>>(ea, eb, cost, (int)m, n, adj->aoff, cursor, adj->akey, adj->au,
                                  d_mcount);
    NG_LAUNCH_CHECK();
  }
}

// The matching iterations on a fixed schedule: grid-wide iterations until
// about 2^11 vertices are left (each iteration leaves a bit over half of the
// active vertices on the synthetic scenes, about 1.2 iterations per
// halving), at least select_check of them, then one workgroup finishes the
// remaining ones on the device.  No host round trip happens; the grids of
// later launches are sized for the expected active count (the kernels stride
// over the actual one).  The first pick sets every partner entry to -1 and
// zeroes counters[0, 64); counters[2] receives the pairs, counters[3] the
// iterations of the finish.  Returns the grid-wide iterations launched.
int ld_iterations(const Adjacency& adj, int n, const int* lg, int* partner, int* pick,
                  unsigned* pcost, int* const act[2], int* pair_a, int* pair_b,
                  unsigned* pair_c, int* counters, const PickState& ps, hipStream_t st) {
  int grid_iters = (int)std::ceil(1.2 * std::log2(std::max((double)n, 2.0) / 2048.0));
  grid_iters = std::max(grid_iters, tuning_for(n).select_check);
  grid_iters = std::max(std::min(grid_iters, 24), 1);  // (the first one initialises)
  int it = 0;
  double expect = n;
  for (; it < grid_iters; ++it) {
    const int* in_list = it == 0 ? nullptr : act[(it + 1) & 1];
    const int* in_cnt = counters + ((it + 1) & 1);
    int* out_list = act[it & 1];
    int* out_cnt = counters + (it & 1);
    const long long span = std::max(2048ll, (long long)expect);
    expect *= 0.6;
    const unsigned g = grid_for(span);
    if (it == 0)
      k_ld_pick_first<<<grid_for(span * kPickLanes), 256, 0, st>>>(adj.aoff, adj.akey, adj.au, n,
                                                                   pick, pcost, counters, partner,
                                                                   ps);
    else
      k_ld_pick<<<g, 256, 0, st>>>(adj.aoff, adj.akey, adj.au, partner, in_list, in_cnt, n, pick,
                                   pcost, out_cnt, ps);
    NG_LAUNCH_CHECK();
    unsigned gm = (unsigned)((span + kMatchBlock - 1) / kMatchBlock);
    gm = gm < 1 ? 1 : (gm > 1024 ? 1024 : gm);
    k_ld_match<<<gm, kMatchBlock, 0, st>>>(in_list, in_cnt, n, pick, pcost, lg, partner,
                                           out_list, out_cnt, pair_a, pair_b, pair_c,
                                           counters + 2);
    NG_LAUNCH_CHECK();
  }
  k_ld_tail<<<1, kMatchBlock, 0, st>>>(adj.aoff, adj.akey, adj.au, partner, act[0], act[1],
                                       counters, (it - 1) & 1, pick, pcost, lg, pair_a, pair_b,
                                       pair_c, counters + 2, ps, counters + 3);
  NG_LAUNCH_CHECK();
  return it;
}

SelectResult select_pairs(const Adjacency& adj, int n, const int* lg, const int* sg, int nseg,
                          const long long* hP, int* partner, void* temp, hipStream_t st,
                          long long* d_npairs, long long* hM, const long long* dP) {
  Carver c(temp);
  int* pick = c.take<int>(n);
  unsigned* pcost = c.take<unsigned>(n);
  int* act[2] = {c.take<int>(n), c.take<int>(n)};
  int* pair_a = c.take<int>(n / 2 + 1);
  int* pair_b = c.take<int>(n / 2 + 1);
  unsigned* pair_c = c.take<unsigned>(n / 2 + 1);
  unsigned* pkey = c.take<unsigned>(n / 2 + 1);
  int* pidx = c.take<int>(n / 2 + 1);
  int* pstart = c.take<int>(nseg);
  int* pend = c.take<int>(nseg);
  long long* Pdev = c.take<long long>(nseg);
  int* mseg = c.take<int>(nseg);
  int* counters = c.take<int>(64);  // [0], [1]: active counts, [2]: pairs, [3]: tail iterations
  PickState ps;
  ps.tkey = c.take<unsigned long long>((long long)n * kTop);
  ps.tu = c.take<int>((long long)n * kTop);
  ps.tn = c.take<int>(n);
  void* stemp = (char*)temp + c.bytes();
  long long* host = pinned_host();

  SelectResult r{0, 0};
  const int it = ld_iterations(adj, n, lg, partner, pick, pcost, act, pair_a, pair_b, pair_c,
                               counters, ps, st);
  if (dP) {
    // device budget, single segment: keep the P smallest of the matching
    k_topp_seg<<<1, 1024, 0, st>>>(pair_a, pair_b, pair_c, nullptr, pstart, pend, counters + 2, dP,
                                   lg, partner, mseg);
    NG_LAUNCH_CHECK();
    if (d_npairs) {
      k_store_npairs<<<1, 64, 0, st>>>(mseg, d_npairs);
      NG_LAUNCH_CHECK();
    }
    return SelectResult{-1, -1};
  }
  NG_HIP(hipMemcpyAsync(host, counters, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  NG_HIP(hipStreamSynchronize(st));
  if (((const int*)host)[3] < 0) throw HipError{"internal: the matching did not converge"};
  r.iters = it + ((const int*)host)[3];
  const long long M = ((const int*)host)[2];
  // per-segment budgets (the matching of each segment, then its P smallest)
  NG_HIP(hipMemcpyAsync(Pdev, hP, nseg * sizeof(long long), hipMemcpyHostToDevice, st));
  const int* idx = nullptr;
  if (nseg > 1) {
    fill_i32(pstart, 0, nseg, st);
    fill_i32(pend, 0, nseg, st);
    if (M > 0) {
      k_pair_seg<<<blocks_for(M, 256), 256, 0, st>>>(pair_a, sg, counters + 2, (int)M,
                                                     (unsigned)nseg, pkey, pidx);
      NG_LAUNCH_CHECK();
      int bits = 1;
      while ((1 << bits) < nseg) ++bits;
      sort_pairs_u32(pkey, pidx, M, bits, stemp, st);
      k_seg_runs<<<blocks_for(M, 256), 256, 0, st>>>(pkey, counters + 2, pstart, pend);
      NG_LAUNCH_CHECK();
    }
    idx = pidx;
  }
  k_topp_seg<<<nseg, 1024, 0, st>>>(pair_a, pair_b, pair_c, idx, pstart, pend, counters + 2, Pdev,
                                     lg, partner, mseg);
  NG_LAUNCH_CHECK();
  if (d_npairs) {
    k_store_npairs<<<1, 64, 0, st>>>(mseg, d_npairs);
    NG_LAUNCH_CHECK();
  }
  long long total = 0;
  if (hM) {
    int* hm = (int*)(host + 8);
    for (int s0 = 0; s0 < nseg; s0 += 96) {
      const int cnt = nseg - s0 < 96 ? nseg - s0 : 96;
      NG_HIP(hipMemcpyAsync(hm, mseg + s0, cnt * sizeof(int), hipMemcpyDeviceToHost, st));
      NG_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < cnt; ++i) {
        hM[s0 + i] = hm[i];
        total += hm[i];
      }
    }
  } else {
    NG_HIP(hipStreamSynchronize(st));  // hP may be a stack value of the caller
    total = M;
    for (int i = 0; i < nseg; ++i) total = total < hP[i] ? total : hP[i];
  }
  r.pairs = total;
  return r;
}

// As select_pairs, with nothing read back and no synchronisation: the
// budgets come from hP in page-locked host memory (copied asynchronously;
// the caller keeps them unchanged until the stream reaches this point), the
// pairs kept per segment stay in device memory (*d_mseg, nseg ints) and so
// does the number of matching iterations the single-workgroup finish ran
// (*d_tail_iters).  Returns the grid-wide iterations launched.  Launches
// that depend on the pair count cover its capacity (n / 2 + 1).
int select_pairs_async(const Adjacency& adj, int n, const int* lg, const int* sg, int nseg,
                       const long long* dP, int* partner, void* temp, hipStream_t st,
                       const int** d_mseg, const int** d_tail_iters) {
  Carver c(temp);
  int* pick = c.take<int>(n);
  unsigned* pcost = c.take<unsigned>(n);
  int* act[2] = {c.take<int>(n), c.take<int>(n)};
  int* pair_a = c.take<int>(n / 2 + 1);
  int* pair_b = c.take<int>(n / 2 + 1);
  unsigned* pair_c = c.take<unsigned>(n / 2 + 1);
  unsigned* pkey = c.take<unsigned>(n / 2 + 1);
  int* pidx = c.take<int>(n / 2 + 1);
  int* pstart = c.take<int>(nseg);
  int* pend = c.take<int>(nseg);
  int* mseg = c.take<int>(nseg);
  int* counters = c.take<int>(64);
  PickState ps;
  ps.tkey = c.take<unsigned long long>((long long)n * kTop);
  ps.tu = c.take<int>((long long)n * kTop);
  ps.tn = c.take<int>(n);
  void* stemp = (char*)temp + c.bytes();

  const int it = ld_iterations(adj, n, lg, partner, pick, pcost, act, pair_a, pair_b, pair_c,
                               counters, ps, st);
  const int* idx = nullptr;
  if (nseg > 1) {
    const int cap = n / 2 + 1;
    fill_i32(pstart, 0, nseg, st);
    fill_i32(pend, 0, nseg, st);
    k_pair_seg<<<blocks_for(cap, 256), 256, 0, st>>>(pair_a, sg, counters + 2, cap,
                                                     (unsigned)nseg, pkey, pidx);
    NG_LAUNCH_CHECK();
    int bits = 1;
    while ((1 << bits) <= nseg) ++bits;  // the padding key nseg included
    sort_pairs_u32(pkey, pidx, cap, bits, stemp, st);
    k_seg_runs<<<blocks_for(cap, 256), 256, 0, st>>>(pkey, counters + 2, pstart, pend);
    NG_LAUNCH_CHECK();
    idx = pidx;
  }
  k_topp_seg<<<nseg, 1024, 0, st>>>(pair_a, pair_b, pair_c, idx, pstart, pend, counters + 2, dP,
                                     lg, partner, mseg);
  NG_LAUNCH_CHECK();
  *d_mseg = mseg;
  *d_tail_iters = counters + 3;
  return it;
}

}  // namespace ng
