// Device-wide exclusive prefix sums and fills.
#include "internal.h"

namespace ng {
namespace {

constexpr int SCAN_BS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_ITEMS;

// Exclusive scan of the per-thread values v across the block (256 threads).
__device__ int block_exclusive_scan(int v, int* total) {
  __shared__ int wsum[SCAN_BS / 64];
  const int lane = lane_id();
  const int w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_BS / 64; ++i) {
    int s = wsum[i];
    off += (i < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ void __launch_bounds__(SCAN_BS)
k_scan_tiles(const int* __restrict__ in, int* __restrict__ out, long long n,
             int* __restrict__ tile_sums, int* __restrict__ total) {
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    long long idx = base + i;
    v[i] = idx < n ? in[idx] : 0;
    s += v[i];
  }
  int tot;
  int run = block_exclusive_scan(s, &tot);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    long long idx = base + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) {
    if (tile_sums) tile_sums[blockIdx.x] = tot;
    if (total) *total = tot;
  }
}

// Two-kernel scan for up to kScanDirect tiles: the tile sums, then every
// tile adds up the sums of the tiles before it (a few KB that all blocks
// read from L2) and scans itself.  Reads the input twice and writes it
// once, in two launches.
constexpr int kScanDirect = 8192;

__device__ int block_sum(int v) {
  __shared__ int wsum[SCAN_BS / 64];
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  if (lane_id() == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int i = 0; i < SCAN_BS / 64; ++i) t += wsum[i];
  __syncthreads();
  return t;
}

// (blockIdx.y = 1: the second array of a two-array scan, in_b / sums_b)
__global__ void __launch_bounds__(SCAN_BS)
k_scan_reduce(const int* __restrict__ in, long long n, int* __restrict__ sums,
              const int* __restrict__ in_b, int* __restrict__ sums_b) {
  if (blockIdx.y) {
    in = in_b;
    sums = sums_b;
  }
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  int s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const long long idx = base + i;
    s += idx < n ? in[idx] : 0;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

__global__ void __launch_bounds__(SCAN_BS)
k_scan_apply(const int* __restrict__ in, int* __restrict__ out, long long n,
             const int* __restrict__ sums, int* __restrict__ total, const int* __restrict__ in_b,
             int* __restrict__ out_b, const int* __restrict__ sums_b, int* __restrict__ total_b) {
  if (blockIdx.y) {
    in = in_b;
    out = out_b;
    sums = sums_b;
    total = total_b;
  }
  int pre = 0;
  for (int t = threadIdx.x; t < (int)blockIdx.x; t += SCAN_BS) pre += sums[t];
  pre = block_sum(pre);
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const long long idx = base + i;
    v[i] = idx < n ? in[idx] : 0;
    s += v[i];
  }
  int tot;
  int run = block_exclusive_scan(s, &tot) + pre;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const long long idx = base + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
  if (total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = pre + tot;
}

__global__ void __launch_bounds__(SCAN_BS)
k_scan_add(int* __restrict__ out, long long n, const int* __restrict__ tile_off) {
  const int add = tile_off[blockIdx.x];
  const long long base = (long long)blockIdx.x * SCAN_TILE;
  for (int i = threadIdx.x; i < SCAN_TILE; i += SCAN_BS) {
    long long idx = base + i;
    if (idx < n) out[idx] += add;
  }
}

__global__ void k_fill_i32(int* p, int v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_set_i64(long long* d, long long v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *d = v;
}

__global__ void k_widen_i32(const int* __restrict__ s, long long* __restrict__ d) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *d = *s;
}

}  // namespace

namespace {
Tuning g_tuning[TUNE_BUCKETS];
}

int tune_bucket(long long n) { return n < 65536 ? 0 : n < 524288 ? 1 : 2; }
const Tuning& tuning_for(long long n) { return g_tuning[tune_bucket(n)]; }
void set_tuning(int bucket, const Tuning& t) { g_tuning[bucket] = t; }

void set_i64(long long* d, long long v, hipStream_t st) {
  k_set_i64<<<1, 64, 0, st>>>(d, v);
  NG_LAUNCH_CHECK();
}

void widen_i32(const int* s, long long* d, hipStream_t st) {
  k_widen_i32<<<1, 64, 0, st>>>(s, d);
  NG_LAUNCH_CHECK();
}

long long* pinned_host() {
  thread_local long long* buf = nullptr;
  if (!buf) NG_HIP(hipHostMalloc((void**)&buf, 64 * sizeof(long long), hipHostMallocDefault));
  return buf;
}

size_t scan_temp_bytes(long long n) {
  size_t b = 0;
  while (n > SCAN_TILE) {
    long long nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    b += 2 * (size_t)nt * sizeof(int) + 512;
    n = nt;
  }
  return b + 256;
}

void scan_exclusive_i32(const int* in, int* out, long long n, int* total, void* temp,
                        hipStream_t st) {
  if (n <= 0) {
    if (total) fill_i32(total, 0, 1, st);
    return;
  }
  if (n <= SCAN_TILE) {
    k_scan_tiles<<<1, SCAN_BS, 0, st>>>(in, out, n, nullptr, total);
    NG_LAUNCH_CHECK();
    return;
  }
  long long nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  Carver c(temp);
  int* sums = c.take<int>(nt);
  int* offs = c.take<int>(nt);
  void* rest = (char*)temp + c.bytes();
  if (nt <= kScanDirect) {
    k_scan_reduce<<<(unsigned)nt, SCAN_BS, 0, st>>>(in, n, sums, nullptr, nullptr);
    NG_LAUNCH_CHECK();
    k_scan_apply<<<(unsigned)nt, SCAN_BS, 0, st>>>(in, out, n, sums, total, nullptr, nullptr,
                                                   nullptr, nullptr);
    NG_LAUNCH_CHECK();
    return;
  }
  k_scan_tiles<<<(unsigned)nt, SCAN_BS, 0, st>>>(in, out, n, sums, nullptr);
  NG_LAUNCH_CHECK();
  scan_exclusive_i32(sums, offs, nt, total, rest, st);
  k_scan_add<<<(unsigned)nt, SCAN_BS, 0, st>>>(out, n, offs);
  NG_LAUNCH_CHECK();
}

void scan_exclusive2_i32(const int* in_a, int* out_a, int* total_a, const int* in_b, int* out_b,
                         int* total_b, long long n, void* temp, hipStream_t st) {
  const long long nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (n <= SCAN_TILE || nt > kScanDirect) {
    scan_exclusive_i32(in_a, out_a, n, total_a, temp, st);
    scan_exclusive_i32(in_b, out_b, n, total_b, temp, st);
    return;
  }
  // the two arrays' tile sums where one scan keeps its sums and offsets
  Carver c(temp);
  int* sums_a = c.take<int>(nt);
  int* sums_b = c.take<int>(nt);
  const dim3 grid((unsigned)nt, 2);
  k_scan_reduce<<<grid, SCAN_BS, 0, st>>>(in_a, n, sums_a, in_b, sums_b);
  NG_LAUNCH_CHECK();
  k_scan_apply<<<grid, SCAN_BS, 0, st>>>(in_a, out_a, n, sums_a, total_a, in_b, out_b, sums_b,
                                         total_b);
  NG_LAUNCH_CHECK();
}

__global__ void k_count_i32(const long long* __restrict__ d, long long cap, int* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const long long v = *d;
    *out = (int)(v < 0 ? 0 : (v > cap ? cap : v));
  }
}

void count_to_i32(const long long* d, long long cap, int* out, hipStream_t st) {
  k_count_i32<<<1, 64, 0, st>>>(d, cap, out);
  NG_LAUNCH_CHECK();
}

void fill_i32(int* p, int v, long long n, hipStream_t st) {
  if (n <= 0) return;
  k_fill_i32<<<blocks_for(n, 256), 256, 0, st>>>(p, v, n);
  NG_LAUNCH_CHECK();
}

void fill_u64(unsigned long long* p, unsigned long long v, long long n, hipStream_t st) {
  if (n <= 0) return;
  k_fill_u64<<<blocks_for(n, 256), 256, 0, st>>>(p, v, n);
  NG_LAUNCH_CHECK();
}

}  // namespace ng
