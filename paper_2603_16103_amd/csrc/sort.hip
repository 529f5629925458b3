// Stable least-significant-digit radix sort of (uint32 key, int32 value)
// pairs, 8-bit digits.  Each pass: per-tile digit counts (digit-major), one
// device-wide exclusive scan of the counts, then a scatter in which every
// tile ranks its keys stably (wave ballots give the rank among lanes with the
// same digit, LDS carries the count across waves and iterations).
#include "internal.h"

namespace ng {
namespace {

constexpr int SB = 256;       // threads per tile
constexpr int SITEMS = 8;     // keys per thread
constexpr int STILE = SB * SITEMS;

__global__ void __launch_bounds__(SB)
k_digit_counts(const unsigned* __restrict__ keys, long long n, int shift,
               int* __restrict__ counts, int ntiles) {
  __shared__ int hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * STILE;
#pragma unroll
  for (int i = 0; i < SITEMS; ++i) {
    long long idx = base + i * SB + threadIdx.x;
    if (idx < n) atomicAdd(&hist[(keys[idx] >> shift) & 255u], 1);
  }
  __syncthreads();
  counts[(long long)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ void __launch_bounds__(SB)
k_digit_scatter(const unsigned* __restrict__ kin, const int* __restrict__ vin,
                unsigned* __restrict__ kout, int* __restrict__ vout, long long n, int shift,
                const int* __restrict__ offs, int ntiles) {
  __shared__ int s_base[256];
  __shared__ int s_wc[SB / 64][256];
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int lane = lane_id();
  s_base[t] = offs[(long long)t * ntiles + blockIdx.x];
  const long long base = (long long)blockIdx.x * STILE;
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int i = 0; i < SITEMS; ++i) {
#pragma unroll
    for (int j = 0; j < SB / 64; ++j) s_wc[j][t] = 0;
    __syncthreads();
    const long long idx = base + (long long)i * SB + t;
    const bool valid = idx < n;
    const unsigned key = valid ? kin[idx] : 0u;
    const unsigned d = (key >> shift) & 255u;
    unsigned long long mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bal = __ballot(valid && bit);
      mask &= bit ? bal : ~bal;
    }
    const int rank_w = __popcll(mask & lt_mask);
    if (valid && rank_w == 0) s_wc[w][d] = __popcll(mask);
    __syncthreads();
    if (valid) {
      int pre = 0;
      for (int j = 0; j < w; ++j) pre += s_wc[j][d];
      const int pos = s_base[d] + pre + rank_w;
      kout[pos] = key;
      vout[pos] = vin[idx];
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int j = 0; j < SB / 64; ++j) add += s_wc[j][t];
    s_base[t] += add;
    __syncthreads();
  }
}

}  // namespace

size_t sort_temp_bytes(long long n) {
  long long nt = (n + STILE - 1) / STILE;
  if (nt < 1) nt = 1;
  Carver c(nullptr);
  c.take<unsigned>(n);
  c.take<int>(n);
  c.take<int>(256 * nt);
  c.take<int>(256 * nt);
  return c.bytes() + scan_temp_bytes(256 * nt);
}

void sort_pairs_u32(unsigned* keys, int* vals, long long n, int key_bits, void* temp,
                    hipStream_t st, int** out_vals) {
  if (out_vals) *out_vals = vals;
  if (n <= 1) return;
  long long nt = (n + STILE - 1) / STILE;
  Carver c(temp);
  unsigned* k2 = c.take<unsigned>(n);
  int* v2 = c.take<int>(n);
  int* counts = c.take<int>(256 * nt);
  int* offs = c.take<int>(256 * nt);
  void* stemp = (char*)temp + c.bytes();
  unsigned* ka = keys;
  int* va = vals;
  unsigned* kb = k2;
  int* vb = v2;
  int passes = (key_bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    int shift = 8 * p;
    k_digit_counts<<<(unsigned)nt, SB, 0, st>>>(ka, n, shift, counts, (int)nt);
    NG_LAUNCH_CHECK();
    scan_exclusive_i32(counts, offs, 256 * nt, nullptr, stemp, st);
    k_digit_scatter<<<(unsigned)nt, SB, 0, st>>>(ka, va, kb, vb, n, shift, offs, (int)nt);
    NG_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    if (out_vals) {  // the caller takes the values where they are
      *out_vals = va;
      return;
    }
    NG_HIP(hipMemcpyAsync(keys, ka, n * sizeof(unsigned), hipMemcpyDeviceToDevice, st));
    NG_HIP(hipMemcpyAsync(vals, va, n * sizeof(int), hipMemcpyDeviceToDevice, st));
  }
}

}  // namespace ng
