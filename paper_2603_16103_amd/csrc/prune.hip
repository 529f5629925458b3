// Opacity pre-filter of Algorithm 1 (the step before the loop): with
// tau' = min(tau, median of the opacities), keep the splats whose opacity
// alpha >= tau' (survivors keep their order).  The median of an even count
// is the mean of the two middle values.  The opacities are the activated
// float values (alpha = sigmoid(logit) rounded to float, as the rest of the
// library computes them); the median and the comparison are taken in double
// from those floats.  The median comes from a radix sort of the order-
// preserving keys of the opacities.
#include <algorithm>

#include "internal.h"

namespace ng {
namespace {

// activated opacity of a stored logit (the activation's own formula)
NG_DEV float alpha_of_logit(float op) { return (float)(1.0 / (1.0 + exp(-(double)op))); }

NG_DEV float alpha_at(const float* alpha, const float* logit, int i) {
  return alpha ? alpha[i] : alpha_of_logit(logit[i]);
}

__global__ void k_alpha_keys(const float* __restrict__ alpha, const float* __restrict__ logit,
                             int n, unsigned* __restrict__ keys, int* __restrict__ vals,
                             int* __restrict__ nonfinite) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float a = alpha_at(alpha, logit, i);
  if (!isfinite(a) || (logit && !isfinite(logit[i]))) atomicOr(nonfinite, 1);
  keys[i] = f2ord(a);
  vals[i] = i;
}

// tau' = min(tau, median) from the sorted keys (one thread)
__global__ void k_prune_tau(const unsigned* __restrict__ sorted, int n, float tau,
                            double* __restrict__ tau_out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double hi = (double)ord2f(sorted[n / 2]);
  const double med = (n % 2) ? hi : 0.5 * ((double)ord2f(sorted[n / 2 - 1]) + hi);
  *tau_out = fmin((double)tau, med);
}

__global__ void k_prune_keep(const float* __restrict__ alpha, const float* __restrict__ logit,
                             int n, const double* __restrict__ tau_p, int* __restrict__ keep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keep[i] = (double)alpha_at(alpha, logit, i) >= *tau_p ? 1 : 0;
}

// survivors of activated plain arrays, in order
__global__ void k_prune_gather_splats(const float* __restrict__ mu, const float* __restrict__ sc,
                                      const float* __restrict__ q, const float* __restrict__ al,
                                      const float* __restrict__ sh, const int* __restrict__ org,
                                      int n, const int* __restrict__ keep,
                                      const int* __restrict__ pos, float* __restrict__ mu_o,
                                      float* __restrict__ sc_o, float* __restrict__ q_o,
                                      float* __restrict__ al_o, float* __restrict__ sh_o,
                                      int* __restrict__ org_o, int* __restrict__ kept) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !keep[i]) return;
  const long long o = pos[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mu_o[3 * o + a] = mu[3 * (long long)i + a];
    sc_o[3 * o + a] = sc[3 * (long long)i + a];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) q_o[4 * o + a] = q[4 * (long long)i + a];
  al_o[o] = al[i];
  const float4* s4 = (const float4*)(sh + (long long)i * NG_SH);
  float4* d4 = (float4*)(sh_o + o * NG_SH);
#pragma unroll
  for (int c = 0; c < NG_SH / 4; ++c) d4[c] = s4[c];
  if (org && org_o) org_o[o] = org[i];
  if (kept) kept[o] = i;
}

// survivors of stored-form arrays, in order
__global__ void k_prune_gather_stored(const float* __restrict__ pos, const float* __restrict__ ls,
                                      const float* __restrict__ rot, const float* __restrict__ op,
                                      const float* __restrict__ sh, int n,
                                      const int* __restrict__ keep, const int* __restrict__ at,
                                      float* __restrict__ pos_o, float* __restrict__ ls_o,
                                      float* __restrict__ rot_o, float* __restrict__ op_o,
                                      float* __restrict__ sh_o, int* __restrict__ kept) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !keep[i]) return;
  const long long o = at[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    pos_o[3 * o + a] = pos[3 * (long long)i + a];
    ls_o[3 * o + a] = ls[3 * (long long)i + a];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) rot_o[4 * o + a] = rot[4 * (long long)i + a];
  op_o[o] = op[i];
  const float4* s4 = (const float4*)(sh + (long long)i * NG_SH);
  float4* d4 = (float4*)(sh_o + o * NG_SH);
#pragma unroll
  for (int c = 0; c < NG_SH / 4; ++c) d4[c] = s4[c];
  if (kept) kept[o] = i;
}

__global__ void k_count_to_i64(const int* __restrict__ v, long long* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = (long long)*v;
}

// v[i] = map[v[i]] for i < *count (count on the device, or count_host >= 0)
__global__ void k_remap(int* __restrict__ v, long long count, const int* __restrict__ map) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    if (v[i] >= 0) v[i] = map[v[i]];
}

struct PruneMem {
  unsigned* keys;
  int* vals;
  int* keep;
  int* pos;
  double* tau;
  int* counters;  // [0] survivors, [1] non-finite flag
  void* temp;
};

PruneMem carve_prune(void* base, long long n, size_t* bytes) {
  Carver c(base);
  PruneMem m;
  m.keys = c.take<unsigned>(n);
  m.vals = c.take<int>(n);
  m.keep = c.take<int>(n);
  m.pos = c.take<int>(n);
  m.tau = c.take<double>(1);
  m.counters = c.take<int>(64);
  m.temp = base ? (char*)base + c.bytes() : nullptr;
  if (bytes) *bytes = c.bytes() + std::max(sort_temp_bytes(n), scan_temp_bytes(n));
  return m;
}

// keep flags and output slots of the survivors; survivors' count -> m.counters[0]
void prune_flags(const float* alpha, const float* logit, int n, float tau, const PruneMem& m,
                 hipStream_t st) {
  fill_i32(m.counters, 0, 2, st);
  k_alpha_keys<<<blocks_for(n, 256), 256, 0, st>>>(alpha, logit, n, m.keys, m.vals,
                                                   m.counters + 1);
  NG_LAUNCH_CHECK();
  sort_pairs_u32(m.keys, m.vals, n, 32, m.temp, st);
  k_prune_tau<<<1, 64, 0, st>>>(m.keys, n, tau, m.tau);
  NG_LAUNCH_CHECK();
  k_prune_keep<<<blocks_for(n, 256), 256, 0, st>>>(alpha, logit, n, m.tau, m.keep);
  NG_LAUNCH_CHECK();
  scan_exclusive_i32(m.keep, m.pos, n, m.counters, m.temp, st);
}

}  // namespace

size_t prune_temp_bytes(long long n) {
  size_t b = 0;
  carve_prune(nullptr, n < 1 ? 1 : n, &b);
  return b;
}

void prune_splats(const float* mu, const float* scale, const float* quat, const float* alpha,
                  const float* sh, const int* origin, int n, float tau, float* mu_o,
                  float* scale_o, float* quat_o, float* alpha_o, float* sh_o, int* origin_o,
                  long long* d_nout, void* temp, hipStream_t st) {
  PruneMem m = carve_prune(temp, n, nullptr);
  prune_flags(alpha, nullptr, n, tau, m, st);
  k_prune_gather_splats<<<blocks_for(n, 256), 256, 0, st>>>(mu, scale, quat, alpha, sh, origin, n,
                                                            m.keep, m.pos, mu_o, scale_o, quat_o,
                                                            alpha_o, sh_o, origin_o, nullptr);
  NG_LAUNCH_CHECK();
  k_count_to_i64<<<1, 64, 0, st>>>(m.counters, d_nout);
  NG_LAUNCH_CHECK();
}

long long prune_stored(const float* pos, const float* ls, const float* rot, const float* op,
                       const float* sh, int n, float tau, float* pos_o, float* ls_o,
                       float* rot_o, float* op_o, float* sh_o, int* kept, bool* nonfinite,
                       void* temp, hipStream_t st) {
  PruneMem m = carve_prune(temp, n, nullptr);
  prune_flags(nullptr, op, n, tau, m, st);
  k_prune_gather_stored<<<blocks_for(n, 256), 256, 0, st>>>(pos, ls, rot, op, sh, n, m.keep,
                                                            m.pos, pos_o, ls_o, rot_o, op_o, sh_o,
                                                            kept);
  NG_LAUNCH_CHECK();
  long long* host = pinned_host();
  NG_HIP(hipMemcpyAsync(host, m.counters, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  NG_HIP(hipStreamSynchronize(st));
  *nonfinite = ((int*)host)[1] != 0;
  return ((int*)host)[0];
}

void remap_indices(int* v, long long count, const int* map, hipStream_t st) {
  if (count <= 0) return;
  unsigned b = blocks_for(count, 256);
  if (b > 4096) b = 4096;
  k_remap<<<b, 256, 0, st>>>(v, count, map);
  NG_LAUNCH_CHECK();
}

}  // namespace ng
