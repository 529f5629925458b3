// Boundary conversions between the stored 3DGS form, the plain activated
// arrays of the stage entry points, and the library's working layout.
//
// Activation (stored -> activated) is computed in double and rounded to
// float: s = exp(log_scale), alpha = 1 / (1 + exp(-logit)), q = r / |r|
// (r = 0 gives the identity rotation).  Deactivation clips alpha to [0, 1]
// (the last step of Algorithm 1), clamps it to [2^-24, 1 - 2^-24] so the
// logit stays finite in float, and returns log(s) and q with w >= 0.
#include "internal.h"

namespace ng {
namespace {

struct Act {
  float s0, s1, s2, alpha, qw, qx, qy, qz;
  bool finite;
};

NG_DEV Act activate_one(const float* ls, const float* rot, float op) {
  Act a;
  bool fin = isfinite(ls[0]) && isfinite(ls[1]) && isfinite(ls[2]) && isfinite(op) &&
             isfinite(rot[0]) && isfinite(rot[1]) && isfinite(rot[2]) && isfinite(rot[3]);
  a.s0 = (float)exp((double)ls[0]);
  a.s1 = (float)exp((double)ls[1]);
  a.s2 = (float)exp((double)ls[2]);
  a.alpha = (float)(1.0 / (1.0 + exp(-(double)op)));
  double w = rot[0], x = rot[1], y = rot[2], z = rot[3];
  double nr = sqrt(w * w + x * x + y * y + z * z);
  if (nr > 0.0) {
    a.qw = (float)(w / nr);
    a.qx = (float)(x / nr);
    a.qy = (float)(y / nr);
    a.qz = (float)(z / nr);
  } else {
    a.qw = 1.f;
    a.qx = a.qy = a.qz = 0.f;
  }
  a.finite = fin;
  return a;
}

struct Deact {
  float ls0, ls1, ls2, op, qw, qx, qy, qz;
};

NG_DEV Deact deactivate_one(float s0, float s1, float s2, float alpha, float qw, float qx,
                            float qy, float qz) {
  Deact d;
  d.ls0 = (float)log((double)s0);
  d.ls1 = (float)log((double)s1);
  d.ls2 = (float)log((double)s2);
  const double eps = 5.9604644775390625e-08;  // 2^-24
  double a = fmin(fmax((double)alpha, 0.0), 1.0);
  a = fmin(fmax(a, eps), 1.0 - eps);
  d.op = (float)log(a / (1.0 - a));
  double w = qw, x = qx, y = qy, z = qz;
  double nr = sqrt(w * w + x * x + y * y + z * z);
  if (!(nr > 0.0)) {
    w = 1.0;
    x = y = z = 0.0;
    nr = 1.0;
  }
  double sg = (w < 0.0) ? -1.0 : 1.0;
  d.qw = (float)(sg * w / nr);
  d.qx = (float)(sg * x / nr);
  d.qy = (float)(sg * y / nr);
  d.qz = (float)(sg * z / nr);
  return d;
}

__global__ void k_activate_stored(const float* __restrict__ pos, const float* __restrict__ ls,
                                  const float* __restrict__ rot, const float* __restrict__ op,
                                  const int* __restrict__ perm, int n, int lbase,
                                  float4* __restrict__ cen, int* __restrict__ lg,
                                  float4* __restrict__ shp, int* __restrict__ org,
                                  int* __restrict__ sg, int sgid, int* __restrict__ nonfinite) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int i = perm ? perm[p] : p;
  if (sg) sg[p] = sgid;
  float x = pos[3 * (long long)i], y = pos[3 * (long long)i + 1], z = pos[3 * (long long)i + 2];
  Act a = activate_one(ls + 3 * (long long)i, rot + 4 * (long long)i, op[i]);
  if (!(a.finite && isfinite(x) && isfinite(y) && isfinite(z))) *nonfinite = 1;
  cen[p] = make_float4(x, y, z, __int_as_float(lbase + i));
  lg[p] = lbase + i;
  shp[2 * (long long)p] = make_float4(a.s0, a.s1, a.s2, a.alpha);
  shp[2 * (long long)p + 1] = make_float4(a.qw, a.qx, a.qy, a.qz);
  org[p] = i;
}

// Two-step form: first the rows in input order (coalesced reads), then a
// gather of the activated rows in the working order (two 16-byte-aligned
// reads per row instead of four scattered input fields).
__global__ void k_activate_in(const float* __restrict__ pos, const float* __restrict__ ls,
                              const float* __restrict__ rot, const float* __restrict__ op, int n,
                              int lbase, float4* __restrict__ cen_t, float4* __restrict__ shp_t,
                              int* __restrict__ nonfinite) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long i3 = 3 * (long long)i;
  const float x = pos[i3], y = pos[i3 + 1], z = pos[i3 + 2];
  Act a = activate_one(ls + i3, rot + 4 * (long long)i, op[i]);
  if (!(a.finite && isfinite(x) && isfinite(y) && isfinite(z))) *nonfinite = 1;
  cen_t[i] = make_float4(x, y, z, __int_as_float(lbase + i));
  shp_t[2 * (long long)i] = make_float4(a.s0, a.s1, a.s2, a.alpha);
  shp_t[2 * (long long)i + 1] = make_float4(a.qw, a.qx, a.qy, a.qz);
}

__global__ void k_gather_act(const int* __restrict__ perm, int n, int lbase,
                             const float4* __restrict__ cen_t, const float4* __restrict__ shp_t,
                             float4* __restrict__ cen, int* __restrict__ lg,
                             float4* __restrict__ shp, int* __restrict__ org,
                             int* __restrict__ sg, int sgid) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int i = perm[p];
  const float4 c = cen_t[i], s0 = shp_t[2 * (long long)i], s1 = shp_t[2 * (long long)i + 1];
  cen[p] = c;
  shp[2 * (long long)p] = s0;
  shp[2 * (long long)p + 1] = s1;
  lg[p] = lbase + i;
  org[p] = i;
  if (sg) sg[p] = sgid;
}

__global__ void k_activate_plain(const float* __restrict__ pos, const float* __restrict__ ls,
                                 const float* __restrict__ rot, const float* __restrict__ op,
                                 int n, float* __restrict__ mu, float* __restrict__ scale,
                                 float* __restrict__ quat, float* __restrict__ alpha,
                                 int* __restrict__ nonfinite) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  long long i3 = 3 * (long long)i, i4 = 4 * (long long)i;
  float x = pos[i3], y = pos[i3 + 1], z = pos[i3 + 2];
  Act a = activate_one(ls + i3, rot + i4, op[i]);
  if (nonfinite && !(a.finite && isfinite(x) && isfinite(y) && isfinite(z))) *nonfinite = 1;
  mu[i3] = x;
  mu[i3 + 1] = y;
  mu[i3 + 2] = z;
  scale[i3] = a.s0;
  scale[i3 + 1] = a.s1;
  scale[i3 + 2] = a.s2;
  alpha[i] = a.alpha;
  quat[i4] = a.qw;
  quat[i4 + 1] = a.qx;
  quat[i4 + 2] = a.qy;
  quat[i4 + 3] = a.qz;
}

__global__ void k_check_finite(const float* __restrict__ x, long long count,
                               int* __restrict__ nonfinite) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  bool bad = false;
  for (; i < count; i += stride) bad |= !isfinite(x[i]);
  if (bad) *nonfinite = 1;
}

// thread per (row, 16-byte chunk): consecutive threads touch consecutive
// 16-byte words of a row, so each row is read and written in full lines.
// nonfinite (nullable): set to 1 if a copied value is NaN or infinite.
__global__ void k_copy_sh_rows(const float4* __restrict__ src, const int* __restrict__ src_map,
                               float4* __restrict__ dst, const int* __restrict__ dst_map,
                               int dst_base, int rows, int* __restrict__ nonfinite) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)rows * 12) return;
  int r = (int)(t / 12), c = (int)(t % 12);
  int sr = src_map ? src_map[r] : r;
  int dr = dst_map ? dst_map[r] - dst_base : r;
  const float4 v = src[(long long)sr * 12 + c];
  dst[(long long)dr * 12 + c] = v;
  if (nonfinite && !(isfinite(v.x) && isfinite(v.y) && isfinite(v.z) && isfinite(v.w)))
    *nonfinite = 1;
}

__global__ void k_deactivate_work(const float4* __restrict__ cen, const int* __restrict__ lg,
                                  const float4* __restrict__ shp, const int* __restrict__ org,
                                  int n, int lbase, float* __restrict__ pos,
                                  float* __restrict__ ls, float* __restrict__ rot,
                                  float* __restrict__ op, int* __restrict__ origin_out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  long long L = lg[p] - lbase;
  float4 c = cen[p];
  float4 a = shp[2 * (long long)p];
  float4 q = shp[2 * (long long)p + 1];
  Deact d = deactivate_one(a.x, a.y, a.z, a.w, q.x, q.y, q.z, q.w);
  pos[3 * L] = c.x;
  pos[3 * L + 1] = c.y;
  pos[3 * L + 2] = c.z;
  ls[3 * L] = d.ls0;
  ls[3 * L + 1] = d.ls1;
  ls[3 * L + 2] = d.ls2;
  op[L] = d.op;
  rot[4 * L] = d.qw;
  rot[4 * L + 1] = d.qx;
  rot[4 * L + 2] = d.qy;
  rot[4 * L + 3] = d.qz;
  if (origin_out) origin_out[L] = org[p];
}

__global__ void k_deactivate_plain(const float* __restrict__ mu, const float* __restrict__ scale,
                                   const float* __restrict__ quat,
                                   const float* __restrict__ alpha, int n,
                                   float* __restrict__ pos, float* __restrict__ ls,
                                   float* __restrict__ rot, float* __restrict__ op) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  long long i3 = 3 * (long long)i, i4 = 4 * (long long)i;
  Deact d = deactivate_one(scale[i3], scale[i3 + 1], scale[i3 + 2], alpha[i], quat[i4],
                           quat[i4 + 1], quat[i4 + 2], quat[i4 + 3]);
  pos[i3] = mu[i3];
  pos[i3 + 1] = mu[i3 + 1];
  pos[i3 + 2] = mu[i3 + 2];
  ls[i3] = d.ls0;
  ls[i3 + 1] = d.ls1;
  ls[i3 + 2] = d.ls2;
  op[i] = d.op;
  rot[i4] = d.qw;
  rot[i4 + 1] = d.qx;
  rot[i4 + 2] = d.qy;
  rot[i4 + 3] = d.qz;
}

__global__ void k_pack(const float* __restrict__ mu, const float* __restrict__ scale,
                       const float* __restrict__ quat, const float* __restrict__ alpha,
                       const int* __restrict__ origin, int n, float4* __restrict__ cen,
                       int* __restrict__ lg, float4* __restrict__ shp, int* __restrict__ org) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  long long p3 = 3 * (long long)p, p4 = 4 * (long long)p;
  cen[p] = make_float4(mu[p3], mu[p3 + 1], mu[p3 + 2], __int_as_float(p));
  lg[p] = p;
  shp[2 * (long long)p] = make_float4(scale[p3], scale[p3 + 1], scale[p3 + 2], alpha[p]);
  shp[2 * (long long)p + 1] = make_float4(quat[p4], quat[p4 + 1], quat[p4 + 2], quat[p4 + 3]);
  org[p] = origin ? origin[p] : p;
}

__global__ void k_unpack(const float4* __restrict__ cen, const float4* __restrict__ shp,
                         const int* __restrict__ org, int n, float* __restrict__ mu,
                         float* __restrict__ scale, float* __restrict__ quat,
                         float* __restrict__ alpha, int* __restrict__ origin,
                         const int* __restrict__ d_n) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (d_n) n = min(n, *d_n);
  if (p >= n) return;
  long long p3 = 3 * (long long)p, p4 = 4 * (long long)p;
  float4 c = cen[p], a = shp[2 * (long long)p], q = shp[2 * (long long)p + 1];
  mu[p3] = c.x;
  mu[p3 + 1] = c.y;
  mu[p3 + 2] = c.z;
  scale[p3] = a.x;
  scale[p3 + 1] = a.y;
  scale[p3 + 2] = a.z;
  alpha[p] = a.w;
  quat[p4] = q.x;
  quat[p4 + 1] = q.y;
  quat[p4 + 2] = q.z;
  quat[p4 + 3] = q.w;
  if (origin) origin[p] = org[p];
}

}  // namespace

void launch_activate_stored(const float* pos, const float* log_scale, const float* rot,
                            const float* opacity, const int* perm, int n, int lbase, float4* cen,
                            int* lg, float4* shp, int* org, int* sg, int sgid, int* nonfinite,
                            hipStream_t st, float4* cen_t, float4* shp_t) {
  if (n <= 0) return;
  if (perm && cen_t && shp_t) {
    k_activate_in<<<blocks_for(n, 256), 256, 0, st>>>(pos, log_scale, rot, opacity, n, lbase,
                                                      cen_t, shp_t, nonfinite);
    NG_LAUNCH_CHECK();
    k_gather_act<<<blocks_for(n, 256), 256, 0, st>>>(perm, n, lbase, cen_t, shp_t, cen, lg, shp,
                                                     org, sg, sgid);
    NG_LAUNCH_CHECK();
    return;
  }
  k_activate_stored<<<blocks_for(n, 256), 256, 0, st>>>(pos, log_scale, rot, opacity, perm, n,
                                                        lbase, cen, lg, shp, org, sg, sgid,
                                                        nonfinite);
  NG_LAUNCH_CHECK();
}

void launch_check_finite(const float* x, long long count, int* nonfinite, hipStream_t st) {
  if (count <= 0) return;
  unsigned b = blocks_for(count, 256);
  if (b > 4096) b = 4096;
  k_check_finite<<<b, 256, 0, st>>>(x, count, nonfinite);
  NG_LAUNCH_CHECK();
}

void launch_copy_sh_rows(const float* src, const int* src_map, float* dst, const int* dst_map,
                         int dst_base, int rows, hipStream_t st, int* nonfinite) {
  if (rows <= 0) return;
  k_copy_sh_rows<<<blocks_for((long long)rows * 12, 256), 256, 0, st>>>(
      (const float4*)src, src_map, (float4*)dst, dst_map, dst_base, rows, nonfinite);
  NG_LAUNCH_CHECK();
}

void launch_deactivate_work(const float4* cen, const int* lg, const float4* shp, const int* org,
                            int n, int lbase, float* pos, float* log_scale, float* rot,
                            float* opacity, int* origin_out, hipStream_t st) {
  if (n <= 0) return;
  k_deactivate_work<<<blocks_for(n, 256), 256, 0, st>>>(cen, lg, shp, org, n, lbase, pos,
                                                        log_scale, rot, opacity, origin_out);
  NG_LAUNCH_CHECK();
}

void launch_pack_splats(const float* mu, const float* scale, const float* quat, const float* alpha,
                        const int* origin, int n, float4* cen, int* lg, float4* shp, int* org,
                        hipStream_t st) {
  if (n <= 0) return;
  k_pack<<<blocks_for(n, 256), 256, 0, st>>>(mu, scale, quat, alpha, origin, n, cen, lg, shp, org);
  NG_LAUNCH_CHECK();
}

void launch_unpack_splats(const float4* cen, const float4* shp, const int* org, int n, float* mu,
                          float* scale, float* quat, float* alpha, int* origin, hipStream_t st,
                          const int* d_n) {
  if (n <= 0) return;
  k_unpack<<<blocks_for(n, 256), 256, 0, st>>>(cen, shp, org, n, mu, scale, quat, alpha, origin,
                                               d_n);
  NG_LAUNCH_CHECK();
}

void launch_activate_plain(const float* pos, const float* log_scale, const float* rot,
                           const float* opacity, int n, float* mu, float* scale, float* quat,
                           float* alpha, int* nonfinite, hipStream_t st) {
  if (n <= 0) return;
  k_activate_plain<<<blocks_for(n, 256), 256, 0, st>>>(pos, log_scale, rot, opacity, n, mu, scale,
                                                       quat, alpha, nonfinite);
  NG_LAUNCH_CHECK();
}

void launch_deactivate_plain(const float* mu, const float* scale, const float* quat,
                             const float* alpha, int n, float* pos, float* log_scale, float* rot,
                             float* opacity, hipStream_t st) {
  if (n <= 0) return;
  k_deactivate_plain<<<blocks_for(n, 256), 256, 0, st>>>(mu, scale, quat, alpha, n, pos,
                                                         log_scale, rot, opacity);
  NG_LAUNCH_CHECK();
}

}  // namespace ng
