// Mass-preserved moment matching of the selected pairs (Sec. 3.3) and the new
// splat set (Algorithm 1 MergePairs).
//
// Per pair (i, j), in double: masses w = alpha s0 s1 s2 (Eq. vm_weights; the
// common (2 pi)^{3/2} cancels), pi = w_i / W; mu_m = pi mu_i + (1-pi) mu_j;
// f_m likewise; Sigma_m = pi Sigma_i + (1-pi) Sigma_j + pi (1-pi) d d^T with
// d = mu_i - mu_j, which equals Eq. vm_cov; alpha_m = 1 - (1-alpha_i)(1-alpha_j)
// (Eq. vm_alpha).  Sigma_m goes back to the 3DGS (scale, rotation) form through
// a cyclic Jacobi eigen-decomposition: eigenvalues in decreasing order
// (floored at 1e-12 of the largest), scale = sqrt(eigenvalue), the first two
// axes signed so their largest-magnitude component is positive, the third their
// cross product, and the quaternion of that rotation with w >= 0.
//
// Compaction: the merged splat replaces the splat that comes first in the
// logical order, the other is removed, and survivors keep their relative
// order, both in the working array and in the logical numbering.
#include <algorithm>

#include "internal.h"

namespace ng {
namespace {

NG_DEV int logical(const int* lg, int p) { return lg ? lg[p] : p; }

struct Mat3 {
  double m[3][3];
};

NG_DEV Mat3 cov_from(double s0, double s1, double s2, double w, double x, double y, double z) {
  const double nr = sqrt(w * w + x * x + y * y + z * z);
  w /= nr;
  x /= nr;
  y /= nr;
  z /= nr;
  const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                          {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                          {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
  const double l[3] = {s0 * s0, s1 * s1, s2 * s2};
  Mat3 S;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      S.m[i][j] = R[i][0] * l[0] * R[j][0] + R[i][1] * l[1] * R[j][1] + R[i][2] * l[2] * R[j][2];
  return S;
}

// Cyclic Jacobi on a symmetric 3x3: a -> diag(lambda), v columns = vectors.
NG_DEV void jacobi3(double a[3][3], double v[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) v[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > 1e-40 * dia)) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const int r = 3 - p - q;
      const double apq = a[p][q];
      if (apq == 0.0) continue;
      const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
      double t;
      if (fabs(theta) > 1e150) {
        t = 0.5 / theta;
      } else {
        t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
        if (theta < 0.0) t = -t;
      }
      const double c = 1.0 / sqrt(t * t + 1.0);
      const double s = t * c;
      const double arp = a[r][p], arq = a[r][q];
      a[p][p] -= t * apq;
      a[q][q] += t * apq;
      a[p][q] = a[q][p] = 0.0;
      a[r][p] = a[p][r] = c * arp - s * arq;
      a[r][q] = a[q][r] = s * arp + c * arq;
      for (int k = 0; k < 3; ++k) {
        const double vkp = v[k][p], vkq = v[k][q];
        v[k][p] = c * vkp - s * vkq;
        v[k][q] = s * vkp + c * vkq;
      }
    }
  }
}

struct ScaleRot {
  double s[3];
  double q[4];
};

NG_DEV ScaleRot scale_rot_from_cov(Mat3 S) {
  double a[3][3], v[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a[i][j] = S.m[i][j];
  jacobi3(a, v);
  double lam[3] = {a[0][0], a[1][1], a[2][2]};
  int o[3] = {0, 1, 2};
  // decreasing eigenvalues (three compare-exchanges)
  if (lam[o[0]] < lam[o[1]]) { int t = o[0]; o[0] = o[1]; o[1] = t; }
  if (lam[o[1]] < lam[o[2]]) { int t = o[1]; o[1] = o[2]; o[2] = t; }
  if (lam[o[0]] < lam[o[1]]) { int t = o[0]; o[0] = o[1]; o[1] = t; }
  const double top = fmax(lam[o[0]], 0.0);
  ScaleRot r;
  for (int k = 0; k < 3; ++k) r.s[k] = sqrt(fmax(lam[o[k]], 1e-12 * top));
  double e[2][3];
  for (int k = 0; k < 2; ++k) {
    for (int i = 0; i < 3; ++i) e[k][i] = v[i][o[k]];
    int piv = 0;
    for (int i = 1; i < 3; ++i)
      if (fabs(e[k][i]) > fabs(e[k][piv])) piv = i;
    if (e[k][piv] < 0.0)
      for (int i = 0; i < 3; ++i) e[k][i] = -e[k][i];
  }
  const double e3[3] = {e[0][1] * e[1][2] - e[0][2] * e[1][1],
                        e[0][2] * e[1][0] - e[0][0] * e[1][2],
                        e[0][0] * e[1][1] - e[0][1] * e[1][0]};
  // R columns = e1, e2, e3; quaternion by Shepperd's method
  const double R00 = e[0][0], R10 = e[0][1], R20 = e[0][2];
  const double R01 = e[1][0], R11 = e[1][1], R21 = e[1][2];
  const double R02 = e3[0], R12 = e3[1], R22 = e3[2];
  const double tr = R00 + R11 + R22;
  double w, x, y, z;
  if (tr >= R00 && tr >= R11 && tr >= R22) {
    w = 0.5 * sqrt(fmax(1.0 + tr, 0.0));
    x = (R21 - R12) / (4 * w);
    y = (R02 - R20) / (4 * w);
    z = (R10 - R01) / (4 * w);
  } else if (R00 >= R11 && R00 >= R22) {
    x = 0.5 * sqrt(fmax(1.0 + R00 - R11 - R22, 0.0));
    w = (R21 - R12) / (4 * x);
    y = (R01 + R10) / (4 * x);
    z = (R02 + R20) / (4 * x);
  } else if (R11 >= R22) {
    y = 0.5 * sqrt(fmax(1.0 - R00 + R11 - R22, 0.0));
    w = (R02 - R20) / (4 * y);
    x = (R01 + R10) / (4 * y);
    z = (R12 + R21) / (4 * y);
  } else {
    z = 0.5 * sqrt(fmax(1.0 - R00 - R11 + R22, 0.0));
    w = (R10 - R01) / (4 * z);
    x = (R02 + R20) / (4 * z);
    y = (R12 + R21) / (4 * z);
  }
  const double nr = sqrt(w * w + x * x + y * y + z * z);
  const double sg = w < 0.0 ? -1.0 : 1.0;
  r.q[0] = sg * w / nr;
  r.q[1] = sg * x / nr;
  r.q[2] = sg * y / nr;
  r.q[3] = sg * z / nr;
  return r;
}

__global__ void k_keep_flags(const int* __restrict__ partner, const int* __restrict__ lg, int n,
                             const int* __restrict__ sg, const SegInfo* __restrict__ seg,
                             int* __restrict__ keep, int* __restrict__ remL) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int j = partner[p];
  const int lp = logical(lg, p);
  const bool dropped = seg && seg[sg[p]].next < 0;
  const bool removed = dropped || (j >= 0 && j < n && logical(lg, j) < lp);
  keep[p] = removed ? 0 : 1;
  remL[lp] = removed ? 1 : 0;
}

// Mixture weights of a pair (masses w = alpha s0 s1 s2, Eq. vm_weights) and
// the merged centre rounded to float.  One definition for the sort keys and
// the merged rows, so the working set is sorted by the keys of its rows.
NG_DEV void pair_weights(float4 sa, float4 sb, double& pa, double& pb) {
#pragma clang fp contract(off)
  const double wa = (double)sa.w * (double)sa.x * (double)sa.y * (double)sa.z;
  const double wb = (double)sb.w * (double)sb.x * (double)sb.y * (double)sb.z;
  const double W = wa + wb;
  pa = W > 0.0 ? wa / W : 0.5;
  pb = W > 0.0 ? wb / W : 0.5;
}

NG_DEV float merged_coord(double pa, double pb, float a, float b) {
#pragma clang fp contract(off)
  return (float)(pa * (double)a + pb * (double)b);
}

// Output slot of every kept row (stable order) and, with a Morton box, the
// sort key of its output centre.
__global__ void k_out_keys(const float4* __restrict__ cen, const float4* __restrict__ shp, int n,
                           const int* __restrict__ partner, const int* __restrict__ keep,
                           const int* __restrict__ newpos, const int* __restrict__ sg,
                           const SegInfo* __restrict__ seg, unsigned* __restrict__ keys,
                           int* __restrict__ order) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || !keep[p]) return;
  const int q = newpos[p];
  order[q] = p;
  if (!seg) return;
  const unsigned* box = seg[sg[p]].box;
  const float4 ca = cen[p];
  float x = ca.x, y = ca.y, z = ca.z;
  const int j = partner[p];
  if (j >= 0 && j < n) {
    const float4 cb = cen[j];
    double pa, pb;
    pair_weights(shp[2 * (long long)p], shp[2 * (long long)j], pa, pb);
    x = merged_coord(pa, pb, ca.x, cb.x);
    y = merged_coord(pa, pb, ca.y, cb.y);
    z = merged_coord(pa, pb, ca.z, cb.z);
  }
  keys[q] = morton_key(x, y, z, box) >> kSortKeyShift;
}

// segment of each row in the Morton-sorted order (key of the stable second
// sort that groups the rows by segment)
__global__ void k_order_seg(const int* __restrict__ order, const int* __restrict__ sg, int nout,
                            unsigned* __restrict__ segkey) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nout) segkey[q] = (unsigned)sg[order[q]];
}

// float4 desc[q] = (src_a bits, src_b bits, weight_a, weight_b): how output
// row q of the SH array is formed.  Thread per output row q, source row
// order[q].
__global__ void k_merge_attrs(const float4* __restrict__ cen, const int* __restrict__ lg,
                              const float4* __restrict__ shp, const int* __restrict__ org, int n,
                              const int* __restrict__ partner, const int* __restrict__ order,
                              int nout, const int* __restrict__ rsum, const int* __restrict__ sg,
                              int* __restrict__ sg_o, const SegInfo* __restrict__ seg,
                              float4* __restrict__ cen_o, int* __restrict__ lg_o,
                              float4* __restrict__ shp_o, int* __restrict__ org_o,
                              float4* __restrict__ desc, int* __restrict__ trace,
                              int* __restrict__ trace_count, int* __restrict__ parent,
                              const int* __restrict__ d_nout) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (d_nout) nout = min(nout, *d_nout);
  if (q >= nout) return;
  const int p = order[q];
  const int lp = logical(lg, p);
  const int newL = lp - rsum[lp];
  if (sg_o) sg_o[q] = seg ? seg[sg[p]].next : 0;
  const int j = partner[p];
  const float4 ca = cen[p];
  const float4 sa = shp[2 * (long long)p], qa = shp[2 * (long long)p + 1];
  if (parent) {
    // hierarchy: both ends of a merged pair (or a lone splat) point at the
    // output splat they become, by logical index
    parent[lp] = newL;
    if (j >= 0 && j < n) parent[logical(lg, j)] = newL;
  }
  if (j < 0 || j >= n) {
    cen_o[q] = make_float4(ca.x, ca.y, ca.z, __int_as_float(newL));
    lg_o[q] = newL;
    shp_o[2 * (long long)q] = sa;
    shp_o[2 * (long long)q + 1] = qa;
    org_o[q] = org[p];
    desc[q] = make_float4(__int_as_float(p), __int_as_float(-1), 1.f, 0.f);
    return;
  }
  const float4 cb = cen[j];
  const float4 sb = shp[2 * (long long)j], qb = shp[2 * (long long)j + 1];
  double pa, pb;
  pair_weights(sa, sb, pa, pb);
  const double ma[3] = {ca.x, ca.y, ca.z}, mb[3] = {cb.x, cb.y, cb.z};
  const float mf[3] = {merged_coord(pa, pb, ca.x, cb.x), merged_coord(pa, pb, ca.y, cb.y),
                       merged_coord(pa, pb, ca.z, cb.z)};
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = ma[k] - mb[k];
  const Mat3 Sa = cov_from(sa.x, sa.y, sa.z, qa.x, qa.y, qa.z, qa.w);
  const Mat3 Sb = cov_from(sb.x, sb.y, sb.z, qb.x, qb.y, qb.z, qb.w);
  Mat3 Sm;
  const double c = pa * pb;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Sm.m[i][k] = pa * Sa.m[i][k] + pb * Sb.m[i][k] + c * d[i] * d[k];
  const double am = 1.0 - (1.0 - (double)sa.w) * (1.0 - (double)sb.w);
  const ScaleRot sr = scale_rot_from_cov(Sm);
  cen_o[q] = make_float4(mf[0], mf[1], mf[2], __int_as_float(newL));
  lg_o[q] = newL;
  shp_o[2 * (long long)q] = make_float4((float)sr.s[0], (float)sr.s[1], (float)sr.s[2], (float)am);
  shp_o[2 * (long long)q + 1] =
      make_float4((float)sr.q[0], (float)sr.q[1], (float)sr.q[2], (float)sr.q[3]);
  const int oa = org[p], ob = org[j];
  org_o[q] = min(oa, ob);
  desc[q] = make_float4(__int_as_float(p), __int_as_float(j), (float)pa, (float)pb);
  if (trace) {
    const int t = atomicAdd(trace_count, 1);
    trace[2 * (long long)t] = min(oa, ob);
    trace[2 * (long long)t + 1] = max(oa, ob);
  }
}

// thread per (output row, 16-byte chunk)
__global__ void k_merge_sh(const float4* __restrict__ sh, const float4* __restrict__ desc, int nout,
                           float4* __restrict__ sh_o, const int* __restrict__ d_nout) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (d_nout) nout = min(nout, *d_nout);
  if (t >= (long long)nout * 12) return;
  const int q = (int)(t / 12), c = (int)(t % 12);
  const float4 dq = desc[q];
  const int a = __float_as_int(dq.x), b = __float_as_int(dq.y);
  float4 x = sh[(long long)a * 12 + c];
  if (b >= 0) {
    const float4 y = sh[(long long)b * 12 + c];
    x.x = dq.z * x.x + dq.w * y.x;
    x.y = dq.z * x.y + dq.w * y.y;
    x.z = dq.z * x.z + dq.w * y.z;
    x.w = dq.z * x.w + dq.w * y.w;
  }
  sh_o[(long long)q * 12 + c] = x;
}

}  // namespace

size_t merge_temp_bytes(long long n) {
  Carver c(nullptr);
  c.take<int>(n);
  c.take<int>(n);
  c.take<int>(n);
  c.take<int>(n);
  c.take<unsigned>(n);
  c.take<int>(n);
  c.take<float4>(n);
  c.take<int>(64);
  return c.bytes() + std::max(scan_temp_bytes(n), sort_temp_bytes(n));
}

long long merge_compact(const float4* cen, const int* lg, const float4* shp, const float* sh,
                        const int* org, int n, const int* partner, float4* cen_o, int* lg_o,
                        float4* shp_o, float* sh_o, int* org_o, int* trace, void* temp,
                        hipStream_t st, int* d_nout_i32, const int* sg, int* sg_o,
                        const SegInfo* seg, int nseg, int* parent, bool host_count) {
  Carver c(temp);
  int* keep = c.take<int>(n);
  int* newpos = c.take<int>(n);
  int* remL = c.take<int>(n);
  int* rsum = c.take<int>(n);
  unsigned* keys = c.take<unsigned>(n);
  int* order = c.take<int>(n);
  float4* desc = c.take<float4>(n);
  int* counters = c.take<int>(64);
  void* stemp = (char*)temp + c.bytes();
  long long* host = pinned_host();
  k_keep_flags<<<blocks_for(n, 256), 256, 0, st>>>(partner, lg, n, seg ? sg : nullptr, seg, keep,
                                                   remL);
  NG_LAUNCH_CHECK();
  scan_exclusive2_i32(keep, newpos, counters, remL, rsum, counters + 1, n, stemp, st);
  if (trace) fill_i32(counters + 2, 0, 1, st);
  k_out_keys<<<blocks_for(n, 256), 256, 0, st>>>(cen, shp, n, partner, keep, newpos,
                                                 seg ? sg : nullptr, seg, keys, order);
  NG_LAUNCH_CHECK();
  if (d_nout_i32)
    NG_HIP(hipMemcpyAsync(d_nout_i32, counters, sizeof(int), hipMemcpyDeviceToDevice, st));
  if (!host_count) {
    // the count stays on the device: the launches cover n rows and read it
    k_merge_attrs<<<blocks_for(n, 256), 256, 0, st>>>(cen, lg, shp, org, n, partner, order, n,
                                                      rsum, nullptr, nullptr, nullptr, cen_o,
                                                      lg_o, shp_o, org_o, desc, trace,
                                                      counters + 2, parent, counters);
    NG_LAUNCH_CHECK();
    k_merge_sh<<<blocks_for((long long)n * 12, 256), 256, 0, st>>>((const float4*)sh, desc, n,
                                                                   (float4*)sh_o, counters);
    NG_LAUNCH_CHECK();
    return -1;
  }
  NG_HIP(hipMemcpyAsync(host, counters, sizeof(int), hipMemcpyDeviceToHost, st));
  NG_HIP(hipStreamSynchronize(st));
  const long long nout = *(int*)host;
  if (seg && nout > 0) {
    // Morton order of the output centres within each segment (stable:
    // equal keys keep the compacted order), then grouped by segment
    if (nseg > 1) {
      sort_pairs_u32(keys, order, nout, kSortKeyBits, stemp, st);
      k_order_seg<<<blocks_for(nout, 256), 256, 0, st>>>(order, sg, (int)nout, keys);
      NG_LAUNCH_CHECK();
      int bits = 1;
      while ((1 << bits) < nseg) ++bits;
      sort_pairs_u32(keys, order, nout, bits, stemp, st);
    } else {
      // (one segment: the sorted order is read where the sort left it; the
      // sort's temp is not touched again before the gathers below)
      sort_pairs_u32(keys, order, nout, kSortKeyBits, stemp, st, &order);
    }
  }
  if (nout > 0) {
    k_merge_attrs<<<blocks_for(nout, 256), 256, 0, st>>>(cen, lg, shp, org, n, partner, order,
                                                         (int)nout, rsum, seg ? sg : nullptr,
                                                         sg_o, seg, cen_o, lg_o, shp_o, org_o,
                                                         desc, trace, counters + 2, parent,
                                                         nullptr);
    NG_LAUNCH_CHECK();
    k_merge_sh<<<blocks_for(nout * 12, 256), 256, 0, st>>>((const float4*)sh, desc, (int)nout,
                                                           (float4*)sh_o, nullptr);
    NG_LAUNCH_CHECK();
  }
  return nout;
}

}  // namespace ng
