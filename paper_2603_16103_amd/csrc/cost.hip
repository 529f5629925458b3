// Merge cost of every candidate edge (Sec. 3.2): C = D_geo + D_app
// (Eq. cost), D_geo = KL(p~_ij || q_m) estimated with the S shared draws of
// Appendix A, D_app = ||f_i - f_j||^2.
//
// Arithmetic, per edge (i = first endpoint, j = second):
//   pi = w_i / (w_i + w_j) (Eq. norm_mixture), d = mu_i - mu_j,
//   merged covariance (Eq. vm_cov) = A + pi (1-pi) d d^T with
//   A = pi Sigma_i + (1-pi) Sigma_j.
// A is never formed: with Sigma = L L^T for each splat, A = G G^T for
// G = [sqrt(pi) L_i | sqrt(1-pi) L_j] (3x6), and six Givens rotations reduce
// G to its 3x3 lower-triangular LQ factor L_A, the Cholesky factor of A.  The
// rank-one dispersion term enters in closed form: with e = L_A^-1 d and
// c = pi (1-pi),
//   log det Sigma_m = 2 log det L_A + log(1 + c |e|^2),
//   y^T Sigma_m^-1 y for y = beta d + t, v = L_A^-1 t:
//     |v - (v.e^)e^|^2 + (beta |e| + v.e^)^2 / (1 + c |e|^2).
// A draw (u, z) picks splat i when u < pi, x = mu_c + L_c z, so
//   log N_c(x) = -|z|^2/2 - log det L_c exactly, and the other two log
// densities are triangular solves.  The -(3/2) log 2 pi constant cancels.
// Working with the factors keeps the float error near eps * sqrt(cond)
// instead of eps * cond; edges whose factors still look ill-conditioned
// (a diagonal ratio below fb_ratio) or give a non-finite value are recomputed
// in double from (s, q) by a second kernel.
#include "../../include/nanogs.h"
#include "internal.h"

namespace ng {
namespace {

template <typename T>
struct V3 {
  T x, y, z;
};
template <typename T>
NG_DEV V3<T> v3(T x, T y, T z) {
  return {x, y, z};
}
template <typename T>
NG_DEV T dot(const V3<T>& a, const V3<T>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}

// lower-triangular [[a00,0,0],[a10,a11,0],[a20,a21,a22]]
template <typename T>
struct Tri {
  T a00, a10, a11, a20, a21, a22;
};

// Reciprocal, square root and reciprocal square root: in float the
// hardware's single-instruction forms (about 1 ulp; every float result is
// checked against the fallback trigger and compared with a tolerance), in
// double the correctly rounded ones.
NG_DEV float rcp_of(float x) { return __builtin_amdgcn_rcpf(x); }
NG_DEV double rcp_of(double x) { return 1.0 / x; }
NG_DEV float sqrt_of(float x) { return __builtin_amdgcn_sqrtf(x); }
NG_DEV double sqrt_of(double x) { return sqrt(x); }
// Logarithm and exponential: in float the hardware's base-2 forms (an
// absolute error of a few 1e-7 on the logarithms that enter the cost), in
// double the library's.
NG_DEV float log_of(float x) { return __logf(x); }
NG_DEV double log_of(double x) { return log(x); }
NG_DEV float log1p_of(float x) { return __logf(1.0f + x); }
NG_DEV double log1p_of(double x) { return log1p(x); }
NG_DEV float exp_of(float x) { return __expf(x); }
NG_DEV double exp_of(double x) { return exp(x); }

template <typename T>
NG_DEV V3<T> tri_mul(const Tri<T>& L, const V3<T>& z) {
  return {L.a00 * z.x, L.a10 * z.x + L.a11 * z.y, L.a20 * z.x + L.a21 * z.y + L.a22 * z.z};
}

template <typename T>
NG_DEV V3<T> tri_solve(const Tri<T>& L, const V3<T>& y) {
  V3<T> v;
  v.x = y.x * rcp_of(L.a00);
  v.y = (y.y - L.a10 * v.x) * rcp_of(L.a11);
  v.z = (y.z - L.a20 * v.x - L.a21 * v.y) * rcp_of(L.a22);
  return v;
}

template <typename T>
NG_DEV T tri_ratio(const Tri<T>& L) {
  T mn = fmin(fmin(L.a00, L.a11), L.a22);
  T mx = fmax(fmax(L.a00, L.a11), L.a22);
  return mn * rcp_of(mx);
}

// Rotates columns (ci, cj) of the 3 x NC row-major matrix g so that
// g[row][cj] becomes zero and g[row][ci] >= 0.
template <typename T, int NC>
NG_DEV void givens(T (&g)[3][NC], int row, int ci, int cj) {
  const T x = g[row][ci], y = g[row][cj];
  const T r = sqrt_of(x * x + y * y);
  if (!(r > T(0))) return;
  const T ir = rcp_of(r);
  const T c = x * ir, s = y * ir;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (i >= row) {
      const T gi = g[i][ci], gj = g[i][cj];
      g[i][ci] = c * gi + s * gj;
      g[i][cj] = c * gj - s * gi;
    }
  }
}

// Cholesky factor of pa * La La^T + pb * Lb Lb^T, by LQ of [ra La | rb Lb].
template <typename T>
NG_DEV Tri<T> chol_of_mix(const Tri<T>& La, const Tri<T>& Lb, T ra, T rb) {
  T g[3][6] = {{ra * La.a00, T(0), T(0), rb * Lb.a00, T(0), T(0)},
               {ra * La.a10, ra * La.a11, T(0), rb * Lb.a10, rb * Lb.a11, T(0)},
               {ra * La.a20, ra * La.a21, ra * La.a22, rb * Lb.a20, rb * Lb.a21, rb * Lb.a22}};
  givens<T, 6>(g, 0, 0, 3);
  givens<T, 6>(g, 1, 1, 3);
  givens<T, 6>(g, 1, 1, 4);
  givens<T, 6>(g, 2, 2, 3);
  givens<T, 6>(g, 2, 2, 4);
  givens<T, 6>(g, 2, 2, 5);
  return {g[0][0], g[1][0], g[1][1], g[2][0], g[2][1], g[2][2]};
}

// Cholesky factor of R(q) diag(s^2) R(q)^T by LQ of M = R(q) diag(s).
template <typename T>
NG_DEV Tri<T> chol_from_scale_rot(T s0, T s1, T s2, T w, T x, T y, T z) {
  const T nr = sqrt(w * w + x * x + y * y + z * z);
  w /= nr;
  x /= nr;
  y /= nr;
  z /= nr;
  const T R00 = T(1) - T(2) * (y * y + z * z), R01 = T(2) * (x * y - w * z),
          R02 = T(2) * (x * z + w * y);
  const T R10 = T(2) * (x * y + w * z), R11 = T(1) - T(2) * (x * x + z * z),
          R12 = T(2) * (y * z - w * x);
  const T R20 = T(2) * (x * z - w * y), R21 = T(2) * (y * z + w * x),
          R22 = T(1) - T(2) * (x * x + y * y);
  T g[3][3] = {{R00 * s0, R01 * s1, R02 * s2},
               {R10 * s0, R11 * s1, R12 * s2},
               {R20 * s0, R21 * s1, R22 * s2}};
  givens<T, 3>(g, 0, 0, 1);
  givens<T, 3>(g, 0, 0, 2);
  givens<T, 3>(g, 1, 1, 2);
  const T l22 = g[2][2] < T(0) ? -g[2][2] : g[2][2];
  return {g[0][0], g[1][0], g[1][1], g[2][0], g[2][1], l22};
}

// Back substitution with the transpose: h = L^-T y.
template <typename T>
NG_DEV V3<T> tri_solve_t(const Tri<T>& L, const V3<T>& y) {
  V3<T> h;
  h.z = y.z * rcp_of(L.a22);
  h.y = (y.y - L.a21 * h.z) * rcp_of(L.a11);
  h.x = (y.x - L.a10 * h.y - L.a20 * h.z) * rcp_of(L.a00);
  return h;
}

// L^T h for lower-triangular L.
template <typename T>
NG_DEV V3<T> tri_mul_t(const Tri<T>& L, const V3<T>& h) {
  return {L.a00 * h.x + L.a10 * h.y + L.a20 * h.z, L.a11 * h.y + L.a21 * h.z, L.a22 * h.z};
}

// Geometric term of the cost (NANOGS_COST_*):
//   MC     the Monte Carlo estimate of Appendix A: each draw picks the
//          component by u < pi and evaluates g = log p~(x) - log q_m(x);
//   STRAT  each draw's z is used in both components, weighted pi and 1 - pi
//          (the same expectation, no component draw);
//   BOUND  pi KL(N_i || q_m) + (1 - pi) KL(N_j || q_m) in closed form (the
//          single-Gaussian KL of Appendix A; joint convexity makes it an
//          upper bound of the mixture's divergence), no draws.
// ratio receives the smallest diagonal ratio seen.
template <typename T>
NG_DEV T dgeo_pair(const V3<T>& mua, const V3<T>& mub, const Tri<T>& La, const Tri<T>& Lb,
                   T ldLa, T ldLb, T pa, T pb, double pdec, const float* __restrict__ cv, int S,
                   int mode, T& ratio) {
  const V3<T> d = {mua.x - mub.x, mua.y - mub.y, mua.z - mub.z};
  const Tri<T> LA = chol_of_mix(La, Lb, sqrt_of(pa), sqrt_of(pb));
  ratio = fmin(fmin(tri_ratio(La), tri_ratio(Lb)), tri_ratio(LA));
  const V3<T> e = tri_solve(LA, d);
  const T ee = dot(e, e);
  const T c = pa * pb;
  const T den = T(1) + c * ee;
  const T inv_den = rcp_of(den);
  const T half_logdet_m = log_of(LA.a00 * LA.a11 * LA.a22) + T(0.5) * log1p_of(c * ee);
  if (mode == NANOGS_COST_BOUND) {
    // KL(N_c || q_m) = 1/2 [tr(Sm^-1 Sc) + w_o^2 |e|^2 / den - 3] +
    // half log det Sm - log det L_c, with Sm^-1 = A^-1 - c A^-1 d d^T A^-1
    // / den (A = L_A L_A^T) and w_o the other component's weight
    const V3<T> h = tri_solve_t(LA, e);  // A^-1 d
    auto kl = [&](const Tri<T>& Lc, T ldc, T w_other) {
      const V3<T> c0 = tri_solve(LA, V3<T>{Lc.a00, Lc.a10, Lc.a20});
      const V3<T> c1 = tri_solve(LA, V3<T>{T(0), Lc.a11, Lc.a21});
      const V3<T> c2 = tri_solve(LA, V3<T>{T(0), T(0), Lc.a22});
      const T tr_a = dot(c0, c0) + dot(c1, c1) + dot(c2, c2);
      const V3<T> r = tri_mul_t(Lc, h);
      const T tr = tr_a - c * dot(r, r) * inv_den;
      return T(0.5) * (tr + w_other * w_other * ee * inv_den - T(3)) + half_logdet_m - ldc;
    };
    const T ka = pa > T(0) ? pa * kl(La, ldLa, pb) : T(0);
    const T kb = pb > T(0) ? pb * kl(Lb, ldLb, pa) : T(0);
    return ka + kb;
  }
  const T lpa = log_of(pa), lpb = log_of(pb);
  const T ne = sqrt_of(ee);
  const T inv_ne = ne > T(0) ? rcp_of(ne) : T(0);
  const V3<T> eh = {e.x * inv_ne, e.y * inv_ne, e.z * inv_ne};
  // g = log p~(x) - log q_m(x) at x = mu_c + L_c z (c = a or b)
  auto g_at = [&](bool ca, const V3<T>& zz) {
    const Tri<T>& Lc = ca ? La : Lb;
    const Tri<T>& Lo = ca ? Lb : La;
    const T ldc = ca ? ldLa : ldLb;
    const T ldo = ca ? ldLb : ldLa;
    const V3<T> t = tri_mul(Lc, zz);
    const T lnc = T(-0.5) * dot(zz, zz) - ldc;
    const T sg = ca ? T(1) : T(-1);
    const V3<T> y = {sg * d.x + t.x, sg * d.y + t.y, sg * d.z + t.z};
    const V3<T> v = tri_solve(Lo, y);
    const T lno = T(-0.5) * dot(v, v) - ldo;
    const V3<T> w = tri_solve(LA, t);
    const T beta = ca ? pb : -pa;
    const T ww = dot(w, w);
    const T we = dot(w, eh);
    const T perp = fmax(ww - we * we, T(0));
    const T par = beta * ne + we;
    const T maha = perp + par * par * inv_den;
    const T lnm = T(-0.5) * maha - half_logdet_m;
    const T la = lpa + (ca ? lnc : lno);
    const T lb = lpb + (ca ? lno : lnc);
    const T mx = fmax(la, lb), mn = fmin(la, lb);
    const T lse = mx + log1p_of(exp_of(mn - mx));
    return lse - lnm;
  };
  T acc = T(0);
  for (int s = 0; s < S; ++s) {
    const V3<T> zz = {(T)cv[4 * s + 1], (T)cv[4 * s + 2], (T)cv[4 * s + 3]};
    if (mode == NANOGS_COST_STRAT) {
      const T ga = pa > T(0) ? pa * g_at(true, zz) : T(0);
      const T gb = pb > T(0) ? pb * g_at(false, zz) : T(0);
      acc += ga + gb;
    } else {
      const float u = cv[4 * s];
      acc += g_at((double)u < pdec, zz);
    }
  }
  return S == 1 ? acc : acc * rcp_of((T)S);
}

// D_app = ||f_s - f_t||^2 for the wave's 64 edges (lane j: edge j), 16
// lanes per edge and 4 consecutive edges per step: each lane takes 3 of the
// 48 coefficients of both rows, so a load instruction reads 4 whole rows per
// side instead of 64 scattered 16-byte pieces of 64 rows.  Every lane of the
// wave must call it.  The sum runs as a fixed tree over the 16 lanes.
NG_DEV float dapp_wave(const float* __restrict__ sh, int s, int t, bool live, int app_dims) {
  const int lane = lane_id();
  const int g = lane >> 4, c0 = 3 * (lane & 15);
  float mine = 0.f;
#pragma unroll 4
  for (int r = 0; r < 16; ++r) {
    const int j = 4 * r + g;
    const int sj = __shfl(s, j, 64), tj = __shfl(t, j, 64);
    const bool lj = __shfl((int)live, j, 64) != 0;
    float acc = 0.f;
    if (lj) {
      const float* fa = sh + (long long)sj * NG_SH + c0;
      const float* fb = sh + (long long)tj * NG_SH + c0;
      if (app_dims == NG_SH) {
        const float dx = fa[0] - fb[0], dy = fa[1] - fb[1], dz = fa[2] - fb[2];
        acc = dx * dx + dy * dy + dz * dz;
      } else {
        for (int c = 0; c < 3; ++c)
          if (c0 + c < app_dims) {
            const float d = fa[c] - fb[c];
            acc += d * d;
          }
      }
    }
    acc += __shfl_xor(acc, 8, 64);
    acc += __shfl_xor(acc, 4, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 1, 64);
    const float v = __shfl(acc, 16 * (lane & 3), 64);
    if ((lane >> 2) == r) mine = v;
  }
  return mine;
}

NG_DEV double dapp_f64(const float* __restrict__ sh, long long a, long long b, int app_dims) {
  const float* fa = sh + a * NG_SH;
  const float* fb = sh + b * NG_SH;
  double acc = 0.0;
  for (int c = 0; c < app_dims; ++c) {
    const double dc = (double)fa[c] - (double)fb[c];
    acc += dc * dc;
  }
  return acc;
}

// Mass of a splat up to the common (2 pi)^{3/2} (Eq. vm_weights), in double
// from the float values: ((alpha s0) s1) s2.
NG_DEV double weight_f64(float4 sa) {
#pragma clang fp contract(off)
  return (((double)sa.w * (double)sa.x) * (double)sa.y) * (double)sa.z;
}

// Mixture weights pi = w_a / W and 1 - pi as w_b / W in double
// (Eq. norm_mixture); W = 0 gives 1/2 each.
NG_DEV void mix_weights(double wa, double wb, double& pa, double& pb) {
#pragma clang fp contract(off)
  const double W = wa + wb;
  pa = W > 0.0 ? wa / W : 0.5;
  pb = W > 0.0 ? wb / W : 0.5;
}

// ---- kernels ---------------------------------------------------------------
__global__ void k_precompute(const float4* __restrict__ shp, int n, float4* __restrict__ pre,
                             double* __restrict__ wd) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float4 a = shp[2 * (long long)p];
  wd[p] = weight_f64(a);
  const float4 q = shp[2 * (long long)p + 1];
  const Tri<double> L = chol_from_scale_rot<double>(a.x, a.y, a.z, q.x, q.y, q.z, q.w);
  const double ld = log((double)a.x) + log((double)a.y) + log((double)a.z);
  const float wt = ((a.w * a.x) * a.y) * a.z;
  pre[2 * (long long)p] = make_float4((float)L.a00, (float)L.a10, (float)L.a11, (float)L.a20);
  pre[2 * (long long)p + 1] = make_float4((float)L.a21, (float)L.a22, (float)ld, wt);
}

NG_DEV void append_wave(bool flag, int value, int* list, int* count) {
  const unsigned long long m = __ballot(flag);
  if (m == 0) return;
  const int lane = lane_id();
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(m));
  base = __shfl(base, leader, 64);
  if (flag) {
    const unsigned long long below = lane == 0 ? 0ull : (m & (~0ull >> (64 - lane)));
    list[base + __popcll(below)] = value;
  }
}

NG_DEV unsigned long long adj_key(float c, int other_logical) {
  if (!isfinite(c)) return ~0ull;
  return ((unsigned long long)f2ord(c) << 32) | (unsigned)other_logical;
}

// Writes edge e's two adjacency entries (layout in edges.hip).
NG_DEV void write_adj(const AdjOut& adj, int e, int s, int t, int ls, int lt, float c) {
  if (!adj.akey) return;
  const long long ps = (long long)adj.ioff[s] + e;
  const long long pt = (long long)adj.eoff[t + 1] + adj.ioff[t] + adj.islot[e];
  adj.akey[ps] = adj_key(c, lt);
  adj.au[ps] = t;
  adj.akey[pt] = adj_key(c, ls);
  adj.au[pt] = s;
}

__global__ void __launch_bounds__(256)
k_edge_cost(const float4* __restrict__ cen, const float4* __restrict__ pre,
            const double* __restrict__ wd, const float* __restrict__ sh, int app_dims, const int* __restrict__ ea,
            const int* __restrict__ eb, int m, int n, int orient, const float* __restrict__ crn,
            int S, int mode, const int* __restrict__ sg, const SegInfo* __restrict__ seg,
            float fb_ratio,
            float* __restrict__ cost, float* __restrict__ dgeo_out, int* __restrict__ fb_list,
            int* __restrict__ fb_count, AdjOut adj, const int* __restrict__ d_mcount) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (d_mcount) m = min(m, *d_mcount);
  bool live = e < m;
  bool fb = false;
  int s = 0, t = 0;
  if (live) {
    s = ea[e];
    t = eb[e];
    if (s < 0 || s >= n || t < 0 || t >= n) {
      cost[e] = __int_as_float(0x7fc00000);
      if (dgeo_out) dgeo_out[e] = __int_as_float(0x7fc00000);
      live = false;
    }
  }
  // every per-endpoint load issues before the first use: both ends' factors
  // come in before the orientation (which needs the centres) picks them
  float4 cs{}, ct{}, ps0{}, ps1{}, pt0{}, pt1{};
  double ws = 0.0, wt = 0.0;
  int crow = 0;
  if (live) {
    cs = cen[s];
    ct = cen[t];
    ps0 = pre[2 * (long long)s];
    ps1 = pre[2 * (long long)s + 1];
    pt0 = pre[2 * (long long)t];
    pt1 = pre[2 * (long long)t + 1];
    ws = wd[s];
    wt = wd[t];
    crow = sg ? seg[sg[s]].crn : 0;
  }
  // whole waves past the end skip the cooperative part
  const bool wave_live = __ballot(live) != 0ull;
  const float dapp = wave_live ? dapp_wave(sh, s, t, live, app_dims) : 0.f;
  if (live) {
    const int ls = __float_as_int(cs.w), lt = __float_as_int(ct.w);
    const bool sw = orient && lt < ls;  // first component = smaller logical index
    const float4 ca = sw ? ct : cs, cb = sw ? cs : ct;
    const float4 pa0 = sw ? pt0 : ps0, pa1 = sw ? pt1 : ps1;
    const float4 pb0 = sw ? ps0 : pt0, pb1 = sw ? ps1 : pt1;
    const Tri<float> La = {pa0.x, pa0.y, pa0.z, pa0.w, pa1.x, pa1.y};
    const Tri<float> Lb = {pb0.x, pb0.y, pb0.z, pb0.w, pb1.x, pb1.y};
    double pad, pbd;
    mix_weights(sw ? wt : ws, sw ? ws : wt, pad, pbd);
    const float pa = (float)pad, pb = (float)pbd;
    float ratio;
    const float* cv = crn + NG_CRN_ROW * crow;
    const float dg = dgeo_pair<float>(v3(ca.x, ca.y, ca.z), v3(cb.x, cb.y, cb.z), La, Lb, pa1.z,
                                      pb1.z, pa, pb, pad, cv, S, mode, ratio);
    const float c = dg + dapp;
    fb = !(ratio >= fb_ratio) || !isfinite(c);
    cost[e] = c;
    if (dgeo_out) dgeo_out[e] = dg;
    write_adj(adj, e, s, t, ls, lt, c);
  }
  if (fb_list) append_wave(fb, e, fb_list, fb_count);
}

__global__ void __launch_bounds__(256)
k_edge_cost_fp64(const float4* __restrict__ cen, const float4* __restrict__ shp,
                 const float* __restrict__ sh, int app_dims, const int* __restrict__ ea,
                 const int* __restrict__ eb, int n, int orient, const int* __restrict__ list,
                 const int* __restrict__ d_count, int count_cap, const float* __restrict__ crn,
                 int S, int mode, const int* __restrict__ sg, const SegInfo* __restrict__ seg,
                 float* __restrict__ cost, float* __restrict__ dgeo_out, AdjOut adj) {
  const int count = d_count ? min(*d_count, count_cap) : count_cap;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const int e = list ? list[i] : i;
    const int s = ea[e], t = eb[e];
    if (s < 0 || s >= n || t < 0 || t >= n) {
      cost[e] = __int_as_float(0x7fc00000);
      if (dgeo_out) dgeo_out[e] = __int_as_float(0x7fc00000);
      continue;
    }
    const float4 cs = cen[s], ct = cen[t];
    const int ls = __float_as_int(cs.w), lt = __float_as_int(ct.w);
    const bool sw = orient && lt < ls;
    const int a = sw ? t : s, b = sw ? s : t;
    const float4 ca = sw ? ct : cs, cb = sw ? cs : ct;
    const float4 sa = shp[2 * (long long)a], qa = shp[2 * (long long)a + 1];
    const float4 sb = shp[2 * (long long)b], qb = shp[2 * (long long)b + 1];
    const Tri<double> La = chol_from_scale_rot<double>(sa.x, sa.y, sa.z, qa.x, qa.y, qa.z, qa.w);
    const Tri<double> Lb = chol_from_scale_rot<double>(sb.x, sb.y, sb.z, qb.x, qb.y, qb.z, qb.w);
    const double lda = log((double)sa.x) + log((double)sa.y) + log((double)sa.z);
    const double ldb = log((double)sb.x) + log((double)sb.y) + log((double)sb.z);
    double pa, pb;
    mix_weights(weight_f64(sa), weight_f64(sb), pa, pb);
    double ratio;
    const float* cv = crn + NG_CRN_ROW * (sg ? seg[sg[s]].crn : 0);
    const double dg = dgeo_pair<double>(v3<double>(ca.x, ca.y, ca.z), v3<double>(cb.x, cb.y, cb.z),
                                        La, Lb, lda, ldb, pa, pb, pa, cv, S, mode, ratio);
    const float c = (float)(dg + dapp_f64(sh, a, b, app_dims));
    cost[e] = c;
    if (dgeo_out) dgeo_out[e] = (float)dg;
    write_adj(adj, e, s, t, ls, lt, c);
  }
}

}  // namespace

void launch_precompute(const float4* shp, int n, float4* pre, hipStream_t st) {
  if (n <= 0) return;
  k_precompute<<<blocks_for(n, 256), 256, 0, st>>>(shp, n, pre, pre_weights(pre, n));
  NG_LAUNCH_CHECK();
}

void launch_edge_cost(const float4* cen, const float4* pre, const float* sh, int app_dims,
                      const int* ea, const int* eb, int m, int n, bool orient, const CrnTab& crn,
                      float fb_ratio, float* cost, float* dgeo, int* fb_list, int* fb_count,
                      AdjOut adj, hipStream_t st, const int* d_mcount) {
  if (m <= 0) return;
  const int bs = tuning_for(n).cost_block;
  k_edge_cost<<<blocks_for(m, bs), bs, 0, st>>>(cen, pre, pre_weights((float4*)pre, n), sh,
                                                  app_dims, ea, eb, m, n,
                                                  orient ? 1 : 0, crn.tab, crn.S, crn.mode, crn.sg,
                                                  crn.seg,
                                                  fb_ratio, cost, dgeo, fb_list, fb_count, adj,
                                                  d_mcount);
  NG_LAUNCH_CHECK();
}

void launch_edge_cost_fp64(const float4* cen, const float4* shp, const float* sh, int app_dims,
                           const int* ea, const int* eb, int n, bool orient, const int* list,
                           const int* d_count, int count_cap, const CrnTab& crn, float* cost,
                           float* dgeo, AdjOut adj, hipStream_t st) {
  if (count_cap <= 0) return;
  unsigned b = blocks_for(count_cap, 256);
  if (b > 2048) b = 2048;
  k_edge_cost_fp64<<<b, 256, 0, st>>>(cen, shp, sh, app_dims, ea, eb, n, orient ? 1 : 0, list,
                                      d_count, count_cap, crn.tab, crn.S, crn.mode, crn.sg, crn.seg,
                                      cost,
                                      dgeo, adj);
  NG_LAUNCH_CHECK();
}

}  // namespace ng
