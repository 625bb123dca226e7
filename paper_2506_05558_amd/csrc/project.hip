// Per-Gaussian EWA projection (forward) and its adjoint, including the
// camera-pose gradient reduction.
//
// One lane per Gaussian and up to eight views per launch; parameters are
// read once as SoA planes (every load of a wave is one contiguous 256-byte
// segment per plane) and held in registers across the views, each view's
// pose is a uniform 48-byte read.  Geometry runs in FP64: the render record
// needs a sub-1e-6-pixel mean and the support radii and tile counts must
// agree with an FP64 reference exactly.  On gfx950 FP64 vector FMAs issue at
// half the non-packed FP32 rate, and with the SH coefficients held as
// doubles across the views (two waves per SIMD) the 8-view projection is
// bound by FP64 issue and latency more than by its HBM traffic (236 B in
// per SH-degree-3 Gaussian, 76 B out per view).  The adjoint runs in FP32
// (hardware exp, rcp, rsqrt) with the SH terms streamed one coefficient at a
// time, which keeps its register footprint and with it occupancy up; the
// camera-pose sum over all Gaussians is reduced in FP64.
#include "common.h"

namespace gsmi {
namespace {

constexpr int kBlock = 256;

// Real SH constants: Y_00 = 1/(2 sqrt(pi)); degree 1 sqrt(3/(4 pi));
// degree 2: sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4;
// degree 3: sqrt(35/(2 pi))/4, sqrt(105/pi)/2, sqrt(21/(2 pi))/4,
// sqrt(7/pi)/4, sqrt(105/pi)/4.
constexpr double kY0 = 0.28209479177387814;
constexpr double kY1 = 0.4886025119029199;
constexpr double kY2a = 1.0925484305920792;
constexpr double kY2b = 0.31539156525252005;
constexpr double kY2c = 0.5462742152960396;
constexpr double kY3a = 0.5900435899266435;
constexpr double kY3b = 2.890611442640554;
constexpr double kY3c = 0.4570457994644658;
constexpr double kY3d = 0.3731763325901154;
constexpr double kY3e = 1.445305721320277;

// Basis function k at the unit direction (x, y, z) and its gradient with
// respect to (x, y, z) as a polynomial on R^3.  T is float or double.
template <class T>
__device__ __forceinline__ void sh_term(int k, T x, T y, T z, T &Y, T &gx, T &gy, T &gz) {
  const T xx = x * x, yy = y * y, zz = z * z;
  switch (k) {
    case 0: Y = (T)kY0; gx = gy = gz = 0; break;
    case 1: Y = -(T)kY1 * y; gx = 0; gy = -(T)kY1; gz = 0; break;
    case 2: Y = (T)kY1 * z; gx = 0; gy = 0; gz = (T)kY1; break;
    case 3: Y = -(T)kY1 * x; gx = -(T)kY1; gy = 0; gz = 0; break;
    case 4: Y = (T)kY2a * x * y; gx = (T)kY2a * y; gy = (T)kY2a * x; gz = 0; break;
    case 5: Y = -(T)kY2a * y * z; gx = 0; gy = -(T)kY2a * z; gz = -(T)kY2a * y; break;
    case 6:
      Y = (T)kY2b * (2 * zz - xx - yy); gx = -2 * (T)kY2b * x; gy = -2 * (T)kY2b * y; gz = 4 * (T)kY2b * z;
      break;
    case 7: Y = -(T)kY2a * x * z; gx = -(T)kY2a * z; gy = 0; gz = -(T)kY2a * x; break;
    case 8: Y = (T)kY2c * (xx - yy); gx = 2 * (T)kY2c * x; gy = -2 * (T)kY2c * y; gz = 0; break;
    case 9:
      Y = -(T)kY3a * y * (3 * xx - yy); gx = -6 * (T)kY3a * x * y; gy = -(T)kY3a * (3 * xx - 3 * yy); gz = 0;
      break;
    case 10:
      Y = (T)kY3b * x * y * z; gx = (T)kY3b * y * z; gy = (T)kY3b * x * z; gz = (T)kY3b * x * y;
      break;
    case 11:
      Y = -(T)kY3c * y * (4 * zz - xx - yy);
      gx = 2 * (T)kY3c * x * y; gy = -(T)kY3c * (4 * zz - xx - 3 * yy); gz = -8 * (T)kY3c * y * z;
      break;
    case 12:
      Y = (T)kY3d * z * (2 * zz - 3 * xx - 3 * yy);
      gx = -6 * (T)kY3d * x * z; gy = -6 * (T)kY3d * y * z; gz = (T)kY3d * (6 * zz - 3 * xx - 3 * yy);
      break;
    case 13:
      Y = -(T)kY3c * x * (4 * zz - xx - yy);
      gx = -(T)kY3c * (4 * zz - 3 * xx - yy); gy = 2 * (T)kY3c * x * y; gz = -8 * (T)kY3c * x * z;
      break;
    case 14:
      Y = (T)kY3e * z * (xx - yy); gx = 2 * (T)kY3e * x * z; gy = -2 * (T)kY3e * y * z; gz = (T)kY3e * (xx - yy);
      break;
    default:
      Y = -(T)kY3a * x * (xx - 3 * yy); gx = -(T)kY3a * (3 * xx - 3 * yy); gy = 6 * (T)kY3a * x * y; gz = 0;
      break;
  }
}

// One view: camera and the per-view buffers of the forward (written) and of
// the adjoint (read).
struct ViewArgs {
  const float *pose;  // [12] R row-major, t
  float fx, fy, cx, cy, near_plane;
  int W, H;
  float *rec;
  int32_t *radius, *tiles;     // radius: [2][n] (rx, ry)
  uint32_t *bin;               // [n][4] binning inputs of visible Gaussians, or NULL
  const float *pair_grad;      // [M][12] 2D gradients per (Gaussian, tile) pair (first 10 used)
  const uint32_t *first_slot;  // first pair slot of each visible Gaussian
  double *d_pose, *d_twist;    // pose-gradient outputs (accumulated), may be NULL
};

// The views of one launch share the Gaussians: their parameters are read
// once per Gaussian and its gradients written once, whatever the number of
// views, which is what bounds both kernels (HBM traffic per Gaussian).
constexpr int kMaxViews = 8;

// The sparse Adam step that the last SH pass of the adjoint applies (section
// 4.3): parameter planes and both moments updated in place, one rate per
// group, the per-Gaussian rate (NULL: 1) and its decay after the step.
struct AdamArgs {
  float *p[5], *m1[5], *m2[5];  // means, log_scales, quats, opacity_logits, sh
  float *rate;
  float lr[6];  // means, log_scales, quats, opacity, sh degree 0, sh degree >= 1
  float b1, b2, eps, c1, c2, decay;
};

struct MultiArgs {
  int64_t n;
  int nv;
  float eps2d, alpha_min, guard;
  int mip;    // eps2d is a screen-space filter whose opacity compensation applies
  int store;  // the adjoint stores (=) every Gaussian's gradients instead of adding them
  int adam;   // the SH pass applies the sparse Adam step (opt) instead of storing
  const float *means, *log_scales, *quats, *opac, *sh;
  const float *f3;                 // [n] 3D smoothing-filter variance per Gaussian, or NULL
  float *gm, *gl, *gq, *go, *gsh;  // parameter gradients (accumulated)
  double *partials;                // [nv][gridDim.x][12] pose partial sums
  float *gc;                       // [nv][3][n] clamped colour gradient per view (adjoint workspace)
  int32_t *visible;                // [n] or NULL: 1 where some view's tile count is positive
  int visible_or;                  // OR into visible (later batches of views) instead of writing it
  AdamArgs opt;                    // read by the SH pass's Adam form only
  ViewArgs v[kMaxViews];
};

// One Gaussian's parameters, loaded once for all views.
template <int DEG>
struct GParams {
  static constexpr int NB = (DEG + 1) * (DEG + 1);
  float mu[3], q[4], ls[3], logit, f3;  // f3: 3D smoothing-filter variance (0: none)
  float sh[NB * 3];                     // [k][channel]
};

template <int DEG, bool SH = true>
__device__ __forceinline__ void load_params(const MultiArgs &m, int64_t i, GParams<DEG> &P) {
  const int64_t n = m.n;
#pragma unroll
  for (int k = 0; k < 3; ++k) P.mu[k] = m.means[k * n + i];
#pragma unroll
  for (int k = 0; k < 4; ++k) P.q[k] = m.quats[k * n + i];
#pragma unroll
  for (int k = 0; k < 3; ++k) P.ls[k] = m.log_scales[k * n + i];
  P.logit = m.opac[i];
  P.f3 = m.f3 ? m.f3[i] : 0.0f;
  if (SH) {
#pragma unroll
    for (int k = 0; k < GParams<DEG>::NB * 3; ++k) P.sh[k] = m.sh[(int64_t)k * n + i];
  }
}

// Geometry of one Gaussian in one view: FP64 for the forward projection
// (the render record needs a sub-1e-6-pixel mean), FP32 for the adjoint,
// whose 2D covariance is kept well conditioned by the eps2d dilation.
template <class Real>
struct Geo {
  Real R[9], t[3];
  Real p[3], iz;
  bool clx, cly;
  Real J00, J02, J11, J12;
  Real qn[4], qinv;
  Real Rq[9], s[3], M[9];
  Real s0[3], ofac;  // unfiltered scales; opacity factor prod s0 / s of the 3D filter
  Real T[6], TM[6];
  Real a, b, c, A, B, C;
};

__device__ __forceinline__ double real_exp(double x) { return exp(x); }
__device__ __forceinline__ float real_exp(float x) { return __expf(x); }
__device__ __forceinline__ double real_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float real_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double real_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float real_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double real_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float real_sqrt(float x) { return __builtin_sqrtf(x); }

// Camera-space point and the 2D covariance.  Returns false if culled by
// the near plane or a non-positive determinant.
template <class Real, int DEG>
__device__ __forceinline__ bool geometry(const MultiArgs &m, const ViewArgs &v, const GParams<DEG> &P,
                                         Geo<Real> &f) {
#pragma unroll
  for (int k = 0; k < 9; ++k) f.R[k] = (Real)v.pose[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) f.t[k] = (Real)v.pose[9 + k];
  const Real mu[3] = {(Real)P.mu[0], (Real)P.mu[1], (Real)P.mu[2]};
#pragma unroll
  for (int r = 0; r < 3; ++r)
    f.p[r] = f.R[3 * r] * mu[0] + f.R[3 * r + 1] * mu[1] + f.R[3 * r + 2] * mu[2] + f.t[r];
  if (!(f.p[2] > (Real)v.near_plane)) return false;
  f.iz = real_rcp(f.p[2]);
  const Real limx = (Real)(m.guard * 0.5 * v.W / v.fx), limy = (Real)(m.guard * 0.5 * v.H / v.fy);
  const Real tx = f.p[0] * f.iz, ty = f.p[1] * f.iz;
  f.clx = tx < -limx || tx > limx;
  f.cly = ty < -limy || ty > limy;
  const Real xc = f.clx ? (tx < 0 ? -limx : limx) * f.p[2] : f.p[0];
  const Real yc = f.cly ? (ty < 0 ? -limy : limy) * f.p[2] : f.p[1];
  const Real fx = (Real)v.fx, fy = (Real)v.fy;
  f.J00 = fx * f.iz;
  f.J11 = fy * f.iz;
  f.J02 = -fx * xc * f.iz * f.iz;
  f.J12 = -fy * yc * f.iz * f.iz;

  const Real q0 = P.q[0], q1 = P.q[1], q2 = P.q[2], q3 = P.q[3];
  f.qinv = real_rsqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const Real w = q0 * f.qinv, x = q1 * f.qinv, y = q2 * f.qinv, z = q3 * f.qinv;
  f.qn[0] = w; f.qn[1] = x; f.qn[2] = y; f.qn[3] = z;
  f.Rq[0] = 1 - 2 * (y * y + z * z);
  f.Rq[1] = 2 * (x * y - w * z);
  f.Rq[2] = 2 * (x * z + w * y);
  f.Rq[3] = 2 * (x * y + w * z);
  f.Rq[4] = 1 - 2 * (x * x + z * z);
  f.Rq[5] = 2 * (y * z - w * x);
  f.Rq[6] = 2 * (x * z - w * y);
  f.Rq[7] = 2 * (y * z + w * x);
  f.Rq[8] = 1 - 2 * (x * x + y * y);
#pragma unroll
  for (int k = 0; k < 3; ++k) f.s0[k] = f.s[k] = real_exp((Real)P.ls[k]);
  // 3D smoothing filter: the Gaussian convolved with an isotropic low-pass of
  // variance f3 has axis variances s^2 + f3 in the same rotation, and its
  // opacity is scaled by prod s0 / s so that its integral is unchanged
  f.ofac = (Real)1;
  if (P.f3 > 0.0f) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      f.s[k] = real_sqrt(f.s0[k] * f.s0[k] + (Real)P.f3);
      f.ofac *= f.s0[k] / f.s[k];
    }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) f.M[3 * r + c] = f.Rq[3 * r + c] * f.s[c];
  // Sigma2 = (J R M)(J R M)^T + eps I, with J R formed first (2x3)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    f.T[c] = f.J00 * f.R[c] + f.J02 * f.R[6 + c];
    f.T[3 + c] = f.J11 * f.R[3 + c] + f.J12 * f.R[6 + c];
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      f.TM[3 * r + c] = f.T[3 * r] * f.M[c] + f.T[3 * r + 1] * f.M[3 + c] + f.T[3 * r + 2] * f.M[6 + c];
  f.a = f.TM[0] * f.TM[0] + f.TM[1] * f.TM[1] + f.TM[2] * f.TM[2] + (Real)m.eps2d;
  f.b = f.TM[0] * f.TM[3] + f.TM[1] * f.TM[4] + f.TM[2] * f.TM[5];
  f.c = f.TM[3] * f.TM[3] + f.TM[4] * f.TM[4] + f.TM[5] * f.TM[5] + (Real)m.eps2d;
  const Real det = f.a * f.c - f.b * f.b;
  if (!(det > 0)) return false;
  const Real idet = real_rcp(det);
  f.A = f.c * idet;
  f.B = -f.b * idet;
  f.C = f.a * idet;
  return true;
}


// Opacity compensation of the screen-space filter: rho = sqrt(det0 / det)
// with det0 the determinant of the unfiltered 2D covariance TM TM^T and
// det that of the filtered one.  det0 is the sum of the squared 2x2 minors
// of TM (Cauchy-Binet: never negative, no cancellation between a0 c0 and
// b^2 for thin splats); det = det0 + eps (a0 + c0) + eps^2.
template <class Real>
__device__ __forceinline__ Real mip_rho(const Geo<Real> &f, Real eps, Real &det0, Real &det) {
  const Real m01 = f.TM[0] * f.TM[4] - f.TM[1] * f.TM[3];
  const Real m02 = f.TM[0] * f.TM[5] - f.TM[2] * f.TM[3];
  const Real m12 = f.TM[1] * f.TM[5] - f.TM[2] * f.TM[4];
  det0 = m01 * m01 + m02 * m02 + m12 * m12;
  det = det0 + eps * (f.a + f.c - eps);  // a0 + c0 + eps = a + c - eps
  return real_sqrt(det0 / det);
}

// Unit view direction from the camera centre C = -R^T t and 1/|mu - C|.
template <class Real>
__device__ __forceinline__ void view_dir(const Real R[9], const Real t[3], const Real mu[3], Real d[3], Real &dinv) {
  const Real Cx = -(R[0] * t[0] + R[3] * t[1] + R[6] * t[2]);
  const Real Cy = -(R[1] * t[0] + R[4] * t[1] + R[7] * t[2]);
  const Real Cz = -(R[2] * t[0] + R[5] * t[1] + R[8] * t[2]);
  const Real dx = mu[0] - Cx, dy = mu[1] - Cy, dz = mu[2] - Cz;
  dinv = real_rsqrt(dx * dx + dy * dy + dz * dz);
  d[0] = dx * dinv;
  d[1] = dy * dinv;
  d[2] = dz * dinv;
}

// Forward of Gaussian i in view v: render record, support half-widths, tiles.
template <int DEG>
__device__ __forceinline__ void project_one(const MultiArgs &m, const ViewArgs &v, int64_t i,
                                            const GParams<DEG> &P) {
  const int64_t n = m.n;
  Geo<double> f;
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0, r3 = r0;
  int rx = 0, ry = 0, tiles = 0;
  // a projection that is not finite (NaN or infinite parameters, or an
  // inverse 2D covariance that overflows) is culled
  bool ok = geometry<double, DEG>(m, v, P, f) && isfinite(f.p[0]) && isfinite(f.p[1]) && isfinite(f.p[2]) &&
            isfinite(f.a) && isfinite(f.b) && isfinite(f.c) && isfinite(f.A) && isfinite(f.B) && isfinite(f.C);
  double mx = 0, my = 0, o = 0;
  if (ok) {
    mx = (double)v.fx * f.p[0] * f.iz + (double)v.cx;
    my = (double)v.fy * f.p[1] * f.iz + (double)v.cy;
    ok = fabs(mx) < 8388608.0 && fabs(my) < 8388608.0;  // |mean| < 2^23 px
  }
  if (ok) {
    o = f.ofac / (1.0 + exp(-(double)P.logit));
    if (m.mip) {
      double det0, det;
      o *= mip_rho<double>(f, (double)m.eps2d, det0, det);
    }
    ok = o >= (double)m.alpha_min;  // false for a NaN opacity
  }
  if (ok) {
    // support: o exp(-q/2) >= alpha_min  <=>  q = d^T Sigma2^-1 d <= qmax;
    // its bounding box has half-extents sqrt(qmax a), sqrt(qmax c)
    const double qmax = 2.0 * log(o / (double)m.alpha_min);
    const double hx = sqrt(qmax * f.a), hy = sqrt(qmax * f.c);
    rx = (int)ceil(fmin(hx * (1.0 + 1e-4) + 1e-3, 4194304.0));
    ry = (int)ceil(fmin(hy * (1.0 + 1e-4) + 1e-3, 4194304.0));
    const double mu[3] = {P.mu[0], P.mu[1], P.mu[2]};
    double d[3], dinv;
    view_dir<double>(f.R, f.t, mu, d, dinv);
    double val[3] = {0.5, 0.5, 0.5};
#pragma unroll
    for (int k = 0; k < GParams<DEG>::NB; ++k) {
      double Y, gx, gy, gz;
      sh_term<double>(k, d[0], d[1], d[2], Y, gx, gy, gz);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) val[ch] += (double)P.sh[k * 3 + ch] * Y;
    }
    const double hxm = rint(mx), hym = rint(my);
    r0 = make_float4((float)hxm, (float)hym, (float)(mx - hxm), (float)(my - hym));
    r1 = make_float4((float)f.A, (float)f.B, (float)f.C, (float)o);
    r2 = make_float4((float)fmax(val[0], 0.0), (float)fmax(val[1], 0.0), (float)fmax(val[2], 0.0), (float)f.p[2]);
    r3 = make_float4((float)hx, (float)hy, 0.f, 0.f);
    int tx0, ty0, tx1, ty1;
    if (tile_rect(__fadd_rn(r0.x, r0.z), __fadd_rn(r0.y, r0.w), rx, ry, v.W, v.H, tx0, ty0, tx1, ty1)) {
      tiles = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
      if (v.bin)
        *(uint4 *)(v.bin + 4 * i) = make_uint4(__float_as_uint(r2.w), (uint32_t)tx0 | (uint32_t)ty0 << 16,
                                               (uint32_t)tx1 | (uint32_t)ty1 << 16, 0u);
    }
  }
  float4 *dst = (float4 *)(v.rec + i * GS_REC_FLOATS);
  dst[0] = r0;
  dst[1] = r1;
  dst[2] = r2;
  dst[3] = r3;
  v.radius[i] = rx;
  v.radius[n + i] = ry;
  v.tiles[i] = tiles;
}

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project_views(MultiArgs m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= m.n) return;
  GParams<DEG> P;
  load_params<DEG>(m, i, P);
  // the filters only scale the opacity down (prod s0 / s <= 1, rho <= 1): a
  // Gaussian whose sigmoid opacity is already below alpha_min is culled in
  // every view, with the outputs the full test would give -- the per-view
  // FP64 geometry is skipped (freed pool slots hold such logits)
  if (1.0 / (1.0 + exp(-(double)P.logit)) < (double)m.alpha_min) {
    for (int v = 0; v < m.nv; ++v) {
      const ViewArgs &w = m.v[v];
      float4 *dst = (float4 *)(w.rec + i * GS_REC_FLOATS);
      const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
      dst[0] = z;
      dst[1] = z;
      dst[2] = z;
      dst[3] = z;
      w.radius[i] = 0;
      w.radius[m.n + i] = 0;
      w.tiles[i] = 0;
    }
    return;
  }
  for (int v = 0; v < m.nv; ++v) project_one<DEG>(m, m.v[v], i, P);
}

// ---------------------------------------------------------------- backward
// Gradient accumulators of one Gaussian over the views of a launch.
struct GAcc {
  float gm[3], gl[3], gq[4], go;
};

// Adjoint of Gaussian i in one view where it is visible, in FP32 (the
// forward decided visibility; the adjoint only chains gradients), from the
// summed 2D gradients g0..g2 (whose colour terms are already 0 for a channel
// the projection clamped at 0).
// Adds the geometry and opacity gradients to acc, writes this Gaussian's
// pose terms into pose[12] (dL/dR row-major, dL/dt) and its clamped colour
// gradient into gc[3], which the SH pass chains to the SH coefficients and
// the view direction.
template <int DEG>
__device__ __forceinline__ void backward_view(const MultiArgs &m, const ViewArgs &v, int64_t i, const float4 &g0,
                                              const float4 &g1, const float4 &g2, const GParams<DEG> &P, GAcc &acc,
                                              float pose[12], float gc[3]) {
  Geo<float> f;
  geometry<float, DEG>(m, v, P, f);
  const float mu[3] = {P.mu[0], P.mu[1], P.mu[2]};
  // g0 = (d mean x, d mean y, dA, dB), g1 = (dC, d opacity, d r, d g), g2 = (d b, d z, -, -):
  // the sums of the Gaussian's per-pair 2D gradients

  // colour: the pair gradients carry 0 for a channel the projection clamped at 0
  gc[0] = g1.z;
  gc[1] = g1.w;
  gc[2] = g2.x;

  // opacity o = sigmoid(logit) ofac rho (ofac = 1 without the 3D filter, rho = 1
  // without the screen-space filter)
  const float osig = real_rcp(1.0f + __expf(-P.logit));
  float rho = 1.0f, det0 = 0.f, detf = 1.f;
  if (m.mip) rho = mip_rho<float>(f, m.eps2d, det0, detf);
  acc.go += g1.y * rho * f.ofac * osig * (1.0f - osig);
  if (P.f3 > 0.0f) {
    // ofac = prod s0 / s: d ln ofac / d ln s0_k = 1 - s0_k^2 / s_k^2
    const float od = g1.y * rho * f.ofac * osig;
#pragma unroll
    for (int k = 0; k < 3; ++k) acc.gl[k] += od * (1.0f - (f.s0[k] * f.s0[k]) / (f.s[k] * f.s[k]));
  }

  // conic -> Sigma2: dL/dSigma2 = -Q G Q with G = [[gA, gB/2], [gB/2, gC]]
  const float gA = g0.z, hB = 0.5f * g0.w, gC = g1.x;
  const float QG00 = f.A * gA + f.B * hB, QG01 = f.A * hB + f.B * gC;
  const float QG10 = f.B * gA + f.C * hB, QG11 = f.B * hB + f.C * gC;
  float S00 = -(QG00 * f.A + QG01 * f.B);
  float S01 = -(QG00 * f.B + QG01 * f.C);
  float S11 = -(QG10 * f.B + QG11 * f.C);
  if (m.mip && det0 > 0.f) {
    // rho through the unfiltered covariance (a0, b, c0): d rho = rho / 2 d(ln det0 - ln det),
    // with d ln det0 = (c0, -2 b, a0) / det0 and d ln det = (c, -2 b, a) / det; the
    // off-diagonal b sits in two entries of the full-matrix gradient
    const float k = 0.5f * g1.y * osig * f.ofac * rho, i0 = real_rcp(det0), i1 = real_rcp(detf);
    const float a0 = f.a - m.eps2d, c0 = f.c - m.eps2d;
    S00 += k * (c0 * i0 - f.c * i1);
    S11 += k * (a0 * i0 - f.a * i1);
    S01 += k * f.b * (i1 - i0);
  }

  // Sigma2 = TM TM^T: gTM = 2 S TM
  float gTM[6];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    gTM[c] = 2.0f * (S00 * f.TM[c] + S01 * f.TM[3 + c]);
    gTM[3 + c] = 2.0f * (S01 * f.TM[c] + S11 * f.TM[3 + c]);
  }
  // TM = T M: gT = gTM M^T
  float gT[6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      gT[3 * r + c] = gTM[3 * r] * f.M[3 * c] + gTM[3 * r + 1] * f.M[3 * c + 1] + gTM[3 * r + 2] * f.M[3 * c + 2];

  // M = Rq diag(s), gM = T^T gTM entry by entry: scales and quaternion
  float gRq[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float gs = 0.f;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float gM = f.T[r] * gTM[c] + f.T[3 + r] * gTM[3 + c];
      gRq[3 * r + c] = gM * f.s[c];
      gs += gM * f.Rq[3 * r + c];
    }
    // d s / d log s0 = s0^2 / s (= s without the 3D filter)
    acc.gl[c] += gs * (P.f3 > 0.0f ? f.s0[c] * f.s0[c] / f.s[c] : f.s[c]);
  }
  {
    const float w = f.qn[0], x = f.qn[1], y = f.qn[2], z = f.qn[3];
    const float G0 = gRq[0], G1 = gRq[1], G2 = gRq[2], G3 = gRq[3], G4 = gRq[4], G5 = gRq[5], G6 = gRq[6],
                G7 = gRq[7], G8 = gRq[8];
    const float dw = 2.0f * (z * (G3 - G1) + y * (G2 - G6) + x * (G7 - G5));
    const float dx = 2.0f * (y * (G1 + G3) + z * (G2 + G6) + w * (G7 - G5)) - 4.0f * x * (G4 + G8);
    const float dy = 2.0f * (x * (G1 + G3) + w * (G2 - G6) + z * (G5 + G7)) - 4.0f * y * (G0 + G8);
    const float dz = 2.0f * (w * (G3 - G1) + x * (G2 + G6) + y * (G5 + G7)) - 4.0f * z * (G0 + G4);
    const float proj = dw * w + dx * x + dy * y + dz * z;
    acc.gq[0] += (dw - proj * w) * f.qinv;
    acc.gq[1] += (dx - proj * x) * f.qinv;
    acc.gq[2] += (dy - proj * y) * f.qinv;
    acc.gq[3] += (dz - proj * z) * f.qinv;
  }

  // T = J R: gJ = gT R^T (entries 00, 02, 11, 12); gR from the covariance = J^T gT
  const float gJ00 = gT[0] * f.R[0] + gT[1] * f.R[1] + gT[2] * f.R[2];
  const float gJ02 = gT[0] * f.R[6] + gT[1] * f.R[7] + gT[2] * f.R[8];
  const float gJ11 = gT[3] * f.R[3] + gT[4] * f.R[4] + gT[5] * f.R[5];
  const float gJ12 = gT[3] * f.R[6] + gT[4] * f.R[7] + gT[5] * f.R[8];

  // camera-space point: mean2d, depth and the Jacobian entries
  const float fx = v.fx, fy = v.fy;
  const float gmx = g0.x, gmy = g0.y;
  const float iz2 = f.iz * f.iz;
  float gp0 = gmx * fx * f.iz;
  float gp1 = gmy * fy * f.iz;
  float gp2 = g2.y - (gmx * fx * f.p[0] + gmy * fy * f.p[1]) * iz2 - (gJ00 * fx + gJ11 * fy) * iz2;
  if (f.clx) {
    gp2 -= gJ02 * f.J02 * f.iz;
  } else {
    gp0 -= gJ02 * fx * iz2;
    gp2 += gJ02 * 2.0f * fx * f.p[0] * iz2 * f.iz;
  }
  if (f.cly) {
    gp2 -= gJ12 * f.J12 * f.iz;
  } else {
    gp1 -= gJ12 * fy * iz2;
    gp2 += gJ12 * 2.0f * fy * f.p[1] * iz2 * f.iz;
  }

  // p = R mu + t
  acc.gm[0] += f.R[0] * gp0 + f.R[3] * gp1 + f.R[6] * gp2;
  acc.gm[1] += f.R[1] * gp0 + f.R[4] * gp1 + f.R[7] * gp2;
  acc.gm[2] += f.R[2] * gp0 + f.R[5] * gp1 + f.R[8] * gp2;

  // pose: dL/dR = J^T gT (covariance) + gp mu^T; dL/dt = gp
  const float gp[3] = {gp0, gp1, gp2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    pose[c] = f.J00 * gT[c] + gp0 * mu[c];
    pose[3 + c] = f.J11 * gT[3 + c] + gp1 * mu[c];
    pose[6 + c] = f.J02 * gT[c] + f.J12 * gT[3 + c] + gp2 * mu[c];
    pose[9 + c] = gp[c];
  }
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Sums of the per-pair 2D gradients of each lane's Gaussian in one view.
// Slots are numbered in Gaussian index order, so the pairs of a wave's
// Gaussians form one contiguous range: the wave reads it 64 pairs at a time
// with coalesced loads, stages them in LDS, and each lane adds up its own
// pairs from there in slot order.  (A Gaussian without a first slot did not
// fit the lists; since slots ascend with the index, neither did any later
// one, so the lanes that take part own consecutive ranges.)
__device__ __forceinline__ void pair_sums(const float *pair_grad, uint32_t fs, int nt, float4 (*stage)[64],
                                          float4 &g0, float4 &g1, float4 &g2) {
  const int lane = threadIdx.x & 63;
  g0 = make_float4(0.f, 0.f, 0.f, 0.f);
  g1 = g0;
  g2 = g0;
  const uint64_t act = ballot(nt > 0);
  if (act == 0) return;
  const int first = __builtin_ctzll(act), last = 63 - __builtin_clzll(act);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)fs, first);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(fs + (uint32_t)nt), last);
  const uint32_t e = fs + (uint32_t)(nt > 0 ? nt : 0);
  for (uint32_t base = lo; base < hi; base += 64) {
    const uint32_t q = base + (uint32_t)lane;
    if (q < hi) {
      const float4 *src = (const float4 *)(pair_grad + (size_t)q * 12);
      stage[0][lane] = src[0];
      stage[1][lane] = src[1];
      stage[2][lane] = src[2];
    }
    wave_lds_fence();
    if (nt > 0) {
      const uint32_t j0 = max(fs, base), j1 = min(e, base + 64u);
      for (uint32_t j = j0; j < j1; ++j) {
        const float4 a0 = stage[0][j - base], a1 = stage[1][j - base], a2 = stage[2][j - base];
        g0.x += a0.x; g0.y += a0.y; g0.z += a0.z; g0.w += a0.w;
        g1.x += a1.x; g1.y += a1.y; g1.z += a1.z; g1.w += a1.w;
        g2.x += a2.x; g2.y += a2.y;
      }
    }
    wave_lds_fence();
  }
}

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project_bwd_views(MultiArgs m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < m.n;
  GParams<DEG> P;
  GAcc acc;
  if (valid) load_params<DEG, false>(m, i, P);
#pragma unroll
  for (int k = 0; k < 3; ++k) acc.gm[k] = acc.gl[k] = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) acc.gq[k] = 0.f;
  acc.go = 0.f;
  bool any = false;
  __shared__ float4 stage[kBlock / 64][3][64];
  __shared__ float tb[12][kBlock];
  const int t = threadIdx.x, wv = t >> 6;
  // each view's first slot and tile count are loaded one view ahead, so their
  // latency overlaps work
  uint32_t fs_next = valid && m.nv > 0 ? m.v[0].first_slot[i] : 0xffffffffu;
  int t_next = valid && m.nv > 0 ? m.v[0].tiles[i] : 0;
  bool seen = false;  // some view's tile count is positive (the sparse step's set)
  for (int vi = 0; vi < m.nv; ++vi) {
    const ViewArgs &v = m.v[vi];
    float term[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) term[k] = 0.f;
    // no first slot: the pairs did not fit the lists (see gs_bin_sort_async)
    const uint32_t fs = fs_next;
    const int nt = fs != 0xffffffffu ? t_next : 0;
    seen = seen || t_next > 0;
    if (vi + 1 < m.nv) {
      fs_next = valid ? m.v[vi + 1].first_slot[i] : 0xffffffffu;
      t_next = valid ? m.v[vi + 1].tiles[i] : 0;
    }
    float4 g0, g1, g2;
    pair_sums(v.pair_grad, fs, nt, stage[wv], g0, g1, g2);
    float gc[3] = {0.f, 0.f, 0.f};
    if (nt > 0) {
      backward_view<DEG>(m, v, i, g0, g1, g2, P, acc, term, gc);
      any = true;
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < 3; ++c) m.gc[(int64_t)(vi * 3 + c) * m.n + i] = gc[c];
    }
    // block reduction of this view's 12 pose partials in a fixed order
    // (deterministic): transposed through LDS, 16 lanes per component each
    // add 16 terms in FP64, then a 16-lane tree
    double* part = m.partials + ((int64_t)vi * gridDim.x + blockIdx.x) * 12;
    if (__syncthreads_or(nt > 0)) {
#pragma unroll
      for (int k = 0; k < 12; ++k) tb[k][t] = term[k];
      __syncthreads();
      if (t < 192) {
        const int c = t >> 4, seg = t & 15;
        double x = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) x += (double)tb[c][seg * 16 + k];
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) x += __shfl_down(x, off, 16);
        if (seg == 0) part[c] = x;
      }
      __syncthreads();
    } else if (t < 12) {
      part[t] = 0.0;
    }
  }
  if (valid && m.visible) {
    if (!m.visible_or) m.visible[i] = seen ? 1 : 0;
    else if (seen) m.visible[i] = 1;
  }
  if (!valid || (!any && !m.store)) return;
  // with the Adam step in this launch's last pass, a Gaussian no view saw is
  // left as it is and nothing reads its gradients: no zeros are stored
  if (m.adam && !seen) return;
  const int64_t n = m.n;
  if (m.store) {  // zero where no view saw the Gaussian
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      m.gm[k * n + i] = acc.gm[k];
      m.gl[k * n + i] = acc.gl[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) m.gq[k * n + i] = acc.gq[k];
    m.go[i] = acc.go;
    return;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    m.gm[k * n + i] += acc.gm[k];
    m.gl[k * n + i] += acc.gl[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) m.gq[k * n + i] += acc.gq[k];
  m.go[i] += acc.go;
}

// The Adam step on the SH planes of Gaussian i, six planes at a time with
// every load of a batch issued before its first update (the moment stores of
// one plane would otherwise hold back the next plane's loads: the compiler
// cannot prove they do not alias).  STORE: the gradient is this pass's sum
// (first batch of views); otherwise the earlier batches' stored sum plus it
// (plus nothing if no view of this batch reached the colour).
template <int DEG, bool STORE>
__device__ __forceinline__ void adam_sh(const MultiArgs &m, int64_t i, const float sh[], const float gsh[], bool any,
                                        float lr_dc, float lr_rest) {
  constexpr int NSH = GParams<DEG>::NB * 3, kBatch = 6;
  const AdamArgs &a = m.opt;
  const int64_t n = m.n;
#pragma unroll
  for (int k0 = 0; k0 < NSH; k0 += kBatch) {
    float g[kBatch], p[kBatch], m1[kBatch], m2[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int k = k0 + j;
      if (k >= NSH) break;
      const int64_t e = (int64_t)k * n + i;
      m1[j] = __builtin_nontemporal_load(a.m1[4] + e);
      m2[j] = __builtin_nontemporal_load(a.m2[4] + e);
      if (STORE) {
        g[j] = gsh[k];
      } else {
        const float prev = m.gsh[e];
        g[j] = any ? prev + gsh[k] : prev;
      }
      p[j] = DEG > 0 ? sh[k] : m.sh[e];
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int k = k0 + j;
      if (k >= NSH) break;
      const int64_t e = (int64_t)k * n + i;
      adam_one(g[j], m1[j], m2[j], p[j], k < 3 ? lr_dc : lr_rest, a.b1, a.b2, a.eps, a.c1, a.c2);
      __builtin_nontemporal_store(m1[j], a.m1[4] + e);
      __builtin_nontemporal_store(m2[j], a.m2[4] + e);
      __builtin_nontemporal_store(p[j], a.p[4] + e);
    }
  }
}

// Adam on Gaussian i (visible): the SH planes while their values are still
// in registers (adam_sh), then the eleven geometry planes, all their loads
// issued together.  The gradient of each plane is the value the store form
// leaves there: the geometry pass's stored sum, plus this pass's
// view-direction part for the means.  The rate is read before the step and
// decayed after it, as gs_lr_decay after gs_adam_step.
template <int DEG>
__device__ __forceinline__ void adam_gaussian(const MultiArgs &m, int64_t i, const float mu[3], const float sh[],
                                              const float gm[3], const float gsh[], bool any) {
  const AdamArgs &a = m.opt;
  const int64_t n = m.n;
  const float rate = a.rate ? a.rate[i] : 1.f;
  const auto lr_of = [&](int group) { return a.rate ? a.lr[group] * rate : a.lr[group]; };
  if (m.store) adam_sh<DEG, true>(m, i, sh, gsh, any, lr_of(4), lr_of(5));
  else adam_sh<DEG, false>(m, i, sh, gsh, any, lr_of(4), lr_of(5));
  // geometry planes: means 0..2, log-scales 3..5, quaternion 6..9, opacity 10
  constexpr int kArr[11] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 2, 3};
  constexpr int kRow[11] = {0, 1, 2, 0, 1, 2, 0, 1, 2, 3, 0};
  const float *const grad[4] = {m.gm, m.gl, m.gq, m.go};
  const float *const par[4] = {m.means, m.log_scales, m.quats, m.opac};
  float g[11], p[11], m1[11], m2[11];
#pragma unroll
  for (int j = 0; j < 11; ++j) {
    const int64_t e = kRow[j] * n + i;
    m1[j] = __builtin_nontemporal_load(a.m1[kArr[j]] + e);
    m2[j] = __builtin_nontemporal_load(a.m2[kArr[j]] + e);
    g[j] = grad[kArr[j]][e];
    p[j] = j < 3 ? mu[j] : par[kArr[j]][e];
  }
  if (DEG > 0 && any) {
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] += gm[k];
  }
  const float lr[4] = {lr_of(0), lr_of(1), lr_of(2), lr_of(3)};
#pragma unroll
  for (int j = 0; j < 11; ++j) {
    const int64_t e = kRow[j] * n + i;
    adam_one(g[j], m1[j], m2[j], p[j], lr[kArr[j]], a.b1, a.b2, a.eps, a.c1, a.c2);
    __builtin_nontemporal_store(m1[j], a.m1[kArr[j]] + e);
    __builtin_nontemporal_store(m2[j], a.m2[kArr[j]] + e);
    __builtin_nontemporal_store(p[j], a.p[kArr[j]] + e);
  }
  if (a.rate) a.rate[i] = rate * a.decay;
}

// The SH part of the projection adjoint, a pass of its own so that the SH
// coefficients and their gradients (96 registers at degree 3) do not share
// a lane with the geometry adjoint: per Gaussian and view, from the clamped
// colour gradient gc of the geometry pass, dL/d sh_k += gc Y_k(d) and the
// view-direction part of the mean gradient (the view direction carries no
// pose gradient, section 4.3).  Runs after k_project_bwd_views on the same
// views.
//
// ADAM: the last pass of a window whose step follows at once -- instead of
// storing the gradients it applies the sparse Adam step (adam_gaussian) to
// the Gaussians in visible, which this launch's geometry pass wrote.
template <int DEG, bool ADAM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_project_bwd_sh(MultiArgs m) {
  constexpr int NB = GParams<DEG>::NB;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= m.n) return;
  // the step leaves a Gaussian outside the visible set as it is, and nothing
  // else reads its gradients: skip it before its loads
  if (ADAM && !m.visible[i]) return;
  const int64_t n = m.n;
  float mu[3], sh[NB * 3], gsh[NB * 3], gm[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 3; ++k) mu[k] = m.means[k * n + i];
#pragma unroll
  for (int k = 0; k < NB * 3; ++k) {
    sh[k] = DEG > 0 ? m.sh[(int64_t)k * n + i] : 0.f;
    gsh[k] = 0.f;
  }
  bool any = false;
  // the colour gradients are loaded one view ahead
  float n0 = m.gc[i], n1 = m.gc[n + i], n2 = m.gc[2 * n + i];
  for (int vi = 0; vi < m.nv; ++vi) {
    const float gc0 = n0, gc1 = n1, gc2 = n2;
    if (vi + 1 < m.nv) {
      n0 = m.gc[(int64_t)(vi * 3 + 3) * n + i];
      n1 = m.gc[(int64_t)(vi * 3 + 4) * n + i];
      n2 = m.gc[(int64_t)(vi * 3 + 5) * n + i];
    }
    if (gc0 == 0.f && gc1 == 0.f && gc2 == 0.f) continue;  // not visible, or every channel clamped
    any = true;
    const ViewArgs &v = m.v[vi];
    float R[9], t[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = v.pose[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k] = v.pose[9 + k];
    float d[3], dinv;
    view_dir<float>(R, t, mu, d, dinv);
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      float Y, ax, ay, az;
      sh_term<float>(k, d[0], d[1], d[2], Y, ax, ay, az);
      gsh[k * 3] += gc0 * Y;
      gsh[k * 3 + 1] += gc1 * Y;
      gsh[k * 3 + 2] += gc2 * Y;
      if (DEG > 0) {
        const float wk = gc0 * sh[k * 3] + gc1 * sh[k * 3 + 1] + gc2 * sh[k * 3 + 2];
        gx += wk * ax;
        gy += wk * ay;
        gz += wk * az;
      }
    }
    if (DEG > 0) {
      const float radial = gx * d[0] + gy * d[1] + gz * d[2];
      gm[0] += (gx - radial * d[0]) * dinv;
      gm[1] += (gy - radial * d[1]) * dinv;
      gm[2] += (gz - radial * d[2]) * dinv;
    }
  }
  if (ADAM) {
    adam_gaussian<DEG>(m, i, mu, sh, gm, gsh, any);
    return;
  }
  if (!any && !m.store) return;
  if (DEG > 0 && any) {  // after the geometry pass's store or sum
#pragma unroll
    for (int k = 0; k < 3; ++k) m.gm[k * n + i] += gm[k];
  }
  if (m.store) {
#pragma unroll
    for (int k = 0; k < NB * 3; ++k) m.gsh[(int64_t)k * n + i] = gsh[k];
    return;
  }
#pragma unroll
  for (int k = 0; k < NB * 3; ++k) m.gsh[(int64_t)k * n + i] += gsh[k];
}

struct PoseOut {
  const float *pose;
  double *d_pose, *d_twist;
};
struct PoseOuts {
  PoseOut v[kMaxViews];
};

// Block v: sum of view v's block partials (fixed order) into dL/d[R|t] and
// the left twist.
__global__ __launch_bounds__(256) void k_pose_reduce(const double *partials, int64_t nparts, PoseOuts outs) {
  const PoseOut &po = outs.v[blockIdx.x];
  const double *part = partials + (int64_t)blockIdx.x * nparts * 12;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (int64_t b = threadIdx.x; b < nparts; b += 256)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] += part[b * 12 + k];
  __shared__ double red[4][12];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double g[12];
  for (int k = 0; k < 12; ++k) g[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
  if (po.d_pose)
    for (int k = 0; k < 12; ++k) po.d_pose[k] += g[k];
  if (po.d_twist) {
    double R[9], t[3];
    for (int k = 0; k < 9; ++k) R[k] = po.pose[k];
    for (int k = 0; k < 3; ++k) t[k] = po.pose[9 + k];
    // M = dL/dR R^T + dL/dt t^T; rho = dL/dt; phi = (M21 - M12, M02 - M20, M10 - M01)
    double M[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        M[3 * r + c] = g[3 * r] * R[3 * c] + g[3 * r + 1] * R[3 * c + 1] + g[3 * r + 2] * R[3 * c + 2] +
                       g[9 + r] * t[c];
    po.d_twist[0] += g[9];
    po.d_twist[1] += g[10];
    po.d_twist[2] += g[11];
    po.d_twist[3] += M[7] - M[5];
    po.d_twist[4] += M[2] - M[6];
    po.d_twist[5] += M[3] - M[1];
  }
}

gs_status check_camera(const gs_camera *cam, const char *fn) {
  GS_REQUIRE(cam, "%s: camera is NULL", fn);
  GS_REQUIRE(cam->width > 0 && cam->height > 0 && cam->width <= 16384 && cam->height <= 16384,
             "%s: image size %dx%d out of range", fn, cam->width, cam->height);
  GS_REQUIRE(cam->fx > 0.f && cam->fy > 0.f, "%s: focal lengths must be positive", fn);
  GS_REQUIRE(cam->pose, "%s: camera pose pointer is NULL", fn);
  return GS_OK;
}

gs_status check_gaussians(const gs_gaussians *g, const char *fn) {
  GS_REQUIRE(g, "%s: gaussians struct is NULL", fn);
  GS_REQUIRE(g->n >= 0 && g->n < (int64_t(1) << 31), "%s: n = %lld out of range", fn, (long long)g->n);
  GS_REQUIRE(g->sh_degree >= 0 && g->sh_degree <= 3, "%s: sh_degree %d not in 0..3", fn, g->sh_degree);
  if (g->n > 0)
    GS_REQUIRE(g->means && g->log_scales && g->quats && g->opacity_logits && g->sh, "%s: NULL parameter plane", fn);
  return GS_OK;
}

gs_status check_params(const gs_raster_params *rp, const char *fn) {
  GS_REQUIRE(rp, "%s: params is NULL", fn);
  GS_REQUIRE(rp->alpha_min > 0.f && rp->alpha_min < 1.f && rp->eps2d >= 0.f && rp->guard > 0.f,
             "%s: raster params out of range", fn);
  return GS_OK;
}

MultiArgs multi_args(const gs_raster_params *rp, const gs_gaussians *g) {
  MultiArgs m;
  m.n = g->n;
  m.nv = 0;
  m.eps2d = rp->eps2d;
  m.alpha_min = rp->alpha_min;
  m.guard = rp->guard;
  m.mip = rp->mip_filter != 0;
  m.store = 0;
  m.adam = 0;
  m.means = g->means; m.log_scales = g->log_scales; m.quats = g->quats; m.opac = g->opacity_logits; m.sh = g->sh;
  m.f3 = g->filter3d;
  m.gm = m.gl = m.gq = m.go = m.gsh = nullptr;
  m.partials = nullptr;
  m.gc = nullptr;
  m.visible = nullptr;
  m.visible_or = 0;
  return m;
}

ViewArgs view_args(const gs_camera *cam, const gs_projected *proj) {
  ViewArgs v;
  v.pose = cam->pose;
  v.fx = cam->fx; v.fy = cam->fy; v.cx = cam->cx; v.cy = cam->cy;
  v.near_plane = cam->near_plane;
  v.W = cam->width;
  v.H = cam->height;
  v.rec = proj ? proj->rec : nullptr;
  v.radius = proj ? proj->radius : nullptr;
  v.tiles = proj ? proj->tiles_touched : nullptr;
  v.bin = proj ? proj->bin : nullptr;
  v.pair_grad = nullptr;
  v.first_slot = nullptr;
  v.d_pose = v.d_twist = nullptr;
  return v;
}

int64_t proj_blocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

gs_status launch_project(const MultiArgs &m, int deg, hipStream_t s) {
  const int64_t blocks = proj_blocks(m.n);
  switch (deg) {
    case 0: GS_LAUNCH("project", k_project_views<0>, blocks, kBlock, 0, s, m); break;
    case 1: GS_LAUNCH("project", k_project_views<1>, blocks, kBlock, 0, s, m); break;
    case 2: GS_LAUNCH("project", k_project_views<2>, blocks, kBlock, 0, s, m); break;
    default: GS_LAUNCH("project", k_project_views<3>, blocks, kBlock, 0, s, m); break;
  }
  return GS_OK;
}

gs_status launch_project_bwd(const MultiArgs &m, int deg, hipStream_t s) {
  const int64_t blocks = proj_blocks(m.n);
  switch (deg) {
    case 0: GS_LAUNCH("project_bwd", k_project_bwd_views<0>, blocks, kBlock, 0, s, m); break;
    case 1: GS_LAUNCH("project_bwd", k_project_bwd_views<1>, blocks, kBlock, 0, s, m); break;
    case 2: GS_LAUNCH("project_bwd", k_project_bwd_views<2>, blocks, kBlock, 0, s, m); break;
    default: GS_LAUNCH("project_bwd", k_project_bwd_views<3>, blocks, kBlock, 0, s, m); break;
  }
  if (m.adam) {
    switch (deg) {
      case 0: GS_LAUNCH("project_bwd_adam", (k_project_bwd_sh<0, true>), blocks, kBlock, 0, s, m); break;
      case 1: GS_LAUNCH("project_bwd_adam", (k_project_bwd_sh<1, true>), blocks, kBlock, 0, s, m); break;
      case 2: GS_LAUNCH("project_bwd_adam", (k_project_bwd_sh<2, true>), blocks, kBlock, 0, s, m); break;
      default: GS_LAUNCH("project_bwd_adam", (k_project_bwd_sh<3, true>), blocks, kBlock, 0, s, m); break;
    }
  } else {
    switch (deg) {
      case 0: GS_LAUNCH("project_bwd_sh", (k_project_bwd_sh<0, false>), blocks, kBlock, 0, s, m); break;
      case 1: GS_LAUNCH("project_bwd_sh", (k_project_bwd_sh<1, false>), blocks, kBlock, 0, s, m); break;
      case 2: GS_LAUNCH("project_bwd_sh", (k_project_bwd_sh<2, false>), blocks, kBlock, 0, s, m); break;
      default: GS_LAUNCH("project_bwd_sh", (k_project_bwd_sh<3, false>), blocks, kBlock, 0, s, m); break;
    }
  }
  bool pose = false;
  PoseOuts outs;
  for (int v = 0; v < kMaxViews; ++v) {
    outs.v[v].pose = v < m.nv ? m.v[v].pose : nullptr;
    outs.v[v].d_pose = v < m.nv ? m.v[v].d_pose : nullptr;
    outs.v[v].d_twist = v < m.nv ? m.v[v].d_twist : nullptr;
    pose = pose || outs.v[v].d_pose || outs.v[v].d_twist;
  }
  if (pose) GS_LAUNCH("pose_reduce", k_pose_reduce, m.nv, 256, 0, s, (const double *)m.partials, blocks, outs);
  return GS_OK;
}

}  // namespace
}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_project(const gs_camera *cam, const gs_raster_params *rp, const gs_gaussians *g, gs_projected *out,
                     void *stream) {
  gs_status st = check_camera(cam, "gs_project");
  if (st != GS_OK) return st;
  if ((st = check_gaussians(g, "gs_project")) != GS_OK) return st;
  if ((st = check_params(rp, "gs_project")) != GS_OK) return st;
  GS_REQUIRE(out, "gs_project: output struct is NULL");
  if (g->n == 0) return GS_OK;
  GS_REQUIRE(out->rec && out->radius && out->tiles_touched, "gs_project: NULL output plane");
  GS_REQUIRE(((uintptr_t)out->bin & 15u) == 0, "gs_project: bin must be 16-byte aligned");
  if (finite_checks_on()) {
    if ((st = check_finite(cam->pose, 12, "gs_project", "pose", (hipStream_t)stream)) != GS_OK) return st;
    if ((st = check_finite_gaussians(g, "gs_project", "gaussians", (hipStream_t)stream)) != GS_OK) return st;
  }
  MultiArgs m = multi_args(rp, g);
  m.nv = 1;
  m.v[0] = view_args(cam, out);
  return launch_project(m, g->sh_degree, (hipStream_t)stream);
}

gs_status gs_project_views(int32_t n_views, const gs_view *views, const gs_raster_params *rp,
                           const gs_gaussians *g, void *stream) {
  GS_REQUIRE(n_views >= 0 && (n_views == 0 || views), "gs_project_views: bad view list");
  gs_status st = check_gaussians(g, "gs_project_views");
  if (st != GS_OK) return st;
  if ((st = check_params(rp, "gs_project_views")) != GS_OK) return st;
  for (int v = 0; v < n_views; ++v) {
    if ((st = check_camera(&views[v].cam, "gs_project_views")) != GS_OK) return st;
    if (g->n > 0)
      GS_REQUIRE(views[v].proj.rec && views[v].proj.radius && views[v].proj.tiles_touched,
                 "gs_project_views: view %d has a NULL output plane", v);
    GS_REQUIRE(((uintptr_t)views[v].proj.bin & 15u) == 0, "gs_project_views: view %d: bin must be 16-byte aligned",
               v);
  }
  if (g->n == 0) return GS_OK;
  if (finite_checks_on()) {
    for (int v = 0; v < n_views; ++v)
      if ((st = check_finite(views[v].cam.pose, 12, "gs_project_views", "pose", (hipStream_t)stream)) != GS_OK)
        return st;
    if ((st = check_finite_gaussians(g, "gs_project_views", "gaussians", (hipStream_t)stream)) != GS_OK) return st;
  }
  for (int v0 = 0; v0 < n_views; v0 += kMaxViews) {
    MultiArgs m = multi_args(rp, g);
    m.nv = std::min(kMaxViews, n_views - v0);
    for (int k = 0; k < m.nv; ++k) m.v[k] = view_args(&views[v0 + k].cam, &views[v0 + k].proj);
    if ((st = launch_project(m, g->sh_degree, (hipStream_t)stream)) != GS_OK) return st;
  }
  return GS_OK;
}

gs_status gs_project_bwd_views_workspace(int64_t n, int32_t n_views, size_t *bytes) {
  GS_REQUIRE(bytes && n >= 0 && n_views >= 0, "gs_project_bwd_views_workspace: bad argument");
  const int64_t blocks = proj_blocks(n);
  const int nv = std::max(1, std::min(kMaxViews, (int)n_views));
  // pose partials, then the per-view clamped colour gradients
  *bytes = align_up(sizeof(double) * 12 * (size_t)nv * (size_t)(blocks > 0 ? blocks : 1)) +
           align_up(sizeof(float) * 3 * (size_t)nv * (size_t)(n > 0 ? n : 1));
  return GS_OK;
}

static gs_status project_bwd_views(int32_t n_views, const gs_view *views, const gs_raster_params *rp,
                                   const gs_gaussians *g, gs_gaussians *grads, void *ws, size_t ws_bytes,
                                   void *stream, int store, int32_t *visible, const AdamArgs *adam = nullptr);

gs_status gs_project_bwd_views(int32_t n_views, const gs_view *views, const gs_raster_params *rp,
                               const gs_gaussians *g, gs_gaussians *grads, void *ws, size_t ws_bytes, void *stream) {
  return project_bwd_views(n_views, views, rp, g, grads, ws, ws_bytes, stream, 0, nullptr);
}

gs_status gs_project_bwd_views_store(int32_t n_views, const gs_view *views, const gs_raster_params *rp,
                                     const gs_gaussians *g, gs_gaussians *grads, void *ws, size_t ws_bytes,
                                     int32_t *visible, void *stream) {
  return project_bwd_views(n_views, views, rp, g, grads, ws, ws_bytes, stream, 1, visible);
}

gs_status gs_project_bwd_views_adam(int32_t n_views, const gs_view *views, const gs_raster_params *rp,
                                    gs_gaussians *g, gs_gaussians *m1, gs_gaussians *m2, float *lr_scale,
                                    const gs_adam_groups *opt, gs_gaussians *grads, void *ws, size_t ws_bytes,
                                    int32_t *visible, void *stream) {
  const char *fn = "gs_project_bwd_views_adam";
  gs_status st = check_gaussians(g, fn);
  if (st != GS_OK) return st;
  if ((st = check_gaussians(m1, fn)) != GS_OK || (st = check_gaussians(m2, fn)) != GS_OK) return st;
  GS_REQUIRE(m1->n == g->n && m2->n == g->n && m1->sh_degree == g->sh_degree && m2->sh_degree == g->sh_degree,
             "%s: moment shapes differ from the Gaussians'", fn);
  GS_REQUIRE(opt, "%s: NULL optimiser settings", fn);
  GS_REQUIRE(opt->step >= 1, "%s: step must be >= 1", fn);
  GS_REQUIRE(opt->beta1 >= 0.f && opt->beta1 < 1.f && opt->beta2 >= 0.f && opt->beta2 < 1.f && opt->eps >= 0.f,
             "%s: bad betas or eps", fn);
  GS_REQUIRE(opt->lr_decay > 0.f && opt->lr_decay <= 1.f, "%s: lr_decay must be in (0, 1]", fn);
  if (g->n > 0) GS_REQUIRE(visible, "%s: visible is required", fn);
  AdamArgs a;
  float *const planes[3][5] = {{g->means, g->log_scales, g->quats, g->opacity_logits, g->sh},
                               {m1->means, m1->log_scales, m1->quats, m1->opacity_logits, m1->sh},
                               {m2->means, m2->log_scales, m2->quats, m2->opacity_logits, m2->sh}};
  for (int k = 0; k < 5; ++k) {
    a.p[k] = planes[0][k];
    a.m1[k] = planes[1][k];
    a.m2[k] = planes[2][k];
  }
  a.rate = lr_scale;
  a.lr[0] = opt->lr_means; a.lr[1] = opt->lr_log_scales; a.lr[2] = opt->lr_quats; a.lr[3] = opt->lr_opacity;
  a.lr[4] = opt->lr_sh_dc; a.lr[5] = opt->lr_sh_rest;
  a.b1 = opt->beta1; a.b2 = opt->beta2; a.eps = opt->eps;
  a.c1 = adam_bias(opt->beta1, opt->step);
  a.c2 = adam_bias(opt->beta2, opt->step);
  a.decay = opt->lr_decay;
  return project_bwd_views(n_views, views, rp, g, grads, ws, ws_bytes, stream, 1, visible, &a);
}

}  // extern "C"

static gs_status project_bwd_views(int32_t n_views, const gs_view *views, const gs_raster_params *rp,
                                   const gs_gaussians *g, gs_gaussians *grads, void *ws, size_t ws_bytes,
                                   void *stream, int store, int32_t *visible, const AdamArgs *adam) {
  GS_REQUIRE(n_views >= 0 && (n_views == 0 || views), "gs_project_bwd_views: bad view list");
  gs_status st = check_gaussians(g, "gs_project_bwd_views");
  if (st != GS_OK) return st;
  if ((st = check_gaussians(grads, "gs_project_bwd_views(grads)")) != GS_OK) return st;
  GS_REQUIRE(grads->n == g->n && grads->sh_degree == g->sh_degree, "gs_project_bwd_views: grads shape differs");
  if ((st = check_params(rp, "gs_project_bwd_views")) != GS_OK) return st;
  for (int v = 0; v < n_views; ++v) {
    if ((st = check_camera(&views[v].cam, "gs_project_bwd_views")) != GS_OK) return st;
    if (g->n > 0)
      GS_REQUIRE(views[v].proj.rec && views[v].proj.tiles_touched && views[v].first_slot && views[v].pair_grad,
                 "gs_project_bwd_views: view %d has a NULL input", v);
  }
  size_t need = 0;
  gs_project_bwd_views_workspace(g->n, n_views, &need);
  if (ws_bytes < need || !ws) {
    set_error("gs_project_bwd_views: workspace %zu bytes < %zu", ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  if (g->n == 0) return GS_OK;
  // (with no view the store form still runs once: every gradient becomes 0)
  for (int v0 = 0; v0 < n_views || (store && v0 == 0); v0 += kMaxViews) {
    MultiArgs m = multi_args(rp, g);
    m.gm = grads->means; m.gl = grads->log_scales; m.gq = grads->quats; m.go = grads->opacity_logits;
    m.gsh = grads->sh;
    m.partials = (double *)ws;
    m.gc = (float *)((char *)ws + align_up(sizeof(double) * 12 * (size_t)std::max(1, std::min(kMaxViews, (int)n_views)) *
                                           (size_t)proj_blocks(g->n)));
    m.nv = std::min(kMaxViews, n_views - v0);
    m.store = store && v0 == 0;  // later batches of views add to the first batch's stores
    m.visible = visible;
    m.visible_or = v0 > 0;
    if (adam && v0 + kMaxViews >= n_views) {  // the last batch applies the step
      m.adam = 1;
      m.opt = *adam;
    }
    for (int k = 0; k < m.nv; ++k) {
      const gs_view &gv = views[v0 + k];
      m.v[k] = view_args(&gv.cam, &gv.proj);
      m.v[k].pair_grad = gv.pair_grad;
      m.v[k].first_slot = gv.first_slot;
      m.v[k].d_pose = gv.dL_dpose;
      m.v[k].d_twist = gv.dL_dtwist;
    }
    if ((st = launch_project_bwd(m, g->sh_degree, (hipStream_t)stream)) != GS_OK) return st;
  }
  return GS_OK;
}

extern "C" {

}  // extern "C"

namespace gsmi {

gs_status validate_camera(const gs_camera *cam, const char *fn) { return check_camera(cam, fn); }
gs_status validate_gaussians(const gs_gaussians *g, const char *fn) { return check_gaussians(g, fn); }

}  // namespace gsmi
