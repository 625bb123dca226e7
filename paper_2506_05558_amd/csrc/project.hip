// Per-Gaussian EWA projection (forward) and its adjoint, including the
// camera-pose gradient reduction.
//
// One lane per Gaussian; parameters are read as SoA planes (every load of a
// wave is one contiguous 256-byte segment per plane), the pose is a uniform
// 48-byte read.  Geometry runs in FP64: on gfx950 the FP64 vector rate
// equals the unpacked FP32 rate, so the extra precision costs nothing in a
// kernel bounded by HBM traffic (236 B in + 72 B out per SH-degree-3
// Gaussian).  The adjoint runs in FP32 (hardware exp, rcp, rsqrt) with the
// SH terms streamed one coefficient at a time, which keeps its register
// footprint and with it occupancy up; the camera-pose sum over all Gaussians
// is reduced in FP64.
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

struct ProjArgs {
  int64_t n;
  int W, H;
  double fx, fy, cx, cy, near_plane, eps2d, alpha_min, guard;
  const float *pose;
  const float *means, *log_scales, *quats, *opac, *sh;
  float *rec;
  int32_t *radius, *tiles;  // radius: [2][n] (rx, ry)
};

// Geometry of one Gaussian's forward: FP64 for the forward projection (the
// render record needs a sub-1e-6-pixel mean), FP32 for the adjoint, whose
// 2D covariance is kept well conditioned by the eps2d dilation.
template <class Real>
struct Geo {
  Real R[9];
  Real p[3], iz;
  bool clx, cly;
  Real J00, J02, J11, J12;
  Real qn[4], qinv;
  Real Rq[9], s[3], M[9];
  Real T[6], TM[6];
  Real a, b, c, A, B, C;
};

template <class Real>
__device__ __forceinline__ void load_pose(const float *pose, Real R[9], Real t[3]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = (Real)pose[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) t[k] = (Real)pose[9 + k];
}

__device__ __forceinline__ double real_exp(double x) { return exp(x); }
__device__ __forceinline__ float real_exp(float x) { return __expf(x); }
__device__ __forceinline__ double real_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float real_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double real_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float real_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Camera-space point and the 2D covariance.  Returns false if culled by
// the near plane or a non-positive determinant.
template <class Real>
__device__ __forceinline__ bool geometry(const ProjArgs &a, int64_t i, const Real mu[3], const Real t[3],
                                         Geo<Real> &f) {
  const int64_t n = a.n;
#pragma unroll
  for (int r = 0; r < 3; ++r) f.p[r] = f.R[3 * r] * mu[0] + f.R[3 * r + 1] * mu[1] + f.R[3 * r + 2] * mu[2] + t[r];
  if (!(f.p[2] > (Real)a.near_plane)) return false;
  f.iz = real_rcp(f.p[2]);
  const Real limx = (Real)(a.guard * 0.5 * a.W / a.fx), limy = (Real)(a.guard * 0.5 * a.H / a.fy);
  const Real tx = f.p[0] * f.iz, ty = f.p[1] * f.iz;
  f.clx = tx < -limx || tx > limx;
  f.cly = ty < -limy || ty > limy;
  const Real xc = f.clx ? (tx < 0 ? -limx : limx) * f.p[2] : f.p[0];
  const Real yc = f.cly ? (ty < 0 ? -limy : limy) * f.p[2] : f.p[1];
  const Real fx = (Real)a.fx, fy = (Real)a.fy;
  f.J00 = fx * f.iz;
  f.J11 = fy * f.iz;
  f.J02 = -fx * xc * f.iz * f.iz;
  f.J12 = -fy * yc * f.iz * f.iz;

  const Real q0 = a.quats[i], q1 = a.quats[n + i], q2 = a.quats[2 * n + i], q3 = a.quats[3 * n + i];
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
  for (int k = 0; k < 3; ++k) f.s[k] = real_exp((Real)a.log_scales[k * n + i]);
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
  f.a = f.TM[0] * f.TM[0] + f.TM[1] * f.TM[1] + f.TM[2] * f.TM[2] + (Real)a.eps2d;
  f.b = f.TM[0] * f.TM[3] + f.TM[1] * f.TM[4] + f.TM[2] * f.TM[5];
  f.c = f.TM[3] * f.TM[3] + f.TM[4] * f.TM[4] + f.TM[5] * f.TM[5] + (Real)a.eps2d;
  const Real det = f.a * f.c - f.b * f.b;
  if (!(det > 0)) return false;
  const Real idet = real_rcp(det);
  f.A = f.c * idet;
  f.B = -f.b * idet;
  f.C = f.a * idet;
  return true;
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

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project(ProjArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.n;
  Geo<double> f;
  double t[3];
  load_pose<double>(a.pose, f.R, t);
  const double mu[3] = {a.means[i], a.means[n + i], a.means[2 * n + i]};
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0, r3 = r0;
  int rx = 0, ry = 0, tiles = 0;
  bool ok = geometry<double>(a, i, mu, t, f);
  double mx = 0, my = 0, o = 0;
  if (ok) {
    mx = a.fx * f.p[0] * f.iz + a.cx;
    my = a.fy * f.p[1] * f.iz + a.cy;
    ok = fabs(mx) < 8388608.0 && fabs(my) < 8388608.0;  // |mean| < 2^23 px
  }
  if (ok) {
    o = 1.0 / (1.0 + exp(-(double)a.opac[i]));
    ok = o >= a.alpha_min;
  }
  if (ok) {
    // support: o exp(-q/2) >= alpha_min  <=>  q = d^T Sigma2^-1 d <= qmax;
    // its bounding box has half-extents sqrt(qmax a), sqrt(qmax c)
    const double qmax = 2.0 * log(o / a.alpha_min);
    const double hx = sqrt(qmax * f.a), hy = sqrt(qmax * f.c);
    rx = (int)ceil(fmin(hx * (1.0 + 1e-4) + 1e-3, 4194304.0));
    ry = (int)ceil(fmin(hy * (1.0 + 1e-4) + 1e-3, 4194304.0));
    double d[3], dinv;
    view_dir<double>(f.R, t, mu, d, dinv);
    double val[3] = {0.5, 0.5, 0.5};
    constexpr int NB = (DEG + 1) * (DEG + 1);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      double Y, gx, gy, gz;
      sh_term<double>(k, d[0], d[1], d[2], Y, gx, gy, gz);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) val[ch] += (double)a.sh[(int64_t)(k * 3 + ch) * n + i] * Y;
    }
    const double hxm = rint(mx), hym = rint(my);
    r0 = make_float4((float)hxm, (float)hym, (float)(mx - hxm), (float)(my - hym));
    r1 = make_float4((float)f.A, (float)f.B, (float)f.C, (float)o);
    r2 = make_float4((float)fmax(val[0], 0.0), (float)fmax(val[1], 0.0), (float)fmax(val[2], 0.0), (float)f.p[2]);
    r3 = make_float4((float)hx, (float)hy, 0.f, 0.f);
    int tx0, ty0, tx1, ty1;
    if (tile_rect(__fadd_rn(r0.x, r0.z), __fadd_rn(r0.y, r0.w), rx, ry, a.W, a.H, tx0, ty0, tx1, ty1))
      tiles = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
  }
  float4 *dst = (float4 *)(a.rec + i * GS_REC_FLOATS);
  dst[0] = r0;
  dst[1] = r1;
  dst[2] = r2;
  dst[3] = r3;
  a.radius[i] = rx;
  a.radius[n + i] = ry;
  a.tiles[i] = tiles;
}

// ---------------------------------------------------------------- backward
struct BwdArgs {
  ProjArgs p;
  const float *pair_grad;     // [M][12] 2D gradients per (Gaussian, tile) pair (first 10 used)
  const uint32_t *first_slot; // first pair slot of each visible Gaussian
  float *gm, *gl, *gq, *go, *gsh;  // parameter gradients (accumulated)
  double *partials;  // [gridDim.x][12] pose partial sums
};

// Adjoint of one visible Gaussian, in FP32 (the forward decided
// visibility; the adjoint only chains gradients).  Writes the pose terms of
// this Gaussian into pose[12]: dL/dR (row-major) and dL/dt.
template <int DEG>
__device__ __forceinline__ void backward_one(const BwdArgs &ba, int64_t i, int ntiles, float pose[12]) {
  const ProjArgs &a = ba.p;
  const int64_t n = a.n;
  Geo<float> f;
  float t[3];
  load_pose<float>(a.pose, f.R, t);
  const float mu[3] = {a.means[i], a.means[n + i], a.means[2 * n + i]};
  geometry<float>(a, i, mu, t, f);
  // the Gaussian's pairs are contiguous: sum their 2D gradients in slot order
  float4 g0 = make_float4(0.f, 0.f, 0.f, 0.f), g1 = g0, g2 = g0;
  {
    const float4 *gp4 = (const float4 *)(ba.pair_grad + (size_t)ba.first_slot[i] * 12);
    for (int j = 0; j < ntiles; ++j) {
      const float4 a0 = gp4[3 * j], a1 = gp4[3 * j + 1], a2 = gp4[3 * j + 2];
      g0.x += a0.x; g0.y += a0.y; g0.z += a0.z; g0.w += a0.w;
      g1.x += a1.x; g1.y += a1.y; g1.z += a1.z; g1.w += a1.w;
      g2.x += a2.x; g2.y += a2.y;
    }
  }
  // g0 = (d mean x, d mean y, dA, dB), g1 = (dC, d opacity, d r, d g), g2 = (d b, d z, -, -)
  const float4 rgbz = *(const float4 *)(a.rec + i * GS_REC_FLOATS + 8);

  float gmu[3] = {0.f, 0.f, 0.f};

  // colour -> SH coefficients and view direction (no pose path, section 4.3).
  // A channel whose colour was clamped at 0 passes no gradient.
  {
    const float gc0 = rgbz.x > 0.f ? g1.z : 0.f;
    const float gc1 = rgbz.y > 0.f ? g1.w : 0.f;
    const float gc2 = rgbz.z > 0.f ? g2.x : 0.f;
    float d[3], dinv;
    view_dir<float>(f.R, t, mu, d, dinv);
    float gx = 0.f, gy = 0.f, gz = 0.f;
    constexpr int NB = (DEG + 1) * (DEG + 1);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      float Y, ax, ay, az;
      sh_term<float>(k, d[0], d[1], d[2], Y, ax, ay, az);
      const int64_t o0 = (int64_t)(k * 3) * n + i;
      ba.gsh[o0] += gc0 * Y;
      ba.gsh[o0 + n] += gc1 * Y;
      ba.gsh[o0 + 2 * n] += gc2 * Y;
      if (DEG > 0) {
        const float wk = gc0 * a.sh[o0] + gc1 * a.sh[o0 + n] + gc2 * a.sh[o0 + 2 * n];
        gx += wk * ax;
        gy += wk * ay;
        gz += wk * az;
      }
    }
    if (DEG > 0) {
      const float radial = gx * d[0] + gy * d[1] + gz * d[2];
      gmu[0] += (gx - radial * d[0]) * dinv;
      gmu[1] += (gy - radial * d[1]) * dinv;
      gmu[2] += (gz - radial * d[2]) * dinv;
    }
  }

  {
    const float o = real_rcp(1.0f + __expf(-a.opac[i]));
    ba.go[i] += g1.y * o * (1.0f - o);
  }

  // conic -> Sigma2: dL/dSigma2 = -Q G Q with G = [[gA, gB/2], [gB/2, gC]]
  const float gA = g0.z, hB = 0.5f * g0.w, gC = g1.x;
  const float QG00 = f.A * gA + f.B * hB, QG01 = f.A * hB + f.B * gC;
  const float QG10 = f.B * gA + f.C * hB, QG11 = f.B * hB + f.C * gC;
  const float S00 = -(QG00 * f.A + QG01 * f.B);
  const float S01 = -(QG00 * f.B + QG01 * f.C);
  const float S11 = -(QG10 * f.B + QG11 * f.C);

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
    ba.gl[c * n + i] += gs * f.s[c];
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
    ba.gq[i] += (dw - proj * w) * f.qinv;
    ba.gq[n + i] += (dx - proj * x) * f.qinv;
    ba.gq[2 * n + i] += (dy - proj * y) * f.qinv;
    ba.gq[3 * n + i] += (dz - proj * z) * f.qinv;
  }

  // T = J R: gJ = gT R^T (entries 00, 02, 11, 12); gR from the covariance = J^T gT
  const float gJ00 = gT[0] * f.R[0] + gT[1] * f.R[1] + gT[2] * f.R[2];
  const float gJ02 = gT[0] * f.R[6] + gT[1] * f.R[7] + gT[2] * f.R[8];
  const float gJ11 = gT[3] * f.R[3] + gT[4] * f.R[4] + gT[5] * f.R[5];
  const float gJ12 = gT[3] * f.R[6] + gT[4] * f.R[7] + gT[5] * f.R[8];

  // camera-space point: mean2d, depth and the Jacobian entries
  const float fx = (float)a.fx, fy = (float)a.fy;
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
  gmu[0] += f.R[0] * gp0 + f.R[3] * gp1 + f.R[6] * gp2;
  gmu[1] += f.R[1] * gp0 + f.R[4] * gp1 + f.R[7] * gp2;
  gmu[2] += f.R[2] * gp0 + f.R[5] * gp1 + f.R[8] * gp2;
  ba.gm[i] += gmu[0];
  ba.gm[n + i] += gmu[1];
  ba.gm[2 * n + i] += gmu[2];

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

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project_bwd(BwdArgs ba, const int32_t *tiles) {
  float term[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) term[k] = 0.f;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int nt = i < ba.p.n ? tiles[i] : 0;
  if (nt > 0) backward_one<DEG>(ba, i, nt, term);
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = (double)term[k];

  // block reduction of the 12 pose partials (fixed order: deterministic)
  __shared__ double red[kBlock / 64][12];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) v += red[w][threadIdx.x];
    ba.partials[(int64_t)blockIdx.x * 12 + threadIdx.x] = v;
  }
}

// Sum of the block partials (fixed order) into dL/d[R|t] and the left twist.
__global__ __launch_bounds__(256) void k_pose_reduce(const double *partials, int64_t nparts, const float *pose,
                                                     double *d_pose, double *d_twist) {
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (int64_t b = threadIdx.x; b < nparts; b += 256)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] += partials[b * 12 + k];
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
  if (d_pose)
    for (int k = 0; k < 12; ++k) d_pose[k] += g[k];
  if (d_twist) {
    double R[9], t[3];
    for (int k = 0; k < 9; ++k) R[k] = pose[k];
    for (int k = 0; k < 3; ++k) t[k] = pose[9 + k];
    // M = dL/dR R^T + dL/dt t^T; rho = dL/dt; phi = (M21 - M12, M02 - M20, M10 - M01)
    double M[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        M[3 * r + c] = g[3 * r] * R[3 * c] + g[3 * r + 1] * R[3 * c + 1] + g[3 * r + 2] * R[3 * c + 2] +
                       g[9 + r] * t[c];
    d_twist[0] += g[9];
    d_twist[1] += g[10];
    d_twist[2] += g[11];
    d_twist[3] += M[7] - M[5];
    d_twist[4] += M[2] - M[6];
    d_twist[5] += M[3] - M[1];
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

ProjArgs make_args(const gs_camera *cam, const gs_raster_params *rp, const gs_gaussians *g) {
  ProjArgs a;
  a.n = g->n;
  a.W = cam->width;
  a.H = cam->height;
  a.fx = cam->fx; a.fy = cam->fy; a.cx = cam->cx; a.cy = cam->cy;
  a.near_plane = cam->near_plane;
  a.eps2d = rp->eps2d;
  a.alpha_min = rp->alpha_min;
  a.guard = rp->guard;
  a.pose = cam->pose;
  a.means = g->means; a.log_scales = g->log_scales; a.quats = g->quats; a.opac = g->opacity_logits; a.sh = g->sh;
  a.rec = nullptr; a.radius = nullptr; a.tiles = nullptr;
  return a;
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
  GS_REQUIRE(rp, "gs_project: params is NULL");
  GS_REQUIRE(rp->alpha_min > 0.f && rp->alpha_min < 1.f && rp->eps2d >= 0.f && rp->guard > 0.f,
             "gs_project: raster params out of range");
  GS_REQUIRE(out, "gs_project: output struct is NULL");
  if (g->n == 0) return GS_OK;
  GS_REQUIRE(out->rec && out->radius && out->tiles_touched, "gs_project: NULL output plane");
  ProjArgs a = make_args(cam, rp, g);
  a.rec = out->rec;
  a.radius = out->radius;
  a.tiles = out->tiles_touched;
  const int64_t blocks = (g->n + kBlock - 1) / kBlock;
  hipStream_t s = (hipStream_t)stream;
  switch (g->sh_degree) {
    case 0: GS_LAUNCH("project", k_project<0>, blocks, kBlock, 0, s, a); break;
    case 1: GS_LAUNCH("project", k_project<1>, blocks, kBlock, 0, s, a); break;
    case 2: GS_LAUNCH("project", k_project<2>, blocks, kBlock, 0, s, a); break;
    default: GS_LAUNCH("project", k_project<3>, blocks, kBlock, 0, s, a); break;
  }
  return GS_OK;
}

}  // extern "C"

namespace gsmi {

size_t project_bwd_workspace(int64_t n) {
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  return align_up(sizeof(double) * 12 * (size_t)(blocks > 0 ? blocks : 1));
}

gs_status project_bwd(const gs_camera *cam, const gs_raster_params *rp, const gs_gaussians *g,
                      const gs_projected *proj, const float *pair_grad, const uint32_t *first_slot,
                      gs_gaussians *grads, double *d_pose, double *d_twist, void *ws, hipStream_t s) {
  if (g->n == 0) return GS_OK;
  BwdArgs ba;
  ba.p = make_args(cam, rp, g);
  ba.p.rec = proj->rec;
  ba.pair_grad = pair_grad;
  ba.first_slot = first_slot;
  ba.gm = grads->means;
  ba.gl = grads->log_scales;
  ba.gq = grads->quats;
  ba.go = grads->opacity_logits;
  ba.gsh = grads->sh;
  ba.partials = (double *)ws;
  const int64_t blocks = (g->n + kBlock - 1) / kBlock;
  switch (g->sh_degree) {
    case 0: GS_LAUNCH("project_bwd", k_project_bwd<0>, blocks, kBlock, 0, s, ba, proj->tiles_touched); break;
    case 1: GS_LAUNCH("project_bwd", k_project_bwd<1>, blocks, kBlock, 0, s, ba, proj->tiles_touched); break;
    case 2: GS_LAUNCH("project_bwd", k_project_bwd<2>, blocks, kBlock, 0, s, ba, proj->tiles_touched); break;
    default: GS_LAUNCH("project_bwd", k_project_bwd<3>, blocks, kBlock, 0, s, ba, proj->tiles_touched); break;
  }
  if (d_pose || d_twist)
    GS_LAUNCH("pose_reduce", k_pose_reduce, 1, 256, 0, s, (const double *)ws, blocks, cam->pose, d_pose, d_twist);
  return GS_OK;
}

gs_status validate_camera(const gs_camera *cam, const char *fn) { return check_camera(cam, fn); }
gs_status validate_gaussians(const gs_gaussians *g, const char *fn) { return check_gaussians(g, fn); }

}  // namespace gsmi
