// Per-Gaussian EWA projection (forward) and its adjoint, including the
// camera-pose gradient reduction.
//
// One lane per Gaussian; parameters are read as SoA planes (every load of a
// wave is one contiguous 256-byte segment per plane), the pose is a uniform
// 48-byte read.  The geometry runs in FP64: on gfx950 the FP64 vector rate
// equals the unpacked FP32 rate, so the extra precision is free in a kernel
// bounded by HBM traffic (236 B in + 56 B out per SH-degree-3 Gaussian).
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

template <int DEG>
__device__ __forceinline__ void sh_basis(double x, double y, double z, double *Y) {
  Y[0] = kY0;
  if (DEG >= 1) {
    Y[1] = -kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = -kY1 * x;
  }
  if (DEG >= 2) {
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kY2a * x * y;
    Y[5] = -kY2a * y * z;
    Y[6] = kY2b * (2.0 * zz - xx - yy);
    Y[7] = -kY2a * x * z;
    Y[8] = kY2c * (xx - yy);
    if (DEG >= 3) {
      Y[9] = -kY3a * y * (3.0 * xx - yy);
      Y[10] = kY3b * x * y * z;
      Y[11] = -kY3c * y * (4.0 * zz - xx - yy);
      Y[12] = kY3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
      Y[13] = -kY3c * x * (4.0 * zz - xx - yy);
      Y[14] = kY3e * z * (xx - yy);
      Y[15] = -kY3a * x * (xx - 3.0 * yy);
    }
  }
}

// Gradient of sum_k w[k] Y_k(x, y, z) with respect to (x, y, z), the basis
// polynomials differentiated as functions on R^3.
template <int DEG>
__device__ __forceinline__ void sh_basis_vjp(double x, double y, double z, const double *w, double &gx, double &gy,
                                             double &gz) {
  gx = gy = gz = 0.0;
  if (DEG >= 1) {
    gy -= kY1 * w[1];
    gz += kY1 * w[2];
    gx -= kY1 * w[3];
  }
  if (DEG >= 2) {
    gx += kY2a * y * w[4];
    gy += kY2a * x * w[4];
    gy -= kY2a * z * w[5];
    gz -= kY2a * y * w[5];
    gx -= 2.0 * kY2b * x * w[6];
    gy -= 2.0 * kY2b * y * w[6];
    gz += 4.0 * kY2b * z * w[6];
    gx -= kY2a * z * w[7];
    gz -= kY2a * x * w[7];
    gx += 2.0 * kY2c * x * w[8];
    gy -= 2.0 * kY2c * y * w[8];
  }
  if (DEG >= 3) {
    const double xx = x * x, yy = y * y, zz = z * z;
    gx -= 6.0 * kY3a * x * y * w[9];
    gy -= kY3a * (3.0 * xx - 3.0 * yy) * w[9];
    gx += kY3b * y * z * w[10];
    gy += kY3b * x * z * w[10];
    gz += kY3b * x * y * w[10];
    gx += 2.0 * kY3c * x * y * w[11];
    gy -= kY3c * (4.0 * zz - xx - 3.0 * yy) * w[11];
    gz -= 8.0 * kY3c * y * z * w[11];
    gx -= 6.0 * kY3d * x * z * w[12];
    gy -= 6.0 * kY3d * y * z * w[12];
    gz += kY3d * (6.0 * zz - 3.0 * xx - 3.0 * yy) * w[12];
    gx -= kY3c * (4.0 * zz - 3.0 * xx - yy) * w[13];
    gy += 2.0 * kY3c * x * y * w[13];
    gz -= 8.0 * kY3c * x * z * w[13];
    gx += 2.0 * kY3e * x * z * w[14];
    gy -= 2.0 * kY3e * y * z * w[14];
    gz += kY3e * (xx - yy) * w[14];
    gx -= kY3a * (3.0 * xx - 3.0 * yy) * w[15];
    gy += 6.0 * kY3a * x * y * w[15];
  }
}

struct ProjArgs {
  int64_t n;
  int W, H;
  double fx, fy, cx, cy, near_plane, eps2d, alpha_min, guard;
  const float *pose;
  const float *means, *log_scales, *quats, *opac, *sh;
  float *rec;
  int32_t *radius, *tiles;
};

// Everything one Gaussian's forward produces, in FP64.
struct Fwd {
  double R[9], t[3];
  double mu[3], p[3], z, iz;
  bool clx, cly;
  double J00, J02, J11, J12;
  double qn[4], qinv;  // normalised quaternion, 1/|q|
  double Rq[9], s[3], M[9];
  double T[6], TM[6];  // T = J R (2x3), TM = T M
  double a, b, c, A, B, C;
  double mx, my, o;
  double dhat[3], dinv;
  double val[3];
  int radius;
};

__device__ __forceinline__ void load_pose(const float *pose, double R[9], double t[3]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = (double)pose[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) t[k] = (double)pose[9 + k];
}

// Returns false for culled Gaussians (then only R, t, mu, p are valid).
template <int DEG>
__device__ __forceinline__ bool forward_one(const ProjArgs &a, int64_t i, Fwd &f) {
  const int64_t n = a.n;
  load_pose(a.pose, f.R, f.t);
  f.mu[0] = a.means[i];
  f.mu[1] = a.means[n + i];
  f.mu[2] = a.means[2 * n + i];
#pragma unroll
  for (int r = 0; r < 3; ++r) f.p[r] = f.R[3 * r] * f.mu[0] + f.R[3 * r + 1] * f.mu[1] + f.R[3 * r + 2] * f.mu[2] + f.t[r];
  f.z = f.p[2];
  if (!(f.z > a.near_plane)) return false;
  f.iz = 1.0 / f.z;

  // perspective Jacobian, guard band on x/z and y/z
  const double limx = a.guard * 0.5 * a.W / a.fx, limy = a.guard * 0.5 * a.H / a.fy;
  const double tx = f.p[0] * f.iz, ty = f.p[1] * f.iz;
  f.clx = tx < -limx || tx > limx;
  f.cly = ty < -limy || ty > limy;
  const double xc = f.clx ? (tx < 0.0 ? -limx : limx) * f.z : f.p[0];
  const double yc = f.cly ? (ty < 0.0 ? -limy : limy) * f.z : f.p[1];
  f.J00 = a.fx * f.iz;
  f.J11 = a.fy * f.iz;
  f.J02 = -a.fx * xc * f.iz * f.iz;
  f.J12 = -a.fy * yc * f.iz * f.iz;

  // rotation of the Gaussian
  const double q0 = a.quats[i], q1 = a.quats[n + i], q2 = a.quats[2 * n + i], q3 = a.quats[3 * n + i];
  f.qinv = 1.0 / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const double w = q0 * f.qinv, x = q1 * f.qinv, y = q2 * f.qinv, z = q3 * f.qinv;
  f.qn[0] = w; f.qn[1] = x; f.qn[2] = y; f.qn[3] = z;
  f.Rq[0] = 1.0 - 2.0 * (y * y + z * z);
  f.Rq[1] = 2.0 * (x * y - w * z);
  f.Rq[2] = 2.0 * (x * z + w * y);
  f.Rq[3] = 2.0 * (x * y + w * z);
  f.Rq[4] = 1.0 - 2.0 * (x * x + z * z);
  f.Rq[5] = 2.0 * (y * z - w * x);
  f.Rq[6] = 2.0 * (x * z - w * y);
  f.Rq[7] = 2.0 * (y * z + w * x);
  f.Rq[8] = 1.0 - 2.0 * (x * x + y * y);
#pragma unroll
  for (int k = 0; k < 3; ++k) f.s[k] = exp((double)a.log_scales[k * n + i]);
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
  f.a = f.TM[0] * f.TM[0] + f.TM[1] * f.TM[1] + f.TM[2] * f.TM[2] + a.eps2d;
  f.b = f.TM[0] * f.TM[3] + f.TM[1] * f.TM[4] + f.TM[2] * f.TM[5];
  f.c = f.TM[3] * f.TM[3] + f.TM[4] * f.TM[4] + f.TM[5] * f.TM[5] + a.eps2d;
  const double det = f.a * f.c - f.b * f.b;
  if (!(det > 0.0)) return false;
  const double idet = 1.0 / det;
  f.A = f.c * idet;
  f.B = -f.b * idet;
  f.C = f.a * idet;

  f.mx = a.fx * f.p[0] * f.iz + a.cx;
  f.my = a.fy * f.p[1] * f.iz + a.cy;
  if (!(fabs(f.mx) < 8388608.0 && fabs(f.my) < 8388608.0)) return false;  // |mean| < 2^23 px

  f.o = 1.0 / (1.0 + exp(-(double)a.opac[i]));
  if (!(f.o >= a.alpha_min)) return false;
  const double hd = 0.5 * (f.a - f.c);
  const double lmax = 0.5 * (f.a + f.c) + sqrt(hd * hd + f.b * f.b);
  const double rr = sqrt(2.0 * log(f.o / a.alpha_min) * lmax);
  f.radius = (int)ceil(fmin(rr * (1.0 + 1e-4) + 1e-3, 4194304.0));

  // colour: view direction from the camera centre C = -R^T t
  const double Cx = -(f.R[0] * f.t[0] + f.R[3] * f.t[1] + f.R[6] * f.t[2]);
  const double Cy = -(f.R[1] * f.t[0] + f.R[4] * f.t[1] + f.R[7] * f.t[2]);
  const double Cz = -(f.R[2] * f.t[0] + f.R[5] * f.t[1] + f.R[8] * f.t[2]);
  const double dx = f.mu[0] - Cx, dy = f.mu[1] - Cy, dz = f.mu[2] - Cz;
  f.dinv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
  f.dhat[0] = dx * f.dinv;
  f.dhat[1] = dy * f.dinv;
  f.dhat[2] = dz * f.dinv;
  constexpr int NB = (DEG + 1) * (DEG + 1);
  double Y[16];
  sh_basis<DEG>(f.dhat[0], f.dhat[1], f.dhat[2], Y);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    double v = 0.5;
#pragma unroll
    for (int k = 0; k < NB; ++k) v += (double)a.sh[(int64_t)(k * 3 + ch) * n + i] * Y[k];
    f.val[ch] = v;
  }
  return true;
}

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project(ProjArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  Fwd f;
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
  int radius = 0, tiles = 0;
  if (forward_one<DEG>(a, i, f)) {
    const double hx = rint(f.mx), hy = rint(f.my);
    r0 = make_float4((float)hx, (float)hy, (float)(f.mx - hx), (float)(f.my - hy));
    r1 = make_float4((float)f.A, (float)f.B, (float)f.C, (float)f.o);
    r2 = make_float4((float)fmax(f.val[0], 0.0), (float)fmax(f.val[1], 0.0), (float)fmax(f.val[2], 0.0),
                     (float)f.z);
    radius = f.radius;
    int tx0, ty0, tx1, ty1;
    if (tile_rect(__fadd_rn(r0.x, r0.z), __fadd_rn(r0.y, r0.w), radius, a.W, a.H, tx0, ty0, tx1, ty1))
      tiles = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
  }
  float4 *dst = (float4 *)(a.rec + i * GS_REC_FLOATS);
  dst[0] = r0;
  dst[1] = r1;
  dst[2] = r2;
  a.radius[i] = radius;
  a.tiles[i] = tiles;
}

// ---------------------------------------------------------------- backward
struct BwdArgs {
  ProjArgs p;
  const float *g2d;  // [n][12] per-Gaussian 2D gradients (first 10 used)
  float *gm, *gl, *gq, *go, *gsh;  // parameter gradients (accumulated)
  double *partials;  // [gridDim.x][12] pose partial sums
};

template <int DEG>
__device__ __forceinline__ void backward_one(const BwdArgs &ba, int64_t i, double pose_acc[12]) {
  const ProjArgs &a = ba.p;
  Fwd f;
  if (!forward_one<DEG>(a, i, f)) return;
  const int64_t n = a.n;
  const float4 *gp4 = (const float4 *)(ba.g2d + i * 12);
  const float4 g0 = gp4[0], g1 = gp4[1], g2 = gp4[2];
  // g0 = (d mean x, d mean y, dA, dB), g1 = (dC, d opacity, d r, d g), g2 = (d b, d z, -, -)
  const double gmx = g0.x, gmy = g0.y, gA = g0.z, gB = g0.w, gC = g1.x, gop = g1.y, gz = g2.y;
  const double gcol[3] = {g1.z, g1.w, g2.x};

  double gmu[3] = {0.0, 0.0, 0.0};

  // colour -> SH coefficients and view direction (no pose path, section 4.3)
  {
    constexpr int NB = (DEG + 1) * (DEG + 1);
    double Y[16], wk[16];
    sh_basis<DEG>(f.dhat[0], f.dhat[1], f.dhat[2], Y);
#pragma unroll
    for (int k = 0; k < NB; ++k) wk[k] = 0.0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      if (!(f.val[ch] > 0.0)) continue;
      const double gv = gcol[ch];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int64_t off = (int64_t)(k * 3 + ch) * n + i;
        ba.gsh[off] += (float)(gv * Y[k]);
        wk[k] += gv * (double)a.sh[off];
      }
    }
    if (DEG > 0) {
      double gx, gy, gzz;
      sh_basis_vjp<DEG>(f.dhat[0], f.dhat[1], f.dhat[2], wk, gx, gy, gzz);
      const double radial = gx * f.dhat[0] + gy * f.dhat[1] + gzz * f.dhat[2];
      gmu[0] += (gx - radial * f.dhat[0]) * f.dinv;
      gmu[1] += (gy - radial * f.dhat[1]) * f.dinv;
      gmu[2] += (gzz - radial * f.dhat[2]) * f.dinv;
    }
  }

  ba.go[i] += (float)(gop * f.o * (1.0 - f.o));

  // conic -> Sigma2: dL/dSigma2 = -Q G Q with G = [[gA, gB/2], [gB/2, gC]]
  const double hB = 0.5 * gB;
  const double QG00 = f.A * gA + f.B * hB, QG01 = f.A * hB + f.B * gC;
  const double QG10 = f.B * gA + f.C * hB, QG11 = f.B * hB + f.C * gC;
  const double S00 = -(QG00 * f.A + QG01 * f.B);
  const double S01 = -(QG00 * f.B + QG01 * f.C);
  const double S11 = -(QG10 * f.B + QG11 * f.C);

  // Sigma2 = TM TM^T: gTM = 2 S TM
  double gTM[6];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    gTM[c] = 2.0 * (S00 * f.TM[c] + S01 * f.TM[3 + c]);
    gTM[3 + c] = 2.0 * (S01 * f.TM[c] + S11 * f.TM[3 + c]);
  }
  // TM = T M: gT = gTM M^T, gM = T^T gTM
  double gT[6], gM[9];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      gT[3 * r + c] = gTM[3 * r] * f.M[3 * c] + gTM[3 * r + 1] * f.M[3 * c + 1] + gTM[3 * r + 2] * f.M[3 * c + 2];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) gM[3 * r + c] = f.T[r] * gTM[c] + f.T[3 + r] * gTM[3 + c];

  // M = Rq diag(s): scales and quaternion
  double gRq[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double gs = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      gRq[3 * r + c] = gM[3 * r + c] * f.s[c];
      gs += gM[3 * r + c] * f.Rq[3 * r + c];
    }
    ba.gl[c * n + i] += (float)(gs * f.s[c]);
  }
  {
    const double w = f.qn[0], x = f.qn[1], y = f.qn[2], z = f.qn[3];
    const double G0 = gRq[0], G1 = gRq[1], G2 = gRq[2], G3 = gRq[3], G4 = gRq[4], G5 = gRq[5], G6 = gRq[6],
                 G7 = gRq[7], G8 = gRq[8];
    const double dw = 2.0 * (z * (G3 - G1) + y * (G2 - G6) + x * (G7 - G5));
    const double dx = 2.0 * (y * (G1 + G3) + z * (G2 + G6) + w * (G7 - G5)) - 4.0 * x * (G4 + G8);
    const double dy = 2.0 * (x * (G1 + G3) + w * (G2 - G6) + z * (G5 + G7)) - 4.0 * y * (G0 + G8);
    const double dz = 2.0 * (w * (G3 - G1) + x * (G2 + G6) + y * (G5 + G7)) - 4.0 * z * (G0 + G4);
    const double proj = dw * w + dx * x + dy * y + dz * z;
    ba.gq[i] += (float)((dw - proj * w) * f.qinv);
    ba.gq[n + i] += (float)((dx - proj * x) * f.qinv);
    ba.gq[2 * n + i] += (float)((dy - proj * y) * f.qinv);
    ba.gq[3 * n + i] += (float)((dz - proj * z) * f.qinv);
  }

  // T = J R: gJ = gT R^T (entries 00, 02, 11, 12), gR from the covariance = J^T gT
  const double gJ00 = gT[0] * f.R[0] + gT[1] * f.R[1] + gT[2] * f.R[2];
  const double gJ02 = gT[0] * f.R[6] + gT[1] * f.R[7] + gT[2] * f.R[8];
  const double gJ11 = gT[3] * f.R[3] + gT[4] * f.R[4] + gT[5] * f.R[5];
  const double gJ12 = gT[3] * f.R[6] + gT[4] * f.R[7] + gT[5] * f.R[8];
  double gR[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    gR[c] = f.J00 * gT[c];
    gR[3 + c] = f.J11 * gT[3 + c];
    gR[6 + c] = f.J02 * gT[c] + f.J12 * gT[3 + c];
  }

  // camera-space point: mean2d, depth and the Jacobian entries
  const double iz2 = f.iz * f.iz;
  double gp0 = gmx * a.fx * f.iz;
  double gp1 = gmy * a.fy * f.iz;
  double gp2 = gz - (gmx * a.fx * f.p[0] + gmy * a.fy * f.p[1]) * iz2 - (gJ00 * a.fx + gJ11 * a.fy) * iz2;
  if (f.clx) {
    gp2 -= gJ02 * f.J02 * f.iz;
  } else {
    gp0 -= gJ02 * a.fx * iz2;
    gp2 += gJ02 * 2.0 * a.fx * f.p[0] * iz2 * f.iz;
  }
  if (f.cly) {
    gp2 -= gJ12 * f.J12 * f.iz;
  } else {
    gp1 -= gJ12 * a.fy * iz2;
    gp2 += gJ12 * 2.0 * a.fy * f.p[1] * iz2 * f.iz;
  }

  // p = R mu + t
  gmu[0] += f.R[0] * gp0 + f.R[3] * gp1 + f.R[6] * gp2;
  gmu[1] += f.R[1] * gp0 + f.R[4] * gp1 + f.R[7] * gp2;
  gmu[2] += f.R[2] * gp0 + f.R[5] * gp1 + f.R[8] * gp2;
  ba.gm[i] += (float)gmu[0];
  ba.gm[n + i] += (float)gmu[1];
  ba.gm[2 * n + i] += (float)gmu[2];

  const double gp[3] = {gp0, gp1, gp2};
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) pose_acc[3 * r + c] += gR[3 * r + c] + gp[r] * f.mu[c];
    pose_acc[9 + r] += gp[r];
  }
}

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project_bwd(BwdArgs ba, const int32_t *tiles) {
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ba.p.n; i += stride)
    if (tiles[i] > 0) backward_one<DEG>(ba, i, acc);

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
__global__ __launch_bounds__(256) void k_pose_reduce(const double *partials, int nparts, const float *pose,
                                                     double *d_pose, double *d_twist) {
  __shared__ double red[12][17];
  const int q = threadIdx.x / 16, r = threadIdx.x % 16;
  if (q < 12) {
    double v = 0.0;
    for (int b = r; b < nparts; b += 16) v += partials[(int64_t)b * 12 + q];
    red[q][r] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double g[12];
    for (int k = 0; k < 12; ++k) {
      double v = 0.0;
      for (int j = 0; j < 16; ++j) v += red[k][j];
      g[k] = v;
    }
    if (d_pose)
      for (int k = 0; k < 12; ++k) d_pose[k] += g[k];
    if (d_twist) {
      double R[9], t[3];
      for (int k = 0; k < 9; ++k) R[k] = pose[k];
      for (int k = 0; k < 3; ++k) t[k] = pose[9 + k];
      // M = dL/dR R^T + dL/dt t^T; rho = dL/dt; phi = (M21 - M12, M02 - M20, M10 - M01)
      double M[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          M[3 * i + j] = g[3 * i] * R[3 * j] + g[3 * i + 1] * R[3 * j + 1] + g[3 * i + 2] * R[3 * j + 2] +
                         g[9 + i] * t[j];
      d_twist[0] += g[9];
      d_twist[1] += g[10];
      d_twist[2] += g[11];
      d_twist[3] += M[7] - M[5];
      d_twist[4] += M[2] - M[6];
      d_twist[5] += M[3] - M[1];
    }
  }
}

__global__ void k_zero_f32(float *p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0f;
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

constexpr int kMaxBwdBlocks = 2048;

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
  (void)n;
  return align_up(sizeof(double) * 12 * kMaxBwdBlocks);
}

gs_status project_bwd(const gs_camera *cam, const gs_raster_params *rp, const gs_gaussians *g,
                      const gs_projected *proj, const float *g2d, gs_gaussians *grads, double *d_pose,
                      double *d_twist, void *ws, hipStream_t s) {
  if (g->n == 0) return GS_OK;
  BwdArgs ba;
  ba.p = make_args(cam, rp, g);
  ba.g2d = g2d;
  ba.gm = grads->means;
  ba.gl = grads->log_scales;
  ba.gq = grads->quats;
  ba.go = grads->opacity_logits;
  ba.gsh = grads->sh;
  ba.partials = (double *)ws;
  int64_t blocks = (g->n + kBlock - 1) / kBlock;
  if (blocks > kMaxBwdBlocks) blocks = kMaxBwdBlocks;
  switch (g->sh_degree) {
    case 0: GS_LAUNCH("project_bwd", k_project_bwd<0>, blocks, kBlock, 0, s, ba, proj->tiles_touched); break;
    case 1: GS_LAUNCH("project_bwd", k_project_bwd<1>, blocks, kBlock, 0, s, ba, proj->tiles_touched); break;
    case 2: GS_LAUNCH("project_bwd", k_project_bwd<2>, blocks, kBlock, 0, s, ba, proj->tiles_touched); break;
    default: GS_LAUNCH("project_bwd", k_project_bwd<3>, blocks, kBlock, 0, s, ba, proj->tiles_touched); break;
  }
  if (d_pose || d_twist)
    GS_LAUNCH("pose_reduce", k_pose_reduce, 1, 256, 0, s, (const double *)ws, (int)blocks, cam->pose, d_pose,
              d_twist);
  return GS_OK;
}

gs_status zero_f32(float *p, int64_t count, hipStream_t s) {
  if (count <= 0) return GS_OK;
  GS_LAUNCH("zero", k_zero_f32, (count + 255) / 256, 256, 0, s, p, count);
  return GS_OK;
}

gs_status validate_camera(const gs_camera *cam, const char *fn) { return check_camera(cam, fn); }
gs_status validate_gaussians(const gs_gaussians *g, const char *fn) { return check_gaussians(g, fn); }

}  // namespace gsmi
