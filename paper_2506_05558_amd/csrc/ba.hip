// Mini bundle adjustment of the initial pose estimation (section 4.1 and the
// appendix on initial pose estimation), as fixed-size problems that each run
// whole on the device from one launch, so that a frame's pose costs three
// launches and the bootstrapping one (all iterations inside, no host round
// trip; graph capture then adds nothing but is possible).
//
// Levenberg-Marquardt with the appendix's schedule: damping lambda starts at
// 1e-5; a step that lowers the cost is kept and lambda divided by nu = 2,
// otherwise the step is dropped and lambda multiplied by 2.  The damped
// normal equations are (H + lambda diag H) delta = -g with H = J^T W J and
// g = J^T W r (a variable whose diagonal is 0 -- none of its observations
// kept -- holds still).  Robustness: the Huber loss on each observation's
// reprojection error e (IRLS weights min(1, delta / e)) and the rejection of
// the observations with e > median + 4 MAD of the errors at the iterate.
// Poses are world->camera [R | t], updated by left perturbations
// exp(xi^) T, xi = (rho, phi); everything is FP64 (the problems are small).
//
// * k_ransac: one wave per hypothesis.  The hypothesis draws its minimal set
//   of m correspondences with the counter-based SplitMix64 stream (draw c is
//   splitmix64(seed + h 2^32 + c) mod K, repeats skipped), runs plain LM from
//   the previous pose on it, and counts the correspondences whose
//   reprojection error is below tau (in front of the camera).
// * k_ransac_best: the hypothesis with most inliers (the first on ties).
// * k_pose_refine: one workgroup: the winner's inliers, then robust LM on
//   them; the median and MAD come from a bitonic sort in LDS.
// * k_bootstrap: one workgroup: focal length (fx = fy), the poses of views
//   1..V-1 (view 0 fixed at the identity) and P points seen in every view,
//   from f0, identity poses and unit depth along view 0's rays; the points
//   are eliminated per point (3x3 blocks) and the reduced camera system
//   (1 + 6 (V - 1) unknowns) is solved by Cholesky; the rejection applies
//   from a given iteration on.
#include <cmath>

#include "common.h"

namespace gsmi {
namespace {

constexpr int kMaxSample = 16;
constexpr int kRefineThreads = 256;
constexpr int kMaxCorr = 8192;          // correspondences of one refinement
constexpr int kMaxViews = 8;            // views of the bootstrapping
constexpr int kMaxObs = 8192;           // views x points of the bootstrapping
constexpr int kMaxCam = 1 + 6 * (kMaxViews - 1);  // 43 camera unknowns

struct Intr {
  double fx, fy, cx, cy;
};

struct PoseD {
  double R[9], t[3];
};

__device__ __forceinline__ void so3_exp(const double w[3], double R[9]) {
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], th = sqrt(th2);
  double a, b;
  if (th < 1e-12) {
    a = 1.0;
    b = 0.5;
  } else {
    a = sin(th) / th;
    b = (1.0 - cos(th)) / th2;
  }
  // R = I + a K + b K^2, K = w^
  const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double k2 = 0.0;
      for (int e = 0; e < 3; ++e) k2 += K[3 * i + e] * K[3 * e + j];
      R[3 * i + j] = (i == j ? 1.0 : 0.0) + a * K[3 * i + j] + b * k2;
    }
}

// T <- exp(xi^) T with the SE(3) V matrix for the translation
__device__ __forceinline__ void se3_left(const PoseD &T, const double xi[6], PoseD &out) {
  const double *rho = xi, *phi = xi + 3;
  double dR[9];
  so3_exp(phi, dR);
  const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2], th = sqrt(th2);
  double b, c;
  if (th < 1e-12) {
    b = 0.5;
    c = 1.0 / 6.0;
  } else {
    b = (1.0 - cos(th)) / th2;
    c = (th - sin(th)) / (th2 * th);
  }
  const double K[9] = {0.0, -phi[2], phi[1], phi[2], 0.0, -phi[0], -phi[1], phi[0], 0.0};
  double Vm[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double k2 = 0.0;
      for (int e = 0; e < 3; ++e) k2 += K[3 * i + e] * K[3 * e + j];
      Vm[3 * i + j] = (i == j ? 1.0 : 0.0) + b * K[3 * i + j] + c * k2;
    }
  for (int i = 0; i < 3; ++i) {
    double tt = 0.0;
    for (int e = 0; e < 3; ++e) tt += dR[3 * i + e] * T.t[e] + Vm[3 * i + e] * rho[e];
    out.t[i] = tt;
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int e = 0; e < 3; ++e) s += dR[3 * i + e] * T.R[3 * e + j];
      out.R[3 * i + j] = s;
    }
  }
}

// camera-frame point, projection, residual
__device__ __forceinline__ void reproject(const PoseD &T, const Intr &in, double X0, double X1, double X2, double p[3],
                                          double uvp[2]) {
  for (int i = 0; i < 3; ++i) p[i] = T.R[3 * i] * X0 + T.R[3 * i + 1] * X1 + T.R[3 * i + 2] * X2 + T.t[i];
  uvp[0] = in.fx * p[0] / p[2] + in.cx;
  uvp[1] = in.fy * p[1] / p[2] + in.cy;
}

// d uv / d xi (2 x 6, row-major) at camera-frame point p
__device__ __forceinline__ void pose_jac(const double p[3], double fx, double fy, double J[12]) {
  const double iz = 1.0 / p[2], iz2 = iz * iz;
  const double a0 = fx * iz, a2 = -fx * p[0] * iz2, b1 = fy * iz, b2 = -fy * p[1] * iz2;
  // [Jp | Jp (-p^)], Jp = [[a0, 0, a2], [0, b1, b2]]
  J[0] = a0, J[1] = 0.0, J[2] = a2;
  J[6] = 0.0, J[7] = b1, J[8] = b2;
  // -p^ = [[0, p2, -p1], [-p2, 0, p0], [p1, -p0, 0]]
  J[3] = a2 * p[1];
  J[4] = a0 * p[2] - a2 * p[0];
  J[5] = -a0 * p[1];
  J[9] = -b1 * p[2] + b2 * p[1];
  J[10] = -b2 * p[0];
  J[11] = b1 * p[0];
}

__device__ __forceinline__ double huber(double e, double d) { return e <= d ? 0.5 * e * e : d * (e - 0.5 * d); }
__device__ __forceinline__ double huber_w(double e, double d) { return e <= d ? 1.0 : d / fmax(e, 1e-300); }

// Cholesky solve of the damped system on the live variables (diag > 0);
// A is n x n row-major (only the lower triangle is read), overwritten.
// Returns false if the damped matrix is not positive definite (no step).
__device__ bool damped_cholesky_solve(double *A, const double *g, double lam, int n, double *step, int stride) {
  // damping and the live set: dead variables get a unit row / column
  for (int i = 0; i < n; ++i) {
    const double d = A[i * stride + i];
    if (d > 0.0) {
      A[i * stride + i] = d + lam * d;
      step[i] = -g[i];
    } else {
      for (int j = 0; j < n; ++j) A[i * stride + j] = A[j * stride + i] = 0.0;
      A[i * stride + i] = 1.0;
      step[i] = 0.0;
    }
  }
  for (int j = 0; j < n; ++j) {
    double s = A[j * stride + j];
    for (int k = 0; k < j; ++k) s -= A[j * stride + k] * A[j * stride + k];
    if (!(s > 0.0)) return false;
    const double l = sqrt(s);
    A[j * stride + j] = l;
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * stride + j];
      for (int k = 0; k < j; ++k) t -= A[i * stride + k] * A[j * stride + k];
      A[i * stride + j] = t / l;
    }
  }
  for (int i = 0; i < n; ++i) {  // L y = b
    double t = step[i];
    for (int k = 0; k < i; ++k) t -= A[i * stride + k] * step[k];
    step[i] = t / A[i * stride + i];
  }
  for (int i = n - 1; i >= 0; --i) {  // L^T x = y
    double t = step[i];
    for (int k = i + 1; k < n; ++k) t -= A[k * stride + i] * step[k];
    step[i] = t / A[i * stride + i];
  }
  return true;
}

// The same for a fixed size N held in registers (fully unrolled).
template <int N>
__device__ __forceinline__ bool damped_cholesky_solve_fixed(double (&A)[N * N], const double *g, double lam,
                                                            double (&step)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double d = A[i * N + i];
    const bool live = d > 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if (!live) A[i * N + j] = A[j * N + i] = 0.0;
    }
    A[i * N + i] = live ? d + lam * d : 1.0;
    step[i] = live ? -g[i] : 0.0;
  }
  bool ok = true;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double s = A[j * N + j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= A[j * N + k] * A[j * N + k];
    ok = ok && s > 0.0;
    const double l = sqrt(fmax(s, 1e-300));
    A[j * N + j] = l;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      double t = A[i * N + j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= A[i * N + k] * A[j * N + k];
      A[i * N + j] = t / l;
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double t = step[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= A[i * N + k] * step[k];
    step[i] = t / A[i * N + i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double t = step[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) t -= A[k * N + i] * step[k];
    step[i] = t / A[i * N + i];
  }
  return ok;
}

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// ---------------------------------------------------------------- RANSAC
struct RansacArgs {
  const float *X, *uv;  // [3][K], [2][K]
  int K;
  Intr in;
  PoseD pose0;
  int m, iters;
  double tau;
  uint64_t seed;
  double *hyp_pose;  // [H][12]
  int32_t *hyp_count;
};

__global__ __launch_bounds__(64) void k_ransac(RansacArgs a) {
  const int h = blockIdx.x, lane = threadIdx.x;
  __shared__ int idx[kMaxSample];
  __shared__ double cand[12];
  const int m = min(a.m, a.K);
  if (lane == 0) {
    int got = 0;
    for (uint64_t c = 0; got < m; ++c) {
      const int j = (int)(splitmix64(a.seed + ((uint64_t)h << 32) + c) % (uint64_t)a.K);
      bool dup = false;
      for (int q = 0; q < got; ++q) dup |= idx[q] == j;
      if (!dup) idx[got++] = j;
    }
  }
  __syncthreads();
  PoseD T = a.pose0;
  double lam = 1e-5;
  double X0 = 0, X1 = 0, X2 = 0, u = 0, v = 0;
  if (lane < m) {
    const int j = idx[lane];
    X0 = a.X[j], X1 = a.X[a.K + j], X2 = a.X[2 * a.K + j];
    u = a.uv[j], v = a.uv[a.K + j];
  }
  for (int it = 0; it < a.iters; ++it) {
    double Hs[21], g[6], cost = 0.0;
#pragma unroll
    for (int q = 0; q < 21; ++q) Hs[q] = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) g[q] = 0.0;
    if (lane < m) {
      double p[3], uvp[2], J[12];
      reproject(T, a.in, X0, X1, X2, p, uvp);
      const double r0 = uvp[0] - u, r1 = uvp[1] - v;
      const double e = sqrt(r0 * r0 + r1 * r1);
      cost = 0.5 * e * e;
      pose_jac(p, a.in.fx, a.in.fy, J);
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        g[i] = J[i] * r0 + J[6 + i] * r1;
#pragma unroll
        for (int j = 0; j <= i; ++j) Hs[i * (i + 1) / 2 + j] = J[i] * J[j] + J[6 + i] * J[6 + j];
      }
    }
#pragma unroll
    for (int q = 0; q < 21; ++q) Hs[q] = wave_sum_d(Hs[q]);
#pragma unroll
    for (int q = 0; q < 6; ++q) g[q] = wave_sum_d(g[q]);
    cost = wave_sum_d(cost);
    if (lane == 0) {
      double A[36], step[6];
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) A[6 * i + j] = A[6 * j + i] = Hs[i * (i + 1) / 2 + j];
      PoseD Tn = T;
      if (damped_cholesky_solve_fixed<6>(A, g, lam, step)) se3_left(T, step, Tn);
      for (int e = 0; e < 9; ++e) cand[e] = Tn.R[e];
      for (int e = 0; e < 3; ++e) cand[9 + e] = Tn.t[e];
    }
    __syncthreads();
    PoseD Tn;
    for (int e = 0; e < 9; ++e) Tn.R[e] = cand[e];
    for (int e = 0; e < 3; ++e) Tn.t[e] = cand[9 + e];
    double cn = 0.0;
    if (lane < m) {
      double p[3], uvp[2];
      reproject(Tn, a.in, X0, X1, X2, p, uvp);
      const double r0 = uvp[0] - u, r1 = uvp[1] - v;
      const double e = sqrt(r0 * r0 + r1 * r1);
      cn = 0.5 * e * e;
    }
    cn = wave_sum_d(cn);
    if (cn < cost) {
      T = Tn;
      lam /= 2.0;
    } else {
      lam *= 2.0;
    }
    __syncthreads();
  }
  int cnt = 0;
  for (int k = lane; k < a.K; k += 64) {
    double p[3], uvp[2];
    reproject(T, a.in, a.X[k], a.X[a.K + k], a.X[2 * a.K + k], p, uvp);
    const double r0 = uvp[0] - a.uv[k], r1 = uvp[1] - a.uv[a.K + k];
    cnt += (p[2] > 0.0 && sqrt(r0 * r0 + r1 * r1) < a.tau) ? 1 : 0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if (lane == 0) {
    for (int e = 0; e < 9; ++e) a.hyp_pose[12 * h + e] = T.R[e];
    for (int e = 0; e < 3; ++e) a.hyp_pose[12 * h + 9 + e] = T.t[e];
    a.hyp_count[h] = cnt;
  }
}

// the first hypothesis with the largest count
__global__ __launch_bounds__(256) void k_ransac_best(const int32_t *count, int H, int32_t *best) {
  __shared__ unsigned long long red[256];
  unsigned long long b = 0;
  for (int h = threadIdx.x; h < H; h += 256) {
    // larger count first, then the lower index: key = count << 32 | (2^32 - 1 - h)
    const unsigned long long key = ((unsigned long long)(uint32_t)count[h] << 32) | (0xffffffffull - (unsigned)h);
    b = key > b ? key : b;
  }
  red[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) best[0] = (int32_t)(0xffffffffull - (red[0] & 0xffffffffull));
}

// -------------------------------------------------- block-wide helpers
// Deterministic block sum of NV doubles per thread (fixed tree order).
template <int NT, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *scratch /* [NT / 64][NV] */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum_d(v[q]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) scratch[w * NV + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int i = 0; i < NT / 64; ++i) s += scratch[i * NV + q];
    v[q] = s;
  }
  __syncthreads();
}

// Bitonic sort ascending of n values (n <= cap, cap a power of two), padded
// with +inf.
template <int NT>
__device__ void bitonic_sort(double *s, int n, int cap) {
  for (int i = n + threadIdx.x; i < cap; i += NT) s[i] = INFINITY;
  __syncthreads();
  int len = 1;
  while (len < n) len <<= 1;
  for (int k = 2; k <= len; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < len; i += NT) {
        const int l = i ^ j;
        if (l > i) {
          const double a = s[i], b = s[l];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            s[i] = b;
            s[l] = a;
          }
        }
      }
      __syncthreads();
    }
}

// median of the n sorted values (numpy's: the mean of the middle two for even n)
__device__ __forceinline__ double sorted_median(const double *s, int n) {
  return (n & 1) ? s[n / 2] : 0.5 * (s[n / 2 - 1] + s[n / 2]);
}

// median + 4 MAD of the errors e[0..n) (sort buffer s of cap entries)
template <int NT>
__device__ double mad_threshold(const double *e, int n, double *s, int cap) {
  if (n == 0) return INFINITY;
  for (int i = threadIdx.x; i < n; i += NT) s[i] = e[i];
  __syncthreads();
  bitonic_sort<NT>(s, n, cap);
  const double med = sorted_median(s, n);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) s[i] = fabs(e[i] - med);
  __syncthreads();
  bitonic_sort<NT>(s, n, cap);
  const double mad = sorted_median(s, n);
  __syncthreads();
  return med + 4.0 * mad;
}

// ------------------------------------------------------- pose refinement
struct RefineArgs {
  const float *X, *uv;
  int K;
  Intr in;
  const double *hyp_pose;
  const int32_t *best;
  double tau, delta;
  int iters;
  int32_t *inliers;   // [K] out: 1 for the winner's inliers
  int32_t *n_inl;     // out
  double *pose_out;   // [12] out (FP64)
  float *pose_out32;  // [12] out
  int32_t *list;      // [kMaxCorr] scratch (global): the inliers' indices
};

__global__ __launch_bounds__(kRefineThreads) void k_pose_refine(RefineArgs a) {
  constexpr int NT = kRefineThreads;
  __shared__ double sbuf[kMaxCorr];
  __shared__ double err[kMaxCorr];
  __shared__ double red[(NT / 64) * 28];
  __shared__ double cand[12];
  __shared__ int nin_s;
  __shared__ int wcnt[NT / 64];
  PoseD T;
  const int hb = a.best[0];
  for (int e = 0; e < 9; ++e) T.R[e] = a.hyp_pose[12 * hb + e];
  for (int e = 0; e < 3; ++e) T.t[e] = a.hyp_pose[12 * hb + 9 + e];
  // the winner's inliers, compacted in index order (per-chunk block scan)
  if (threadIdx.x == 0) nin_s = 0;
  __syncthreads();
  for (int base = 0; base < a.K; base += NT) {
    const int k = base + threadIdx.x;
    int in = 0;
    if (k < a.K) {
      double p[3], uvp[2];
      reproject(T, a.in, a.X[k], a.X[a.K + k], a.X[2 * a.K + k], p, uvp);
      const double r0 = uvp[0] - a.uv[k], r1 = uvp[1] - a.uv[a.K + k];
      in = (p[2] > 0.0 && sqrt(r0 * r0 + r1 * r1) < a.tau) ? 1 : 0;
      a.inliers[k] = in;
    }
    const uint64_t bal = ballot(in != 0);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wcnt[w] = __popcll(bal);
    __syncthreads();
    int before = nin_s;
    for (int i = 0; i < w; ++i) before += wcnt[i];
    if (in) {
      const int pos = before + __popcll(bal & lanemask_lt());
      if (pos < kMaxCorr) a.list[pos] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0)
      for (int i = 0; i < NT / 64; ++i) nin_s += wcnt[i];
    __syncthreads();
  }
  const int n = min(nin_s, kMaxCorr);
  double lam = 1e-5;
  for (int it = 0; it < a.iters; ++it) {
    for (int i = threadIdx.x; i < n; i += NT) {
      const int k = a.list[i];
      double p[3], uvp[2];
      reproject(T, a.in, a.X[k], a.X[a.K + k], a.X[2 * a.K + k], p, uvp);
      const double r0 = uvp[0] - a.uv[k], r1 = uvp[1] - a.uv[a.K + k];
      err[i] = sqrt(r0 * r0 + r1 * r1);
    }
    __syncthreads();
    const double thr = mad_threshold<NT>(err, n, sbuf, kMaxCorr);
    double v[28];
#pragma unroll
    for (int q = 0; q < 28; ++q) v[q] = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) {
      const int k = a.list[i];
      double p[3], uvp[2], J[12];
      reproject(T, a.in, a.X[k], a.X[a.K + k], a.X[2 * a.K + k], p, uvp);
      const double r0 = uvp[0] - a.uv[k], r1 = uvp[1] - a.uv[a.K + k];
      const double e = sqrt(r0 * r0 + r1 * r1);
      if (!(e <= thr)) continue;
      const double w = huber_w(e, a.delta);
      v[27] += huber(e, a.delta);
      pose_jac(p, a.in.fx, a.in.fy, J);
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        v[21 + r] += w * (J[r] * r0 + J[6 + r] * r1);
#pragma unroll
        for (int c = 0; c <= r; ++c) v[r * (r + 1) / 2 + c] += w * (J[r] * J[c] + J[6 + r] * J[6 + c]);
      }
    }
    block_sum<NT, 28>(v, red);
    if (threadIdx.x == 0) {
      double A[36], step[6];
#pragma unroll
      for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) A[6 * r + c] = A[6 * c + r] = v[r * (r + 1) / 2 + c];
      PoseD Tn = T;
      if (damped_cholesky_solve_fixed<6>(A, v + 21, lam, step)) se3_left(T, step, Tn);
      for (int e = 0; e < 9; ++e) cand[e] = Tn.R[e];
      for (int e = 0; e < 3; ++e) cand[9 + e] = Tn.t[e];
    }
    __syncthreads();
    PoseD Tn;
    for (int e = 0; e < 9; ++e) Tn.R[e] = cand[e];
    for (int e = 0; e < 3; ++e) Tn.t[e] = cand[9 + e];
    double cn[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += NT) {
      if (!(err[i] <= thr)) continue;
      const int k = a.list[i];
      double p[3], uvp[2];
      reproject(Tn, a.in, a.X[k], a.X[a.K + k], a.X[2 * a.K + k], p, uvp);
      const double r0 = uvp[0] - a.uv[k], r1 = uvp[1] - a.uv[a.K + k];
      cn[0] += huber(sqrt(r0 * r0 + r1 * r1), a.delta);
    }
    block_sum<NT, 1>(cn, red);
    if (cn[0] < v[27]) {
      T = Tn;
      lam /= 2.0;
    } else {
      lam *= 2.0;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int e = 0; e < 9; ++e) a.pose_out[e] = T.R[e], a.pose_out32[e] = (float)T.R[e];
    for (int e = 0; e < 3; ++e) a.pose_out[9 + e] = T.t[e], a.pose_out32[9 + e] = (float)T.t[e];
    a.n_inl[0] = nin_s;
  }
}

// ---------------------------------------------------------- bootstrapping
constexpr int kBootThreads = 512;
constexpr int kObsStride = 24;  // r (2), w, jf (2), jp (2 x 6), jx (2 x 3)
constexpr int kPtStride = 16 + 2 * 3 * kMaxCam;  // Vinv (9), z (3), gp (3), pad, W [NC][3], Y [3][NC]

struct BootArgs {
  const float *uv;  // [V][2][P]
  int V, P, NC;
  double cx, cy, f0, delta;
  int iters, mad_from;
  double *f_out, *pose_out, *X_out;  // [1], [V][12], [3][P]
  double *trace;                     // [iters][3] (cost, candidate cost, lambda) or NULL
  double *X, *Xc, *obs, *pt;         // workspace
};

// Cholesky solve of the symmetric positive definite n x n system in LDS
// (lower triangle used, overwritten); false if a pivot is not positive.
__device__ bool cholesky_solve(double *A, int n, int stride, const double *b, double *x) {
  for (int j = 0; j < n; ++j) {
    double s = A[j * stride + j];
    for (int k = 0; k < j; ++k) s -= A[j * stride + k] * A[j * stride + k];
    if (!(s > 0.0)) return false;
    const double l = sqrt(s);
    A[j * stride + j] = l;
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * stride + j];
      for (int k = 0; k < j; ++k) t -= A[i * stride + k] * A[j * stride + k];
      A[i * stride + j] = t / l;
    }
  }
  for (int i = 0; i < n; ++i) {
    double t = b[i];
    for (int k = 0; k < i; ++k) t -= A[i * stride + k] * x[k];
    x[i] = t / A[i * stride + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = x[i];
    for (int k = i + 1; k < n; ++k) t -= A[k * stride + i] * x[k];
    x[i] = t / A[i * stride + i];
  }
  return true;
}

// d uv / d cam_c of observation o (c = 0: focal length; 1 + 6 (v - 1) + k:
// pose component k of view v), components u and v; 0 if it does not touch it
__device__ __forceinline__ void cam_jac(const double *ob, int view, int c, double &ju, double &jv) {
  if (c == 0) {
    ju = ob[3], jv = ob[4];
    return;
  }
  const int v = 1 + (c - 1) / 6, k = (c - 1) % 6;
  if (v != view) {
    ju = jv = 0.0;
    return;
  }
  ju = ob[5 + k], jv = ob[11 + k];
}

__global__ __launch_bounds__(kBootThreads) void k_bootstrap(BootArgs a) {
  constexpr int NT = kBootThreads;
  __shared__ double err[kMaxObs];
  __shared__ double sbuf[kMaxObs];
  __shared__ double S[kMaxCam * kMaxCam];
  __shared__ double rhs[kMaxCam], stepc[kMaxCam];
  __shared__ double camR[kMaxViews][9], camt[kMaxViews][3], candR[kMaxViews][9], candt[kMaxViews][3];
  __shared__ double fcur, fcand;
  __shared__ double red[NT / 64];
  __shared__ int solved;
  const int V = a.V, P = a.P, NC = a.NC, NO = V * P;
  const int tid = threadIdx.x;
  // start: f0, identity poses, unit depth along view 0's rays
  if (tid == 0) fcur = a.f0;
  for (int i = tid; i < V * 9; i += NT) camR[i / 9][i % 9] = (i % 9) % 4 == 0 ? 1.0 : 0.0;
  for (int i = tid; i < V * 3; i += NT) camt[i / 3][i % 3] = 0.0;
  for (int p = tid; p < P; p += NT) {
    a.X[p] = ((double)a.uv[p] - a.cx) / a.f0;
    a.X[P + p] = ((double)a.uv[P + p] - a.cy) / a.f0;
    a.X[2 * P + p] = 1.0;
  }
  __syncthreads();
  double lam = 1e-5;
  for (int it = 0; it < a.iters; ++it) {
    const double f = fcur;
    // residuals, errors and Jacobians of every observation
    for (int o = tid; o < NO; o += NT) {
      const int v = o / P, p = o % P;
      double pc[3];
      const double X0 = a.X[p], X1 = a.X[P + p], X2 = a.X[2 * P + p];
      for (int i = 0; i < 3; ++i) pc[i] = camR[v][3 * i] * X0 + camR[v][3 * i + 1] * X1 + camR[v][3 * i + 2] * X2 + camt[v][i];
      const double iz = 1.0 / pc[2];
      const double r0 = f * pc[0] * iz + a.cx - (double)a.uv[(v * 2) * P + p];
      const double r1 = f * pc[1] * iz + a.cy - (double)a.uv[(v * 2 + 1) * P + p];
      err[o] = sqrt(r0 * r0 + r1 * r1);
      double *ob = a.obs + (size_t)o * kObsStride;
      ob[0] = r0, ob[1] = r1;
      ob[3] = pc[0] * iz, ob[4] = pc[1] * iz;
      double J[12];
      pose_jac(pc, f, f, J);
      for (int k = 0; k < 6; ++k) {
        ob[5 + k] = v > 0 ? J[k] : 0.0;
        ob[11 + k] = v > 0 ? J[6 + k] : 0.0;
      }
      // d uv / d X = Jp R
      for (int c = 0; c < 3; ++c) {
        ob[17 + c] = J[0] * camR[v][c] + J[2] * camR[v][6 + c];
        ob[20 + c] = J[7] * camR[v][3 + c] + J[8] * camR[v][6 + c];
      }
    }
    __syncthreads();
    const double thr = it >= a.mad_from ? mad_threshold<NT>(err, NO, sbuf, kMaxObs) : INFINITY;
    double cst[1] = {0.0};
    for (int o = tid; o < NO; o += NT) {
      const double e = err[o];
      const bool keep = e <= thr;
      a.obs[(size_t)o * kObsStride + 2] = keep ? huber_w(e, a.delta) : 0.0;
      cst[0] += keep ? huber(e, a.delta) : 0.0;
    }
    block_sum<NT, 1>(cst, red);
    const double cost = cst[0];
    // per point: V_p, g_p, the damped inverse, z = V^-1 g_p, W rows and Y = V^-1 W^T
    for (int p = tid; p < P; p += NT) {
      double Vp[6] = {0, 0, 0, 0, 0, 0}, gp[3] = {0, 0, 0};  // Vp: 00 01 02 11 12 22
      for (int v = 0; v < V; ++v) {
        const double *ob = a.obs + (size_t)(v * P + p) * kObsStride;
        const double w = ob[2];
        if (w == 0.0) continue;
        const double *ju = ob + 17, *jv = ob + 20;
        Vp[0] += w * (ju[0] * ju[0] + jv[0] * jv[0]);
        Vp[1] += w * (ju[0] * ju[1] + jv[0] * jv[1]);
        Vp[2] += w * (ju[0] * ju[2] + jv[0] * jv[2]);
        Vp[3] += w * (ju[1] * ju[1] + jv[1] * jv[1]);
        Vp[4] += w * (ju[1] * ju[2] + jv[1] * jv[2]);
        Vp[5] += w * (ju[2] * ju[2] + jv[2] * jv[2]);
        for (int c = 0; c < 3; ++c) gp[c] += w * (ju[c] * ob[0] + jv[c] * ob[1]);
      }
      // damped 3x3 with dead components held: invert the live block
      double M[9] = {Vp[0], Vp[1], Vp[2], Vp[1], Vp[3], Vp[4], Vp[2], Vp[4], Vp[5]};
      bool live[3];
      for (int i = 0; i < 3; ++i) {
        live[i] = M[4 * i] > 0.0;
        if (live[i]) M[4 * i] += lam * M[4 * i];
      }
      for (int i = 0; i < 3; ++i)
        if (!live[i])
          for (int j = 0; j < 3; ++j) M[3 * i + j] = M[3 * j + i] = (i == j) ? 1.0 : 0.0;
      const double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                         M[2] * (M[3] * M[7] - M[4] * M[6]);
      double Vi[9] = {(M[4] * M[8] - M[5] * M[7]) / det, (M[2] * M[7] - M[1] * M[8]) / det,
                      (M[1] * M[5] - M[2] * M[4]) / det, (M[5] * M[6] - M[3] * M[8]) / det,
                      (M[0] * M[8] - M[2] * M[6]) / det, (M[2] * M[3] - M[0] * M[5]) / det,
                      (M[3] * M[7] - M[4] * M[6]) / det, (M[1] * M[6] - M[0] * M[7]) / det,
                      (M[0] * M[4] - M[1] * M[3]) / det};
      for (int i = 0; i < 3; ++i)
        if (!live[i])
          for (int j = 0; j < 3; ++j) Vi[3 * i + j] = Vi[3 * j + i] = 0.0;
      double *pp = a.pt + (size_t)p * kPtStride;
      for (int e = 0; e < 9; ++e) pp[e] = Vi[e];
      for (int i = 0; i < 3; ++i) {
        pp[9 + i] = Vi[3 * i] * gp[0] + Vi[3 * i + 1] * gp[1] + Vi[3 * i + 2] * gp[2];
        pp[12 + i] = gp[i];
      }
      double *W = pp + 16, *Y = pp + 16 + 3 * kMaxCam;
      for (int c = 0; c < NC; ++c) {
        double row[3] = {0.0, 0.0, 0.0};
        const int v0 = c == 0 ? 0 : 1 + (c - 1) / 6, v1 = c == 0 ? V : v0 + 1;
        for (int v = v0; v < v1; ++v) {
          const double *ob = a.obs + (size_t)(v * P + p) * kObsStride;
          const double w = ob[2];
          if (w == 0.0) continue;
          double ju, jv;
          cam_jac(ob, v, c, ju, jv);
          for (int e = 0; e < 3; ++e) row[e] += w * (ju * ob[17 + e] + jv * ob[20 + e]);
        }
        for (int e = 0; e < 3; ++e) W[3 * c + e] = row[e];
        for (int e = 0; e < 3; ++e) Y[e * kMaxCam + c] = Vi[3 * e] * row[0] + Vi[3 * e + 1] * row[1] + Vi[3 * e + 2] * row[2];
      }
    }
    __threadfence_block();
    __syncthreads();
    // the reduced camera system S = (U + lam diag U) - sum_p W_p V_p^-1 W_p^T and its
    // right-hand side -g_c + sum_p W_p z_p; a camera unknown without a kept observation holds
    for (int q = tid; q < NC * (NC + 1) / 2; q += NT) {
      int i = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
      while (i * (i + 1) / 2 > q) --i;
      while ((i + 1) * (i + 2) / 2 <= q) ++i;
      const int j = q - i * (i + 1) / 2;
      // U_ij over the observations touching both unknowns
      const int vi = i == 0 ? -1 : 1 + (i - 1) / 6, vj = j == 0 ? -1 : 1 + (j - 1) / 6;
      double u = 0.0;
      if (!(vi >= 0 && vj >= 0 && vi != vj)) {
        const int vv = vi >= 0 ? vi : vj;  // the view both touch, or -1 (focal, focal)
        const int va = vv >= 0 ? vv : 0, vb = vv >= 0 ? vv + 1 : V;
        for (int v = va; v < vb; ++v)
          for (int p = 0; p < P; ++p) {
            const double *ob = a.obs + (size_t)(v * P + p) * kObsStride;
            const double w = ob[2];
            if (w == 0.0) continue;
            double iu, iv, ju, jv;
            cam_jac(ob, v, i, iu, iv);
            cam_jac(ob, v, j, ju, jv);
            u += w * (iu * ju + iv * jv);
          }
      }
      double sch = 0.0;
      for (int p = 0; p < P; ++p) {
        const double *pp = a.pt + (size_t)p * kPtStride;
        const double *W = pp + 16, *Y = pp + 16 + 3 * kMaxCam;
        sch += W[3 * i] * Y[j] + W[3 * i + 1] * Y[kMaxCam + j] + W[3 * i + 2] * Y[2 * kMaxCam + j];
      }
      if (i == j) u += lam * u;
      S[i * kMaxCam + j] = u - sch;
      S[j * kMaxCam + i] = u - sch;
      if (i == j) sbuf[i] = u;  // the damped diagonal of U, for the live test
    }
    for (int i = tid; i < NC; i += NT) {
      double g = 0.0, back = 0.0;
      const int vi = i == 0 ? -1 : 1 + (i - 1) / 6;
      const int va = vi >= 0 ? vi : 0, vb = vi >= 0 ? vi + 1 : V;
      for (int v = va; v < vb; ++v)
        for (int p = 0; p < P; ++p) {
          const double *ob = a.obs + (size_t)(v * P + p) * kObsStride;
          const double w = ob[2];
          if (w == 0.0) continue;
          double iu, iv;
          cam_jac(ob, v, i, iu, iv);
          g += w * (iu * ob[0] + iv * ob[1]);
        }
      for (int p = 0; p < P; ++p) {
        const double *pp = a.pt + (size_t)p * kPtStride;
        back += pp[16 + 3 * i] * pp[9] + pp[16 + 3 * i + 1] * pp[10] + pp[16 + 3 * i + 2] * pp[11];
      }
      rhs[i] = -g + back;
    }
    __syncthreads();
    if (tid == 0) {
      for (int i = 0; i < NC; ++i)
        if (!(sbuf[i] > 0.0)) {  // dead unknown: unit row and column, no step
          for (int j = 0; j < NC; ++j) S[i * kMaxCam + j] = S[j * kMaxCam + i] = 0.0;
          S[i * kMaxCam + i] = 1.0;
          rhs[i] = 0.0;
        }
      solved = cholesky_solve(S, NC, kMaxCam, rhs, stepc) ? 1 : 0;
      if (!solved)
        for (int i = 0; i < NC; ++i) stepc[i] = 0.0;
      fcand = f + stepc[0];
      for (int v = 0; v < V; ++v) {
        PoseD T, Tn;
        for (int e = 0; e < 9; ++e) T.R[e] = camR[v][e];
        for (int e = 0; e < 3; ++e) T.t[e] = camt[v][e];
        Tn = T;
        if (v > 0) se3_left(T, stepc + 1 + 6 * (v - 1), Tn);
        for (int e = 0; e < 9; ++e) candR[v][e] = Tn.R[e];
        for (int e = 0; e < 3; ++e) candt[v][e] = Tn.t[e];
      }
    }
    __syncthreads();
    // points: delta_p = V_p^-1 (-g_p - W_p^T delta_c)
    for (int p = tid; p < P; p += NT) {
      const double *pp = a.pt + (size_t)p * kPtStride;
      double b[3];
      for (int e = 0; e < 3; ++e) {
        double s = -pp[12 + e];
        for (int c = 0; c < NC; ++c) s -= pp[16 + 3 * c + e] * stepc[c];
        b[e] = s;
      }
      for (int e = 0; e < 3; ++e)
        a.Xc[e * P + p] = a.X[e * P + p] + (pp[3 * e] * b[0] + pp[3 * e + 1] * b[1] + pp[3 * e + 2] * b[2]);
    }
    __threadfence_block();
    __syncthreads();
    double cn[1] = {0.0};
    for (int o = tid; o < NO; o += NT) {
      if (a.obs[(size_t)o * kObsStride + 2] == 0.0) continue;
      const int v = o / P, p = o % P;
      const double X0 = a.Xc[p], X1 = a.Xc[P + p], X2 = a.Xc[2 * P + p];
      double pc[3];
      for (int i = 0; i < 3; ++i)
        pc[i] = candR[v][3 * i] * X0 + candR[v][3 * i + 1] * X1 + candR[v][3 * i + 2] * X2 + candt[v][i];
      const double r0 = fcand * pc[0] / pc[2] + a.cx - (double)a.uv[(v * 2) * P + p];
      const double r1 = fcand * pc[1] / pc[2] + a.cy - (double)a.uv[(v * 2 + 1) * P + p];
      cn[0] += huber(sqrt(r0 * r0 + r1 * r1), a.delta);
    }
    block_sum<NT, 1>(cn, red);
    const bool acc = cn[0] < cost;
    if (a.trace && tid == 0) {
      a.trace[3 * it] = cost;
      a.trace[3 * it + 1] = cn[0];
      a.trace[3 * it + 2] = lam;
    }
    if (acc) {
      for (int i = tid; i < 3 * P; i += NT) a.X[i] = a.Xc[i];
      if (tid == 0) fcur = fcand;
      for (int i = tid; i < V * 9; i += NT) camR[i / 9][i % 9] = candR[i / 9][i % 9];
      for (int i = tid; i < V * 3; i += NT) camt[i / 3][i % 3] = candt[i / 3][i % 3];
      lam /= 2.0;
    } else {
      lam *= 2.0;
    }
    __threadfence_block();
    __syncthreads();
  }
  if (tid == 0) a.f_out[0] = fcur;
  for (int i = tid; i < V * 12; i += NT) {
    const int v = i / 12, e = i % 12;
    a.pose_out[i] = e < 9 ? camR[v][e] : camt[v][e - 9];
  }
  for (int i = tid; i < 3 * P; i += NT) a.X_out[i] = a.X[i];
}

}  // namespace
}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_pose_ransac_workspace(int32_t n_hyp, size_t *bytes) {
  GS_REQUIRE(bytes && n_hyp >= 1, "gs_pose_ransac_workspace: bad argument");
  *bytes = align_up(sizeof(double) * 12 * (size_t)n_hyp) + align_up(sizeof(int32_t) * (size_t)n_hyp) +
           align_up(sizeof(int32_t)) + align_up(sizeof(int32_t) * kMaxCorr);
  return GS_OK;
}

gs_status gs_pose_ransac(const float *X, const float *uv, int64_t K, float fx, float fy, float cx, float cy,
                         const double *pose0, int32_t n_hyp, int32_t sample, int32_t hyp_iters, float tau,
                         int32_t refine_iters, float huber_delta, uint64_t seed, int32_t *inliers, int32_t *n_inliers,
                         double *pose_out, float *pose_out32, int32_t *hyp_count, void *ws, size_t ws_bytes,
                         void *stream) {
  GS_REQUIRE(K >= 1 && K <= kMaxCorr, "gs_pose_ransac: K must be in [1, %d]", kMaxCorr);
  GS_REQUIRE(X && uv && pose0 && inliers && n_inliers && pose_out && pose_out32, "gs_pose_ransac: NULL argument");
  GS_REQUIRE(n_hyp >= 1 && n_hyp <= 65536 && sample >= 3 && sample <= kMaxSample && hyp_iters >= 0 &&
                 refine_iters >= 0 && tau > 0.f && huber_delta > 0.f && fx > 0.f && fy > 0.f,
             "gs_pose_ransac: parameter out of range");
  size_t need = 0;
  gs_pose_ransac_workspace(n_hyp, &need);
  if (!ws || ws_bytes < need) {
    set_error("gs_pose_ransac: workspace %zu bytes < %zu", ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  Carve cv(ws);
  double *hyp_pose = cv.take<double>(12 * (size_t)n_hyp);
  int32_t *counts = cv.take<int32_t>((size_t)n_hyp);
  int32_t *best = cv.take<int32_t>(1);
  int32_t *list = cv.take<int32_t>(kMaxCorr);
  PoseD P0;
  for (int e = 0; e < 9; ++e) P0.R[e] = pose0[e];
  for (int e = 0; e < 3; ++e) P0.t[e] = pose0[9 + e];
  const Intr in{fx, fy, cx, cy};
  hipStream_t s = (hipStream_t)stream;
  RansacArgs ra{X, uv, (int)K, in, P0, sample, hyp_iters, (double)tau, seed, hyp_pose, counts};
  GS_LAUNCH("pose_ransac", k_ransac, n_hyp, 64, 0, s, ra);
  GS_LAUNCH("pose_ransac", k_ransac_best, 1, 256, 0, s, counts, n_hyp, best);
  RefineArgs rf{X,       uv,        (int)K,   in,         hyp_pose, best, (double)tau, (double)huber_delta,
                refine_iters, inliers, n_inliers, pose_out, pose_out32, list};
  GS_LAUNCH("pose_refine", k_pose_refine, 1, kRefineThreads, 0, s, rf);
  if (hyp_count)
    GS_CHECK_HIP(hipMemcpyAsync(hyp_count, counts, sizeof(int32_t) * n_hyp, hipMemcpyDeviceToDevice, s),
                 "gs_pose_ransac counts");
  return GS_OK;
}

gs_status gs_ba_bootstrap_workspace(int32_t n_views, int32_t n_points, size_t *bytes) {
  GS_REQUIRE(bytes && n_views >= 2 && n_views <= kMaxViews && n_points >= 1 && n_views * n_points <= kMaxObs,
             "gs_ba_bootstrap_workspace: need 2 <= views <= %d, points >= 1, views x points <= %d", kMaxViews,
             kMaxObs);
  *bytes = 2 * align_up(sizeof(double) * 3 * (size_t)n_points) +
           align_up(sizeof(double) * kObsStride * (size_t)n_views * n_points) +
           align_up(sizeof(double) * kPtStride * (size_t)n_points);
  return GS_OK;
}

gs_status gs_ba_bootstrap(const float *uv, int32_t n_views, int32_t n_points, int32_t width, int32_t height,
                          int32_t iters, int32_t mad_from, float huber_delta, double *f_out, double *pose_out,
                          double *X_out, double *trace, void *ws, size_t ws_bytes, void *stream) {
  size_t need = 0;
  gs_status st = gs_ba_bootstrap_workspace(n_views, n_points, &need);
  if (st != GS_OK) return st;
  GS_REQUIRE(uv && f_out && pose_out && X_out, "gs_ba_bootstrap: NULL argument");
  GS_REQUIRE(width > 0 && height > 0 && iters >= 0 && huber_delta > 0.f, "gs_ba_bootstrap: parameter out of range");
  if (!ws || ws_bytes < need) {
    set_error("gs_ba_bootstrap: workspace %zu bytes < %zu", ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  Carve cv(ws);
  BootArgs a;
  a.uv = uv;
  a.V = n_views;
  a.P = n_points;
  a.NC = 1 + 6 * (n_views - 1);
  a.cx = width / 2.0;
  a.cy = height / 2.0;
  a.f0 = 0.7 * width;
  a.delta = huber_delta;
  a.iters = iters;
  a.mad_from = mad_from < 0 ? iters / 2 : mad_from;
  a.f_out = f_out;
  a.pose_out = pose_out;
  a.X_out = X_out;
  a.trace = trace;
  a.X = cv.take<double>(3 * (size_t)n_points);
  a.Xc = cv.take<double>(3 * (size_t)n_points);
  a.obs = cv.take<double>(kObsStride * (size_t)n_views * n_points);
  a.pt = cv.take<double>(kPtStride * (size_t)n_points);
  GS_LAUNCH("ba_bootstrap", k_bootstrap, 1, kBootThreads, 0, (hipStream_t)stream, a);
  return GS_OK;
}

}  // extern "C"
