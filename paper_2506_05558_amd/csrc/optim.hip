// Photometric loss, Adam and the 6D pose parametrisation used by the joint
// pose + Gaussian optimisation (section 4.3).
#include "common.h"

namespace gsmi {
namespace {

constexpr int kLossBlock = 256;
constexpr int kLossMaxBlocks = 1024;

__global__ __launch_bounds__(kLossBlock) void k_loss_l1(const float *img, const float *tgt, int64_t count,
                                                        float scale, float *grad, double *partials) {
  double s1 = 0.0, s2 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kLossBlock;
  for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < count; i += stride) {
    const float d = img[i] - tgt[i];
    s1 += fabs((double)d);
    s2 += (double)d * (double)d;
    if (grad) grad[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_down(s1, off, 64);
    s2 += __shfl_down(s2, off, 64);
  }
  __shared__ double red[kLossBlock / 64][2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[w][0] = s1;
    red[w][1] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < kLossBlock / 64; ++k) {
      a += red[k][0];
      b += red[k][1];
    }
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = b;
  }
}

__global__ __launch_bounds__(64) void k_loss_final(const double *partials, int nparts, double *sums) {
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 64) {
    a += partials[2 * k];
    b += partials[2 * k + 1];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  if (threadIdx.x == 0) {
    sums[0] = a;
    sums[1] = b;
  }
}

// Streaming 16-byte accesses that bypass cache retention: each element of
// the optimiser state is touched once per step.
typedef float v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_stream(const float *q) {
  const v4f x = __builtin_nontemporal_load((const v4f *)q);
  return make_float4(x.x, x.y, x.z, x.w);
}
__device__ __forceinline__ void store_stream(float *q, const float4 &x) {
  __builtin_nontemporal_store((v4f){x.x, x.y, x.z, x.w}, (v4f *)q);
}

// The Adam update (adam_one), four consecutive elements of one plane per
// lane (16-byte non-temporal loads and stores); used when the planes hold a
// multiple of four elements and every array is 16-byte aligned.  A quad with
// no visible Gaussian is not touched; in a partly visible quad the hidden
// elements are stored back unchanged.
// RATE: lr_scale[j] multiplies the rate of every element of Gaussian j.
template <bool RATE>
__global__ __launch_bounds__(256) void k_adam4(float *p, const float *g, float *m, float *v, float lr, float b1,
                                               float b2, float eps, float c1, float c2, const int32_t *visible,
                                               const float *lr_scale, int64_t n_stride) {
  const int64_t j = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (j >= n_stride) return;
  const int64_t i = (int64_t)blockIdx.y * n_stride + j;
  const int4 vis = visible ? *(const int4 *)(visible + j) : make_int4(1, 1, 1, 1);
  if ((vis.x | vis.y | vis.z | vis.w) == 0) return;
  float4 R = make_float4(lr, lr, lr, lr);
  if (RATE) {
    const float4 S = *(const float4 *)(lr_scale + j);
    R = make_float4(lr * S.x, lr * S.y, lr * S.z, lr * S.w);
  }
  const float4 G = load_stream(g + i);
  float4 M = load_stream(m + i), V = load_stream(v + i), P = load_stream(p + i);
  if (vis.x) adam_one(G.x, M.x, V.x, P.x, R.x, b1, b2, eps, c1, c2);
  if (vis.y) adam_one(G.y, M.y, V.y, P.y, R.y, b1, b2, eps, c1, c2);
  if (vis.z) adam_one(G.z, M.z, V.z, P.z, R.z, b1, b2, eps, c1, c2);
  if (vis.w) adam_one(G.w, M.w, V.w, P.w, R.w, b1, b2, eps, c1, c2);
  store_stream(m + i, M);
  store_stream(v + i, V);
  store_stream(p + i, P);
}

// Grid (plane chunks, planes): element i = plane * n_stride + j belongs to
// Gaussian j, so the visibility test and the rate need no division.
__global__ __launch_bounds__(256) void k_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr,
                                              float b1, float b2, float eps, float c1, float c2,
                                              const int32_t *visible, const float *lr_scale, int64_t n_stride) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = (int64_t)blockIdx.y * n_stride + j;
  if (j >= n_stride || i >= count) return;
  if (visible && !visible[j]) return;
  float mi = m[i], vi = v[i], pi = p[i];
  adam_one(g[i], mi, vi, pi, lr_scale ? lr * lr_scale[j] : lr, b1, b2, eps, c1, c2);
  m[i] = mi;
  v[i] = vi;
  p[i] = pi;
}

// The per-Gaussian rates after a sparse step: each Gaussian it processed
// is multiplied by the decay ratio.
__global__ __launch_bounds__(256) void k_lr_decay(float *lr_scale, const int32_t *visible, int64_t n, float decay) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n || (visible && !visible[i])) return;
  lr_scale[i] *= decay;
}

// R's columns from the two 3-vectors of the 6D representation.
__device__ void gram_schmidt(const float *x, double b1[3], double b2[3], double b3[3], double &n1, double &n2,
                             double u2[3]) {
  const double a1[3] = {x[0], x[1], x[2]}, a2[3] = {x[3], x[4], x[5]};
  n1 = sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
  for (int k = 0; k < 3; ++k) b1[k] = a1[k] / n1;
  const double d = b1[0] * a2[0] + b1[1] * a2[1] + b1[2] * a2[2];
  for (int k = 0; k < 3; ++k) u2[k] = a2[k] - d * b1[k];
  n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  for (int k = 0; k < 3; ++k) b2[k] = u2[k] / n2;
  b3[0] = b1[1] * b2[2] - b1[2] * b2[1];
  b3[1] = b1[2] * b2[0] - b1[0] * b2[2];
  b3[2] = b1[0] * b2[1] - b1[1] * b2[0];
}

__global__ void k_pose_from_6d(const float *x, float *pose, int nv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const float *xi = x + 9 * i;
  double b1[3], b2[3], b3[3], n1, n2, u2[3];
  gram_schmidt(xi, b1, b2, b3, n1, n2, u2);
  float *P = pose + 12 * i;
  for (int r = 0; r < 3; ++r) {
    P[3 * r] = (float)b1[r];
    P[3 * r + 1] = (float)b2[r];
    P[3 * r + 2] = (float)b3[r];
  }
  for (int k = 0; k < 3; ++k) P[9 + k] = xi[6 + k];
}

// Adjoint of the Gram-Schmidt map: from dL/dR (columns g1, g2, g3) to dL/da1, dL/da2.
__global__ void k_pose_6d_bwd(const float *x, const double *dpose, float *dx, int nv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const float *xi = x + 9 * i;
  const double *G = dpose + 12 * i;
  double b1[3], b2[3], b3[3], n1, n2, u2[3];
  gram_schmidt(xi, b1, b2, b3, n1, n2, u2);
  double g1[3], g2[3], g3[3];
  for (int r = 0; r < 3; ++r) {
    g1[r] = G[3 * r];
    g2[r] = G[3 * r + 1];
    g3[r] = G[3 * r + 2];
  }
  // b3 = b1 x b2: dL/db1 += b2 x g3, dL/db2 += g3 x b1
  g1[0] += b2[1] * g3[2] - b2[2] * g3[1];
  g1[1] += b2[2] * g3[0] - b2[0] * g3[2];
  g1[2] += b2[0] * g3[1] - b2[1] * g3[0];
  g2[0] += g3[1] * b1[2] - g3[2] * b1[1];
  g2[1] += g3[2] * b1[0] - g3[0] * b1[2];
  g2[2] += g3[0] * b1[1] - g3[1] * b1[0];
  // b2 = u2 / |u2|: dL/du2 = (g2 - b2 (b2.g2)) / |u2|
  const double p2 = b2[0] * g2[0] + b2[1] * g2[1] + b2[2] * g2[2];
  double gu[3];
  for (int k = 0; k < 3; ++k) gu[k] = (g2[k] - b2[k] * p2) / n2;
  // u2 = a2 - (b1.a2) b1: dL/da2 = gu - b1 (b1.gu); dL/db1 += -(b1.a2) gu - (b1.gu) a2
  const double a2[3] = {xi[3], xi[4], xi[5]};
  const double bgu = b1[0] * gu[0] + b1[1] * gu[1] + b1[2] * gu[2];
  const double ba2 = b1[0] * a2[0] + b1[1] * a2[1] + b1[2] * a2[2];
  for (int k = 0; k < 3; ++k) {
    dx[9 * i + 3 + k] += (float)(gu[k] - b1[k] * bgu);
    g1[k] += -ba2 * gu[k] - bgu * a2[k];
  }
  // b1 = a1 / |a1|
  const double p1 = b1[0] * g1[0] + b1[1] * g1[1] + b1[2] * g1[2];
  for (int k = 0; k < 3; ++k) dx[9 * i + k] += (float)((g1[k] - b1[k] * p1) / n1);
  for (int k = 0; k < 3; ++k) dx[9 * i + 6 + k] += (float)G[9 + k];
}

__global__ void k_zero_words(uint32_t *p, int64_t words) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0u;
}

__global__ void k_zero_bytes(uint8_t *p, int64_t bytes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < bytes) p[i] = 0u;
}

__global__ void k_mark_visible(const int32_t *tiles, int64_t n, int32_t *mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && tiles[i] > 0) mask[i] = 1;
}

}  // namespace
}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_loss_workspace(int64_t count, size_t *bytes) {
  GS_REQUIRE(bytes && count >= 0, "gs_loss_workspace: bad argument");
  *bytes = align_up(sizeof(double) * 2 * kLossMaxBlocks);
  return GS_OK;
}

gs_status gs_loss_l1(const float *image, const float *target, int64_t count, float grad_scale, float *dL_dimage,
                     double *sums, void *ws, size_t ws_bytes, void *stream) {
  GS_REQUIRE(count >= 0 && sums, "gs_loss_l1: bad argument");
  if (count > 0) GS_REQUIRE(image && target, "gs_loss_l1: NULL image or target");
  size_t need = 0;
  gs_loss_workspace(count, &need);
  if (ws_bytes < need || !ws) {
    set_error("gs_loss_l1: workspace %zu bytes < %zu", ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  int64_t blocks = (count + kLossBlock - 1) / kLossBlock;
  if (blocks > kLossMaxBlocks) blocks = kLossMaxBlocks;
  if (blocks < 1) blocks = 1;
  GS_LAUNCH("loss_l1", k_loss_l1, blocks, kLossBlock, 0, s, image, target, count, grad_scale, dL_dimage,
            (double *)ws);
  GS_LAUNCH("loss_final", k_loss_final, 1, 64, 0, s, (const double *)ws, (int)blocks, sums);
  return GS_OK;
}

gs_status gs_adam_step(float *param, const float *grad, float *m, float *v, int64_t count, float lr, float beta1,
                       float beta2, float eps, int32_t step, const int32_t *visible, const float *lr_scale,
                       int64_t n_stride, void *stream) {
  GS_REQUIRE(count >= 0 && step >= 1, "gs_adam_step: bad count or step");
  GS_REQUIRE(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f, "gs_adam_step: bad betas");
  if (count == 0) return GS_OK;
  GS_REQUIRE(param && grad && m && v, "gs_adam_step: NULL argument");
  if (visible || lr_scale)
    GS_REQUIRE(n_stride > 0, "gs_adam_step: n_stride must be positive with a visibility mask or per-Gaussian rates");
  const float c1 = adam_bias(beta1, step), c2 = adam_bias(beta2, step);
  // without a mask or rates the whole array is one "plane"
  const int64_t stride = visible || lr_scale ? n_stride : count;
  const int64_t planes = (count + stride - 1) / stride;
  GS_REQUIRE(planes <= 65535, "gs_adam_step: count / n_stride exceeds 65535 planes");
  const auto a16 = [](const void *q) { return ((uintptr_t)q & 15u) == 0; };
  if (stride % 4 == 0 && count % stride == 0 && a16(param) && a16(grad) && a16(m) && a16(v) &&
      (!visible || a16(visible)) && (!lr_scale || a16(lr_scale))) {
    const dim3 grid((unsigned)((stride / 4 + 255) / 256), (unsigned)planes);
    if (lr_scale)
      GS_LAUNCH("adam", k_adam4<true>, grid, 256, 0, (hipStream_t)stream, param, grad, m, v, lr, beta1, beta2, eps,
                c1, c2, visible, lr_scale, stride);
    else
      GS_LAUNCH("adam", k_adam4<false>, grid, 256, 0, (hipStream_t)stream, param, grad, m, v, lr, beta1, beta2, eps,
                c1, c2, visible, lr_scale, stride);
    return GS_OK;
  }
  const dim3 grid((unsigned)((stride + 255) / 256), (unsigned)planes);
  GS_LAUNCH("adam", k_adam, grid, 256, 0, (hipStream_t)stream, param, grad, m, v, count, lr, beta1, beta2, eps, c1,
            c2, visible, lr_scale, stride);
  return GS_OK;
}

gs_status gs_lr_decay(float *lr_scale, const int32_t *visible, int64_t n, float decay, void *stream) {
  GS_REQUIRE(n >= 0, "gs_lr_decay: n < 0");
  GS_REQUIRE(decay > 0.f && decay <= 1.f, "gs_lr_decay: decay must be in (0, 1]");
  if (n == 0) return GS_OK;
  GS_REQUIRE(lr_scale, "gs_lr_decay: NULL rates");
  GS_LAUNCH("lr_decay", k_lr_decay, (unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream, lr_scale, visible, n,
            decay);
  return GS_OK;
}

gs_status gs_zero(void *ptr, size_t bytes, void *stream) {
  if (bytes == 0) return GS_OK;
  GS_REQUIRE(ptr, "gs_zero: NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  if (((uintptr_t)ptr % 4) == 0 && bytes % 4 == 0) {
    const int64_t words = (int64_t)(bytes / 4);
    GS_LAUNCH("zero", k_zero_words, (words + 255) / 256, 256, 0, s, (uint32_t *)ptr, words);
  } else {
    GS_LAUNCH("zero", k_zero_bytes, ((int64_t)bytes + 255) / 256, 256, 0, s, (uint8_t *)ptr, (int64_t)bytes);
  }
  return GS_OK;
}

gs_status gs_mark_visible(const int32_t *tiles_touched, int64_t n, int32_t *mask, void *stream) {
  GS_REQUIRE(n >= 0, "gs_mark_visible: n < 0");
  if (n == 0) return GS_OK;
  GS_REQUIRE(tiles_touched && mask, "gs_mark_visible: NULL argument");
  GS_LAUNCH("mark_visible", k_mark_visible, (n + 255) / 256, 256, 0, (hipStream_t)stream, tiles_touched, n, mask);
  return GS_OK;
}

gs_status gs_pose_from_6d(const float *x, float *pose, int32_t n_views, void *stream) {
  GS_REQUIRE(n_views >= 0, "gs_pose_from_6d: n_views < 0");
  if (n_views == 0) return GS_OK;
  GS_REQUIRE(x && pose, "gs_pose_from_6d: NULL argument");
  GS_LAUNCH("pose_6d", k_pose_from_6d, (n_views + 63) / 64, 64, 0, (hipStream_t)stream, x, pose, n_views);
  return GS_OK;
}

gs_status gs_pose_6d_bwd(const float *x, const double *dL_dpose, float *dL_dx, int32_t n_views, void *stream) {
  GS_REQUIRE(n_views >= 0, "gs_pose_6d_bwd: n_views < 0");
  if (n_views == 0) return GS_OK;
  GS_REQUIRE(x && dL_dpose && dL_dx, "gs_pose_6d_bwd: NULL argument");
  GS_LAUNCH("pose_6d_bwd", k_pose_6d_bwd, (n_views + 63) / 64, 64, 0, (hipStream_t)stream, x, dL_dpose, dL_dx,
            n_views);
  return GS_OK;
}

}  // extern "C"
