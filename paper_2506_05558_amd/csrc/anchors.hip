// Anchor decisions of the scalable construction (section 4.4): the share of
// active Gaussians that look smaller than a pixel from the previous camera
// (an anchor is created above 40 %), and the opacity scaling that blends
// the Gaussians of the two nearest anchors.  HBM-bound streams; the size
// test is taken in FP64 (at no cost in a 24-byte-per-Gaussian stream).
#include "common.h"

namespace gsmi {
namespace {

// flag[i] = f S_i < tau D_i with S_i = exp(max log-scale), D_i = |mu_i - C|.
// A grid-stride loop over at most kSizeBlocks workgroups, each adding its
// count to *count with one 64-bit integer atomic: atomics on one address from
// the 8 XCDs serialise through the fabric, so their number is kept small
// (integer sums are exact, so the total does not depend on the order).
constexpr int kSizeBlocks = 512;
__global__ __launch_bounds__(256) void k_anchor_sizes(const float *means, const float *log_scales, int64_t n,
                                                      double cx, double cy, double cz, double f, double tau,
                                                      int32_t *flags, unsigned long long *count) {
  unsigned int mine = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double dx = (double)means[i] - cx, dy = (double)means[n + i] - cy, dz = (double)means[2 * n + i] - cz;
    const double D = sqrt(dx * dx + dy * dy + dz * dz);
    const float lmax = fmaxf(fmaxf(log_scales[i], log_scales[n + i]), log_scales[2 * n + i]);
    const bool small = f * exp((double)lmax) < tau * D;
    if (flags) flags[i] = small ? 1 : 0;
    mine += small ? 1u : 0u;
  }
  // block sum: wave sums by xor shuffles, then four waves through LDS
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o, 64);
  __shared__ unsigned int wc[4];
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int c = wc[0] + wc[1] + wc[2] + wc[3];
    if (c) atomicAdd(count, (unsigned long long)c);
  }
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long *p) { *p = 0ull; }

// logit' = logit(w sigmoid(logit)), in FP64
__global__ __launch_bounds__(256) void k_scale_opacity(const float *logits, int64_t n, double w, float *out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double o = 1.0 / (1.0 + exp(-(double)logits[i]));
  const double q = w * o;
  out[i] = (float)(log(q) - log1p(-q));
}

}  // namespace
}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_anchor_sizes(const float *means, const float *log_scales, int64_t n, const float *pose, float f,
                          float tau, int32_t *flags, unsigned long long *count, void *stream) {
  GS_REQUIRE(n >= 0, "gs_anchor_sizes: n < 0");
  GS_REQUIRE(pose && count, "gs_anchor_sizes: NULL pose or count");
  GS_REQUIRE(f > 0.f && tau > 0.f, "gs_anchor_sizes: f and tau must be positive");
  if (n > 0) GS_REQUIRE(means && log_scales, "gs_anchor_sizes: NULL parameter planes");
  // camera centre C = -R^T t of the world -> camera pose (host, FP64)
  double C[3];
  for (int c = 0; c < 3; ++c)
    C[c] = -((double)pose[c] * pose[9] + (double)pose[3 + c] * pose[10] + (double)pose[6 + c] * pose[11]);
  hipStream_t s = (hipStream_t)stream;
  GS_LAUNCH("anchor_sizes", k_zero_u64, 1, 1, 0, s, count);
  if (n == 0) return GS_OK;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, kSizeBlocks);
  GS_LAUNCH("anchor_sizes", k_anchor_sizes, blocks, 256, 0, s, means, log_scales, n, C[0], C[1], C[2], (double)f,
            (double)tau, flags, count);
  return GS_OK;
}

gs_status gs_anchor_blend_weight(float d1, float d2, float overlap, float *w) {
  GS_REQUIRE(w, "gs_anchor_blend_weight: NULL output");
  GS_REQUIRE(d1 >= 0.f && d2 > 0.f && d1 <= d2, "gs_anchor_blend_weight: need 0 <= d1 <= d2, d2 > 0");
  GS_REQUIRE(overlap > 0.f && overlap < 0.5f, "gs_anchor_blend_weight: overlap must be in (0, 0.5)");
  const double r = (double)d1 / (double)d2, o = overlap;
  *w = (float)(r < 1.0 - o ? 1.0 : 1.0 - (r - (1.0 - o)) * 0.5 / o);
  return GS_OK;
}

gs_status gs_scale_opacity(const float *logits, int64_t n, float w, float *out, void *stream) {
  GS_REQUIRE(n >= 0, "gs_scale_opacity: n < 0");
  GS_REQUIRE(w >= 0.f && w <= 1.f, "gs_scale_opacity: w must be in [0, 1]");
  if (n == 0) return GS_OK;
  GS_REQUIRE(logits && out, "gs_scale_opacity: NULL argument");
  GS_LAUNCH("scale_opacity", k_scale_opacity, (unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream, logits, n,
            (double)w, out);
  return GS_OK;
}

}  // extern "C"
