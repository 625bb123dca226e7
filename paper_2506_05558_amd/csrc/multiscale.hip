// Multi-scale training helpers of the joint optimisation (section 4.3):
// the coarse-to-fine image pyramid (a newly added image first trains at
// 2^l downsampling, one level less every five iterations) and opacity
// culling (Gaussians whose opacity fell below a threshold are removed, as
// in 3DGS).  All kernels here are HBM-bound streams.
#include "common.h"

namespace gsmi {
namespace {

// Coarse pixel (x, y) of plane c = mean of the S x S fine block at
// (S x, S y).  One lane per coarse pixel: a wave reads S rows of 64 S
// consecutive floats, 16-byte loads where the rows allow them (VEC).
template <int S, bool VEC>
__global__ __launch_bounds__(256) void k_downsample(const float *in, int W, int H, int Wc, int Hc, int64_t total,
                                                    float *out) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= total) return;
  const int x = (int)(o % Wc);
  const int64_t r = o / Wc;
  const int y = (int)(r % Hc);
  const int64_t c = r / Hc;
  const float *src = in + (c * H + (int64_t)S * y) * W + (int64_t)S * x;
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < S; ++i) {
    const float *row = src + (int64_t)i * W;
    if (VEC) {
#pragma unroll
      for (int j = 0; j < S; j += 4) {
        const float4 q = *(const float4 *)(row + j);
        acc += q.x;
        acc += q.y;
        acc += q.z;
        acc += q.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < S; ++j) acc += row[j];
    }
  }
  out[o] = acc * (1.0f / (float)(S * S));  // exact: a power of two
}

__global__ __launch_bounds__(256) void k_keep_flags(const float *logits, int64_t n, float thr, uint32_t *flags) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) flags[i] = logits[i] >= thr ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_keep_index(const uint32_t *flags, const uint32_t *pos, int64_t n,
                                                    int32_t *index) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && flags[i]) index[pos[i]] = (int32_t)i;
}

// Grid (column chunks, planes).  An index outside [0, n_src) gives 0.
__global__ __launch_bounds__(256) void k_gather_planes(const float *src, int64_t n_src, const int32_t *index,
                                                       int64_t m, float *dst) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= m) return;
  const int64_t p = blockIdx.y;
  const int32_t k = index[j];
  dst[p * m + j] = (k >= 0 && k < n_src) ? src[p * n_src + k] : 0.0f;
}

template <int S>
gs_status launch_downsample(const float *in, int W, int H, int Wc, int Hc, int64_t total, float *out,
                            hipStream_t s) {
  const unsigned grid = (unsigned)((total + 255) / 256);
  const bool vec = S % 4 == 0 && W % 4 == 0 && ((uintptr_t)in & 15u) == 0;
  if constexpr (S % 4 == 0) {
    if (vec) {
      GS_LAUNCH("downsample", (k_downsample<S, true>), grid, 256, 0, s, in, W, H, Wc, Hc, total, out);
      return GS_OK;
    }
  }
  GS_LAUNCH("downsample", (k_downsample<S, false>), grid, 256, 0, s, in, W, H, Wc, Hc, total, out);
  return GS_OK;
}

struct PruneLayout {
  uint32_t *flags, *pos, *total;
  void *scan_ws;
  size_t bytes;
};

PruneLayout prune_layout(void *ws, int64_t n) {
  Carve cv(ws);
  PruneLayout L;
  L.flags = cv.take<uint32_t>((size_t)n);
  L.pos = cv.take<uint32_t>((size_t)n);
  L.total = cv.take<uint32_t>(1);
  L.scan_ws = cv.take<char>(scan_workspace(n));
  L.bytes = cv.off;
  return L;
}

}  // namespace

gs_status validate_camera(const gs_camera *cam, const char *fn);

}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_downsample(const float *in, int32_t channels, int32_t width, int32_t height, int32_t level, float *out,
                        void *stream) {
  GS_REQUIRE(channels >= 1 && width >= 1 && height >= 1, "gs_downsample: bad sizes");
  GS_REQUIRE(level >= 0 && level <= 4, "gs_downsample: level must be 0..4");
  const int Wc = width >> level, Hc = height >> level;
  GS_REQUIRE(Wc >= 1 && Hc >= 1, "gs_downsample: image smaller than one 2^level block");
  GS_REQUIRE(in && out, "gs_downsample: NULL argument");
  const int64_t total = (int64_t)channels * Wc * Hc;
  hipStream_t s = (hipStream_t)stream;
  switch (level) {
    case 0: return launch_downsample<1>(in, width, height, Wc, Hc, total, out, s);
    case 1: return launch_downsample<2>(in, width, height, Wc, Hc, total, out, s);
    case 2: return launch_downsample<4>(in, width, height, Wc, Hc, total, out, s);
    case 3: return launch_downsample<8>(in, width, height, Wc, Hc, total, out, s);
    default: return launch_downsample<16>(in, width, height, Wc, Hc, total, out, s);
  }
}

gs_status gs_camera_level(const gs_camera *cam, int32_t level, gs_camera *out) {
  gs_status st = validate_camera(cam, "gs_camera_level");
  if (st != GS_OK) return st;
  GS_REQUIRE(out, "gs_camera_level: NULL output");
  GS_REQUIRE(level >= 0 && level <= 4, "gs_camera_level: level must be 0..4");
  GS_REQUIRE((cam->width >> level) >= 1 && (cam->height >> level) >= 1,
             "gs_camera_level: image smaller than one 2^level block");
  const double s = (double)(1 << level);
  gs_camera c = *cam;
  c.width = cam->width >> level;
  c.height = cam->height >> level;
  c.fx = (float)((double)cam->fx / s);
  c.fy = (float)((double)cam->fy / s);
  c.cx = (float)(((double)cam->cx + 0.5) / s - 0.5);
  c.cy = (float)(((double)cam->cy + 0.5) / s - 0.5);
  *out = c;
  return GS_OK;
}

gs_status gs_prune_workspace(int64_t n, size_t *bytes) {
  GS_REQUIRE(bytes && n >= 0 && n <= INT32_MAX, "gs_prune_workspace: bad argument");
  *bytes = prune_layout(nullptr, n).bytes;
  return GS_OK;
}

gs_status gs_prune_opacity(const float *opacity_logits, int64_t n, float min_opacity, int32_t *keep_index,
                           int64_t *n_keep, void *ws, size_t ws_bytes, void *stream) {
  GS_REQUIRE(n >= 0 && n <= INT32_MAX, "gs_prune_opacity: n out of range");
  GS_REQUIRE(min_opacity > 0.f && min_opacity < 1.f, "gs_prune_opacity: min_opacity must be in (0, 1)");
  GS_REQUIRE(n_keep, "gs_prune_opacity: NULL n_keep");
  *n_keep = 0;
  if (n == 0) return GS_OK;
  GS_REQUIRE(opacity_logits && keep_index, "gs_prune_opacity: NULL argument");
  PruneLayout L = prune_layout(ws, n);
  if (!ws || ws_bytes < L.bytes) {
    set_error("gs_prune_opacity: workspace %zu bytes < %zu", ws_bytes, L.bytes);
    return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  const float thr = (float)log((double)min_opacity / (1.0 - (double)min_opacity));
  const unsigned grid = (unsigned)((n + 255) / 256);
  GS_LAUNCH("prune_flags", k_keep_flags, grid, 256, 0, s, opacity_logits, n, thr, L.flags);
  gs_status st = scan_exclusive(L.flags, L.pos, n, L.total, L.scan_ws, s);
  if (st != GS_OK) return st;
  GS_LAUNCH("prune_index", k_keep_index, grid, 256, 0, s, L.flags, L.pos, n, keep_index);
  uint32_t kept = 0;
  GS_CHECK_HIP(hipMemcpyAsync(&kept, L.total, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read kept count");
  GS_CHECK_HIP(hipStreamSynchronize(s), "sync kept count");
  *n_keep = kept;
  return GS_OK;
}

gs_status gs_gather_planes(const float *src, int64_t n_src, int32_t planes, const int32_t *index, int64_t m,
                           float *dst, void *stream) {
  GS_REQUIRE(n_src >= 0 && m >= 0 && planes >= 0 && planes <= 65535, "gs_gather_planes: bad sizes");
  if (m == 0 || planes == 0) return GS_OK;
  GS_REQUIRE(src && index && dst, "gs_gather_planes: NULL argument");
  GS_REQUIRE(src != dst, "gs_gather_planes: src and dst must not be the same buffer");
  const dim3 grid((unsigned)((m + 255) / 256), (unsigned)planes);
  GS_LAUNCH("gather_planes", k_gather_planes, grid, 256, 0, (hipStream_t)stream, src, n_src, index, m, dst);
  return GS_OK;
}

}  // extern "C"
