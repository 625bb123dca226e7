// Multi-scale training helpers of the joint optimisation (section 4.3):
// the coarse-to-fine image pyramid (a newly added image first trains at
// 2^l downsampling, one level less every five iterations) and opacity
// culling (Gaussians whose opacity fell below a threshold are removed, as
// in 3DGS).  All kernels here are HBM-bound streams.
#include "common.h"

namespace gsmi {
namespace {

// Coarse pixel (x, y) of plane c = mean of the S x S fine block at
// (S x, S y), summed in row order.  VEC (rows a multiple of 4 floats,
// 16-byte aligned): a lane reads one 16-byte segment per row and makes
// PX = max(1, 4 / S) neighbouring coarse pixels, so a wave reads 64
// consecutive segments of each row it touches; otherwise one lane per
// coarse pixel with 4-byte loads.
template <int S, bool VEC>
__global__ __launch_bounds__(256) void k_downsample(const float *in, int W, int H, int Wc, int Hc, int64_t total,
                                                    float *out) {
  constexpr int PX = VEC && S < 4 ? 4 / S : 1;
  const int64_t o = ((int64_t)blockIdx.x * 256 + threadIdx.x) * PX;
  if (o >= total) return;
  const int x = (int)(o % Wc);
  const int64_t r = o / Wc;
  const int y = (int)(r % Hc);
  const int64_t c = r / Hc;
  const float *src = in + (c * H + (int64_t)S * y) * W + (int64_t)S * x;
  float acc[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) acc[k] = 0.f;
#pragma unroll
  for (int i = 0; i < S; ++i) {
    const float *row = src + (int64_t)i * W;
    if (VEC) {
#pragma unroll
      for (int j = 0; j < (S < 4 ? 4 : S); j += 4) {
        const float4 q = *(const float4 *)(row + j);
        const float e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[(j + k) / S % PX] += e[k];
      }
    } else {
#pragma unroll
      for (int j = 0; j < S; ++j) acc[0] += row[j];
    }
  }
  constexpr float kInv = 1.0f / (float)(S * S);  // exact: a power of two
  if constexpr (PX == 4) {
    *(float4 *)(out + o) = make_float4(acc[0] * kInv, acc[1] * kInv, acc[2] * kInv, acc[3] * kInv);
  } else if constexpr (PX == 2) {
    *(float2 *)(out + o) = make_float2(acc[0] * kInv, acc[1] * kInv);
  } else {
    out[o] = acc[0] * kInv;
  }
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

// Grid (column chunks, plane groups of kGatherPlanes).  An index outside
// [0, n_src) gives 0.  VEC (m a multiple of 4, index and dst 16-byte
// aligned): four columns per lane, one 16-byte index load for the whole
// plane group and one 16-byte store per plane.
constexpr int kGatherPlanes = 8;
template <bool VEC>
__global__ __launch_bounds__(256) void k_gather_planes(const float *src, int64_t n_src, int planes,
                                                       const int32_t *index, int64_t m, float *dst) {
  constexpr int PX = VEC ? 4 : 1;
  const int64_t j = ((int64_t)blockIdx.x * 256 + threadIdx.x) * PX;
  if (j >= m) return;
  int32_t k[PX];
  if constexpr (VEC) {
    const int4 q = *(const int4 *)(index + j);
    k[0] = q.x, k[1] = q.y, k[2] = q.z, k[3] = q.w;
  } else {
    k[0] = index[j];
  }
  bool ok[PX];
#pragma unroll
  for (int c = 0; c < PX; ++c) ok[c] = k[c] >= 0 && k[c] < n_src;
  const int p0 = blockIdx.y * kGatherPlanes;
#pragma unroll
  for (int u = 0; u < kGatherPlanes; ++u) {
    const int p = p0 + u;
    if (p >= planes) break;
    const float *plane = src + (int64_t)p * n_src;
    float x[PX];
#pragma unroll
    for (int c = 0; c < PX; ++c) x[c] = ok[c] ? plane[k[c]] : 0.0f;
    if constexpr (VEC)
      *(float4 *)(dst + (int64_t)p * m + j) = make_float4(x[0], x[1], x[2], x[3]);
    else
      dst[(int64_t)p * m + j] = x[0];
  }
}

template <int S>
gs_status launch_downsample(const float *in, int W, int H, int Wc, int Hc, int64_t total, float *out,
                            hipStream_t s) {
  const bool vec = W % 4 == 0 && ((uintptr_t)in & 15u) == 0 && ((uintptr_t)out & 15u) == 0;
  if (vec) {
    constexpr int PX = S < 4 ? 4 / S : 1;
    const unsigned grid = (unsigned)((total / PX + 255) / 256);
    GS_LAUNCH("downsample", (k_downsample<S, true>), grid, 256, 0, s, in, W, H, Wc, Hc, total, out);
    return GS_OK;
  }
  const unsigned grid = (unsigned)((total + 255) / 256);
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
  const auto a16 = [](const void *q) { return ((uintptr_t)q & 15u) == 0; };
  const unsigned groups = (unsigned)((planes + kGatherPlanes - 1) / kGatherPlanes);
  if (m % 4 == 0 && a16(index) && a16(dst)) {
    const dim3 grid((unsigned)((m / 4 + 255) / 256), groups);
    GS_LAUNCH("gather_planes", k_gather_planes<true>, grid, 256, 0, (hipStream_t)stream, src, n_src, (int)planes,
              index, m, dst);
    return GS_OK;
  }
  const dim3 grid((unsigned)((m + 255) / 256), groups);
  GS_LAUNCH("gather_planes", k_gather_planes<false>, grid, 256, 0, (hipStream_t)stream, src, n_src, (int)planes,
            index, m, dst);
  return GS_OK;
}

}  // extern "C"

// ------------------------------------------------- 3D smoothing filter
// Mip-Splatting's 3D filter, which the paper's "proper filtering" of
// multi-scale training cites: a Gaussian's highest sampling rate over the
// training cameras, nu = max f_x / z over the cameras whose image (widened
// by `guard` times its size about its centre) holds the projected mean in
// front of the near plane, and the filter variance (s_f / nu)^2 (0 where no
// camera has seen it).  Binary64 on the binary32 means.
namespace gsmi {
namespace {
constexpr int kF3Views = 8;
struct F3View {
  const float *pose;
  double fx, fy, cx, cy, umin, umax, vmin, vmax, near_plane;
};
struct F3Args {
  const float *means;
  int64_t n;
  int nv;
  F3View v[kF3Views];
  float *nu_max, *filter3d;
  double s_f;
  int last;  // the last batch of views: write the filter variances
};

__global__ __launch_bounds__(256) void k_filter3d(F3Args a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  const double x = a.means[i], y = a.means[a.n + i], z = a.means[2 * a.n + i];
  double nu = (double)a.nu_max[i];
  for (int k = 0; k < a.nv; ++k) {
    const F3View &v = a.v[k];
    const float *P = v.pose;
    const double px = (double)P[0] * x + (double)P[1] * y + (double)P[2] * z + (double)P[9];
    const double py = (double)P[3] * x + (double)P[4] * y + (double)P[5] * z + (double)P[10];
    const double pz = (double)P[6] * x + (double)P[7] * y + (double)P[8] * z + (double)P[11];
    if (!(pz > v.near_plane)) continue;
    const double u = v.fx * px / pz + v.cx, w = v.fy * py / pz + v.cy;
    if (u >= v.umin && u <= v.umax && w >= v.vmin && w <= v.vmax) nu = fmax(nu, v.fx / pz);
  }
  a.nu_max[i] = (float)nu;
  if (a.last && a.filter3d) {
    const double r = a.s_f / nu;
    a.filter3d[i] = nu > 0.0 ? (float)(r * r) : 0.0f;
  }
}
}  // namespace
}  // namespace gsmi

extern "C" gs_status gs_filter3d_update(const float *means, int64_t n, int32_t n_views, const gs_camera *cams,
                                        float guard, float s_f, float *nu_max, float *filter3d, void *stream) {
  using namespace gsmi;
  GS_REQUIRE(n >= 0 && n_views >= 0 && guard >= 1.0f && s_f > 0.0f, "gs_filter3d_update: bad sizes or constants");
  if (n == 0) return GS_OK;
  GS_REQUIRE(means && nu_max && (n_views == 0 || cams), "gs_filter3d_update: NULL argument");
  for (int k = 0; k < n_views; ++k)
    GS_REQUIRE(cams[k].pose && cams[k].width > 0 && cams[k].height > 0 && cams[k].fx > 0.f && cams[k].fy > 0.f,
               "gs_filter3d_update: bad camera %d", k);
  const unsigned grid = (unsigned)((n + 255) / 256);
  int v0 = 0;
  do {
    F3Args a;
    a.means = means;
    a.n = n;
    a.nv = std::min(kF3Views, n_views - v0);
    for (int k = 0; k < a.nv; ++k) {
      const gs_camera &c = cams[v0 + k];
      F3View &v = a.v[k];
      v.pose = c.pose;
      v.fx = c.fx, v.fy = c.fy, v.cx = c.cx, v.cy = c.cy;
      const double g = 0.5 * ((double)guard - 1.0);
      v.umin = -g * c.width, v.umax = (1.0 + g) * c.width;
      v.vmin = -g * c.height, v.vmax = (1.0 + g) * c.height;
      v.near_plane = c.near_plane;
    }
    a.nu_max = nu_max;
    a.filter3d = filter3d;
    a.s_f = s_f;
    v0 += a.nv;
    a.last = v0 >= n_views;
    GS_LAUNCH("filter3d", k_filter3d, grid, 256, 0, (hipStream_t)stream, a);
  } while (v0 < n_views);
  return GS_OK;
}
