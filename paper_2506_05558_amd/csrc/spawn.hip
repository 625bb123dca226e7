// Spawning Gaussians from a new frame (section 4.2): per-pixel probability
// from the Laplacian-of-Gaussian response of the input and of the rendered
// image (Eq. 1-3), counter-based selection, and the direct initialisation
// of the selected primitives (position at the pixel's depth, isotropic
// Clark-Evans scale, the pixel's colour).
//
// The probability is evaluated in binary32 with a fixed operation order
// (taps row by row, each product rounded then added; R, G, B squares added
// in that order; correctly rounded sqrt), and every spawn decision is an
// integer function of it: q = floor(P_s 2^24), Bernoulli draws from
// SplitMix64 of (seed + pixel index), or systematic thresholds over the
// integer masses.  The whole selection is therefore reproducible exactly.
#include <math.h>

#include <vector>

#include "common.h"

namespace gsmi {
namespace {

constexpr int kTile = 16;
constexpr int kMaxR = 8;  // sigma <= 2
constexpr int kMaxTaps = (2 * kMaxR + 1) * (2 * kMaxR + 1);

struct Taps {
  float k[kMaxTaps];
  int r;
};

// Exactly rounded sum of doubles (Shewchuk's partials).
double exact_sum(const std::vector<double> &xs) {
  std::vector<double> partials;
  for (double x : xs) {
    size_t i = 0;
    for (double y : partials) {
      if (fabs(x) < fabs(y)) std::swap(x, y);
      const double hi = x + y;
      const double lo = y - (hi - x);
      if (lo != 0.0) partials[i++] = lo;
      x = hi;
    }
    partials.resize(i);
    partials.push_back(x);
  }
  double s = 0.0;
  for (auto it = partials.rbegin(); it != partials.rend(); ++it) s += *it;
  return s;
}

int make_taps(float sigma, Taps &t) {
  const int r = (int)ceil(4.0 * (double)sigma);
  const int n = 2 * r + 1;
  std::vector<double> k((size_t)n * n);
  const double s = sigma;
  for (int y = -r; y <= r; ++y)
    for (int x = -r; x <= r; ++x) {
      const double rr = (double)(x * x + y * y);
      const double g = exp(-rr / (2 * s * s)) / (2 * M_PI * s * s);
      k[(size_t)(y + r) * n + (x + r)] = (rr - 2 * s * s) / (s * s * s * s) * g;
    }
  const double mean = exact_sum(k) / (double)(n * n);
  for (int i = 0; i < n * n; ++i) t.k[i] = (float)(k[i] - mean);
  t.r = r;
  return r;
}

// Norm of the LoG response of an RGB image at every pixel of a 16x16 tile,
// from an LDS tile with a replicated-border halo.
__device__ __forceinline__ float log_norm(const float (*T)[kTile + 2 * kMaxR][kTile + 2 * kMaxR], const Taps &tp,
                                          int ty, int tx) {
  // every product is rounded before it is added: no fused multiply-add here
#pragma clang fp contract(off)
  const int n = 2 * tp.r + 1;
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
  for (int dy = 0; dy < n; ++dy)
    for (int dx = 0; dx < n; ++dx) {
      const float w = tp.k[dy * n + dx];
      acc0 = acc0 + w * T[0][ty + dy][tx + dx];
      acc1 = acc1 + w * T[1][ty + dy][tx + dx];
      acc2 = acc2 + w * T[2][ty + dy][tx + dx];
    }
  float sq = acc0 * acc0;
  sq = sq + acc1 * acc1;
  sq = sq + acc2 * acc2;
  // correctly rounded binary32 sqrt: the binary64 square root is correctly
  // rounded, and rounding it again to binary32 is innocuous (53 >= 2 * 24 + 2)
  return fminf((float)sqrt((double)sq), 1.0f);
}

__device__ __forceinline__ void load_tile(float (*T)[kTile + 2 * kMaxR][kTile + 2 * kMaxR], const float *img, int W,
                                          int H, int x0, int y0, int r) {
  const int S = kTile + 2 * r;
  const int64_t np = (int64_t)W * H;
  for (int i = threadIdx.x; i < S * S; i += blockDim.x) {
    const int yy = i / S, xx = i % S;
    const int gy = min(max(y0 - r + yy, 0), H - 1), gx = min(max(x0 - r + xx, 0), W - 1);
    const int64_t o = (int64_t)gy * W + gx;
    T[0][yy][xx] = img[o];
    T[1][yy][xx] = img[np + o];
    T[2][yy][xx] = img[2 * np + o];
  }
}

__global__ __launch_bounds__(256) void k_spawn_prob(const float *img, const float *rend, int W, int H, Taps tp,
                                                    float *pl, float *ps) {
  __shared__ float T[3][kTile + 2 * kMaxR][kTile + 2 * kMaxR];
  const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
  const int u = x0 + tx, v = y0 + ty;
  load_tile(T, img, W, H, x0, y0, tp.r);
  __syncthreads();
  const float PL = log_norm(T, tp, ty, tx);
  float PS = PL;
  if (rend) {
    __syncthreads();
    load_tile(T, rend, W, H, x0, y0, tp.r);
    __syncthreads();
    PS = fmaxf(PL - log_norm(T, tp, ty, tx), 0.0f);
  }
  if (u < W && v < H) {
    const int64_t o = (int64_t)v * W + u;
    if (pl) pl[o] = PL;
    ps[o] = PS;
  }
}

__device__ __forceinline__ uint64_t quantize(float ps) { return (uint64_t)floorf(ps * 16777216.0f); }

__global__ void k_select_bernoulli(const float *ps, int64_t np, uint64_t seed, uint32_t *flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const uint64_t u = splitmix64(seed + (uint64_t)p) >> 40;
  flag[p] = u < quantize(ps[p]) ? 1u : 0u;
}

__global__ void k_quantize(const float *ps, int64_t np, uint64_t *q) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) q[p] = quantize(ps[p]);
}

// ceil(a / b) for a possibly negative 128-bit numerator and positive b
__device__ __forceinline__ __int128 ceil_div(__int128 a, __int128 b) {
  return a >= 0 ? (a + b - 1) / b : -((-a) / b);
}

// Pixel p spawns if any systematic threshold t_j = floor((j S + U) / K)
// lies in [a, a + q): t_j >= a <=> j >= ceil((a K - U) / S).
__global__ void k_select_fixed(const uint64_t *q, const uint64_t *prefix, const uint64_t *total, int64_t np,
                               int64_t K, uint32_t off24, uint32_t *flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const uint64_t S = *total;
  uint32_t f = 0;
  if (S > 0 && q[p] > 0) {
    const uint64_t U = (S >> 24) * off24 + (((S & 0xFFFFFFull) * off24) >> 24);
    const __int128 a = (__int128)prefix[p], b = a + (__int128)q[p];
    __int128 lo = ceil_div(a * K - (__int128)U, (__int128)S);
    __int128 hi = ceil_div(b * K - (__int128)U, (__int128)S);
    lo = lo < 0 ? 0 : (lo > K ? K : lo);
    hi = hi < 0 ? 0 : (hi > K ? K : hi);
    f = hi > lo ? 1u : 0u;
  }
  flag[p] = f;
}

__global__ void k_compact_pixels(const uint32_t *flag, const uint32_t *pos, int64_t np, int64_t capacity,
                                 int32_t *pixels) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np || !flag[p]) return;
  const uint32_t o = pos[p];
  if (o < capacity) pixels[o] = (int32_t)p;
}

struct RuleArgs {
  int W, H;
  float fx, fy, cx, cy;
  const float *pose;
  const float *img, *depth, *pl;
  const int32_t *pixels;
  int64_t count;
  float logit, min_prob;
  int nb;  // SH coefficients per channel of the destination
  float *means, *log_scales, *quats, *opac, *sh;
  int64_t stride, offset;
};

// Unit quaternion (w, x, y, z), w >= 0, of the rotation R^T (camera axes in world).
__device__ void camera_axes_quat(const float *pose, float q[4]) {
  // m = R^T: m[i][j] = R[j][i]
  float m[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m[i][j] = pose[3 * j + i];
  const float tr = m[0][0] + m[1][1] + m[2][2];
  if (tr > 0.f) {
    const float s = sqrtf(tr + 1.0f) * 2.f;
    q[0] = 0.25f * s; q[1] = (m[2][1] - m[1][2]) / s; q[2] = (m[0][2] - m[2][0]) / s; q[3] = (m[1][0] - m[0][1]) / s;
  } else if (m[0][0] > m[1][1] && m[0][0] > m[2][2]) {
    const float s = sqrtf(1.f + m[0][0] - m[1][1] - m[2][2]) * 2.f;
    q[0] = (m[2][1] - m[1][2]) / s; q[1] = 0.25f * s; q[2] = (m[0][1] + m[1][0]) / s; q[3] = (m[0][2] + m[2][0]) / s;
  } else if (m[1][1] > m[2][2]) {
    const float s = sqrtf(1.f + m[1][1] - m[0][0] - m[2][2]) * 2.f;
    q[0] = (m[0][2] - m[2][0]) / s; q[1] = (m[0][1] + m[1][0]) / s; q[2] = 0.25f * s; q[3] = (m[1][2] + m[2][1]) / s;
  } else {
    const float s = sqrtf(1.f + m[2][2] - m[0][0] - m[1][1]) * 2.f;
    q[0] = (m[1][0] - m[0][1]) / s; q[1] = (m[0][2] + m[2][0]) / s; q[2] = (m[1][2] + m[2][1]) / s; q[3] = 0.25f * s;
  }
  if (q[0] < 0.f)
    for (int k = 0; k < 4; ++k) q[k] = -q[k];
}

__global__ void k_spawn_rule(RuleArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.count) return;
  const int64_t p = a.pixels[i];
  const int v = (int)(p / a.W), u = (int)(p % a.W);
  const int64_t np = (int64_t)a.W * a.H;
  const float D = a.depth[p];
  const float pc[3] = {D * ((float)u - a.cx) / a.fx, D * ((float)v - a.cy) / a.fy, D};
  const float *R = a.pose, *t = a.pose + 9;
  const int64_t o = a.offset + i, st = a.stride;
  for (int c = 0; c < 3; ++c)
    a.means[c * st + o] = R[c] * (pc[0] - t[0]) + R[3 + c] * (pc[1] - t[1]) + R[6 + c] * (pc[2] - t[2]);
  const float f = sqrtf(a.fx * a.fy);
  const float ls = logf(D / (2.0f * f * sqrtf(fmaxf(a.pl[p], a.min_prob))));
  for (int c = 0; c < 3; ++c) a.log_scales[c * st + o] = ls;
  float q[4];
  camera_axes_quat(a.pose, q);
  for (int c = 0; c < 4; ++c) a.quats[c * st + o] = q[c];
  a.opac[o] = a.logit;
  const float dc = 3.5449077018110318f;  // 2 sqrt(pi): colour offset -> DC coefficient
  for (int c = 0; c < 3; ++c) a.sh[(int64_t)c * st + o] = (a.img[c * np + p] - 0.5f) * dc;
  for (int k = 1; k < a.nb; ++k)
    for (int c = 0; c < 3; ++c) a.sh[(int64_t)(k * 3 + c) * st + o] = 0.0f;
}

inline int64_t grid1(int64_t count, int block = 256) { return (count + block - 1) / block; }

}  // namespace

gs_status validate_camera(const gs_camera *cam, const char *fn);

}  // namespace gsmi

using namespace gsmi;

namespace {

gs_status check_spawn_params(const gs_spawn_params *sp, const char *fn) {
  GS_REQUIRE(sp, "%s: spawn params NULL", fn);
  GS_REQUIRE(sp->sigma > 0.f && ceilf(4.f * sp->sigma) <= kMaxR, "%s: sigma %g outside (0, 2]", fn, sp->sigma);
  GS_REQUIRE(sp->mode == GS_SPAWN_BERNOULLI || sp->mode == GS_SPAWN_FIXED_K, "%s: unknown mode %d", fn, sp->mode);
  GS_REQUIRE(sp->mode != GS_SPAWN_FIXED_K || sp->k >= 0, "%s: k < 0", fn);
  GS_REQUIRE(sp->opacity > 0.f && sp->opacity < 1.f && sp->min_prob > 0.f, "%s: opacity / min_prob out of range",
             fn);
  return GS_OK;
}

struct SelLayout {
  uint32_t *flag, *pos, *scalars;
  uint64_t *q, *prefix, *total;
  void *scan_ws;
  size_t bytes;
};

SelLayout sel_layout(void *ws, int64_t np) {
  Carve cv(ws);
  SelLayout L;
  const size_t n = (size_t)(np > 0 ? np : 1);
  L.flag = cv.take<uint32_t>(n);
  L.pos = cv.take<uint32_t>(n);
  L.q = cv.take<uint64_t>(n);
  L.prefix = cv.take<uint64_t>(n);
  L.total = cv.take<uint64_t>(1);
  L.scalars = cv.take<uint32_t>(2);
  L.scan_ws = cv.take<char>(scan_workspace(np));
  L.bytes = cv.off;
  return L;
}

}  // namespace

extern "C" {

void gs_default_spawn_params(gs_spawn_params *sp) {
  if (!sp) return;
  sp->sigma = 1.0f;
  sp->mode = GS_SPAWN_BERNOULLI;
  sp->k = 0;
  sp->seed = 0;
  sp->opacity = 0.1f;
  sp->min_prob = 1e-4f;
}

gs_status gs_spawn_log_taps(float sigma, float *taps, int32_t *radius) {
  GS_REQUIRE(taps && radius, "gs_spawn_log_taps: NULL argument");
  GS_REQUIRE(sigma > 0.f && ceilf(4.f * sigma) <= kMaxR, "gs_spawn_log_taps: sigma %g outside (0, 2]", sigma);
  Taps t;
  const int r = make_taps(sigma, t);
  for (int i = 0; i < (2 * r + 1) * (2 * r + 1); ++i) taps[i] = t.k[i];
  *radius = r;
  return GS_OK;
}

gs_status gs_spawn_probability(const gs_camera *cam, const float *image, const float *rendered,
                               const gs_spawn_params *sp, float *p_l, float *p_s, void *stream) {
  gs_status st = validate_camera(cam, "gs_spawn_probability");
  if (st != GS_OK) return st;
  if ((st = check_spawn_params(sp, "gs_spawn_probability")) != GS_OK) return st;
  GS_REQUIRE(image && p_s, "gs_spawn_probability: NULL image or p_s");
  Taps tp;
  make_taps(sp->sigma, tp);
  const dim3 grid((cam->width + kTile - 1) / kTile, (cam->height + kTile - 1) / kTile);
  GS_LAUNCH("spawn_prob", k_spawn_prob, grid, kTile * kTile, 0, (hipStream_t)stream, image, rendered, cam->width,
            cam->height, tp, p_l, p_s);
  return GS_OK;
}

gs_status gs_spawn_select_workspace(int32_t width, int32_t height, size_t *bytes) {
  GS_REQUIRE(bytes && width > 0 && height > 0, "gs_spawn_select_workspace: bad argument");
  *bytes = sel_layout(nullptr, (int64_t)width * height).bytes;
  return GS_OK;
}

gs_status gs_spawn_select(const gs_camera *cam, const float *p_s, const gs_spawn_params *sp, int64_t capacity,
                          int32_t *pixels, int64_t *n_selected, void *ws, size_t ws_bytes, void *stream) {
  gs_status st = validate_camera(cam, "gs_spawn_select");
  if (st != GS_OK) return st;
  if ((st = check_spawn_params(sp, "gs_spawn_select")) != GS_OK) return st;
  GS_REQUIRE(p_s && n_selected && capacity >= 0, "gs_spawn_select: bad argument");
  if (capacity > 0) GS_REQUIRE(pixels, "gs_spawn_select: NULL pixels");
  const int64_t np = (int64_t)cam->width * cam->height;
  SelLayout L = sel_layout(ws, np);
  if (!ws || ws_bytes < L.bytes) {
    set_error("gs_spawn_select: workspace %zu bytes < %zu", ws_bytes, L.bytes);
    return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  if (sp->mode == GS_SPAWN_BERNOULLI) {
    GS_LAUNCH("spawn_select", k_select_bernoulli, grid1(np), 256, 0, s, p_s, np, sp->seed, L.flag);
  } else {
    GS_LAUNCH("spawn_select", k_quantize, grid1(np), 256, 0, s, p_s, np, L.q);
    if ((st = scan_exclusive_u64(L.q, L.prefix, np, L.total, L.scan_ws, s)) != GS_OK) return st;
    // systematic offset: top 24 bits of SplitMix64 of the seed (host side, same function)
    const uint64_t z = splitmix64(sp->seed);
    GS_LAUNCH("spawn_select", k_select_fixed, grid1(np), 256, 0, s, L.q, L.prefix, L.total, np, sp->k,
              (uint32_t)(z >> 40), L.flag);
  }
  if ((st = scan_exclusive(L.flag, L.pos, np, L.scalars, L.scan_ws, s)) != GS_OK) return st;
  uint32_t count = 0;
  GS_CHECK_HIP(hipMemcpyAsync(&count, L.scalars, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read count");
  GS_CHECK_HIP(hipStreamSynchronize(s), "sync count");
  *n_selected = count;
  if ((int64_t)count > capacity) {
    set_error("gs_spawn_select: %u pixels exceed capacity %lld", count, (long long)capacity);
    return GS_ERR_CAPACITY;
  }
  if (count > 0)
    GS_LAUNCH("spawn_compact", k_compact_pixels, grid1(np), 256, 0, s, L.flag, L.pos, np, capacity, pixels);
  return GS_OK;
}

gs_status gs_spawn_rule(const gs_camera *cam, const float *image, const float *depth, const float *p_l,
                        const int32_t *pixels, int64_t count, const gs_spawn_params *sp, gs_gaussians *out,
                        int64_t offset, void *stream) {
  gs_status st = validate_camera(cam, "gs_spawn_rule");
  if (st != GS_OK) return st;
  if ((st = check_spawn_params(sp, "gs_spawn_rule")) != GS_OK) return st;
  GS_REQUIRE(out && count >= 0 && offset >= 0, "gs_spawn_rule: bad argument");
  GS_REQUIRE(out->sh_degree >= 0 && out->sh_degree <= 3, "gs_spawn_rule: sh_degree out of range");
  if (count == 0) return GS_OK;
  GS_REQUIRE(image && depth && p_l && pixels, "gs_spawn_rule: NULL input");
  GS_REQUIRE(out->means && out->log_scales && out->quats && out->opacity_logits && out->sh,
             "gs_spawn_rule: NULL output plane");
  if (offset + count > out->n) {
    set_error("gs_spawn_rule: %lld + %lld exceeds the destination's %lld", (long long)offset, (long long)count,
              (long long)out->n);
    return GS_ERR_CAPACITY;
  }
  RuleArgs a;
  a.W = cam->width; a.H = cam->height;
  a.fx = cam->fx; a.fy = cam->fy; a.cx = cam->cx; a.cy = cam->cy;
  a.pose = cam->pose;
  a.img = image; a.depth = depth; a.pl = p_l; a.pixels = pixels; a.count = count;
  a.logit = logf(sp->opacity / (1.0f - sp->opacity));
  a.min_prob = sp->min_prob;
  a.nb = (out->sh_degree + 1) * (out->sh_degree + 1);
  a.means = out->means; a.log_scales = out->log_scales; a.quats = out->quats; a.opac = out->opacity_logits;
  a.sh = out->sh;
  a.stride = out->n;
  a.offset = offset;
  GS_LAUNCH("spawn_rule", k_spawn_rule, grid1(count), 256, 0, (hipStream_t)stream, a);
  return GS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- composite
namespace {

struct InitLayout {
  float *p_l, *p_s;
  int32_t *pixels;
  void *sel_ws;
  size_t sel_bytes, bytes;
};

InitLayout init_layout(void *ws, int32_t W, int32_t H, int64_t capacity) {
  Carve cv(ws);
  InitLayout L;
  const size_t np = (size_t)W * H;
  L.p_l = cv.take<float>(np);
  L.p_s = cv.take<float>(np);
  L.pixels = cv.take<int32_t>((size_t)(capacity > 0 ? capacity : 1));
  L.sel_bytes = sel_layout(nullptr, (int64_t)np).bytes;
  L.sel_ws = cv.take<char>(L.sel_bytes);
  L.bytes = cv.off;
  return L;
}

}  // namespace

extern "C" {

gs_status gs_spawn_mlp(const gs_camera *cam, const float *image, const float *depth, const int32_t *pixels,
                       int64_t count, const void *packed, gs_gaussians *out, int64_t offset, void *stream);

gs_status gs_spawn_init_workspace(int32_t width, int32_t height, int64_t capacity, size_t *bytes) {
  GS_REQUIRE(bytes && width > 0 && height > 0 && capacity >= 0, "gs_spawn_init_workspace: bad argument");
  *bytes = init_layout(nullptr, width, height, capacity).bytes;
  return GS_OK;
}

gs_status gs_spawn_init(const gs_camera *cam, const float *image, const float *depth, const float *rendered,
                        const gs_spawn_params *sp, const void *mlp_packed, gs_gaussians *out, int64_t offset,
                        int64_t *n_spawned, void *ws, size_t ws_bytes, void *stream) {
  gs_status st = validate_camera(cam, "gs_spawn_init");
  if (st != GS_OK) return st;
  GS_REQUIRE(out && n_spawned && offset >= 0 && offset <= out->n, "gs_spawn_init: bad argument");
  const int64_t capacity = out->n - offset;
  InitLayout L = init_layout(ws, cam->width, cam->height, capacity);
  if (!ws || ws_bytes < L.bytes) {
    set_error("gs_spawn_init: workspace %zu bytes < %zu", ws_bytes, L.bytes);
    return GS_ERR_WORKSPACE;
  }
  if ((st = gs_spawn_probability(cam, image, rendered, sp, L.p_l, L.p_s, stream)) != GS_OK) return st;
  if ((st = gs_spawn_select(cam, L.p_s, sp, capacity, L.pixels, n_spawned, L.sel_ws, L.sel_bytes, stream)) !=
      GS_OK)
    return st;
  if ((st = gs_spawn_rule(cam, image, depth, L.p_l, L.pixels, *n_spawned, sp, out, offset, stream)) != GS_OK)
    return st;
  if (mlp_packed)
    return gs_spawn_mlp(cam, image, depth, L.pixels, *n_spawned, mlp_packed, out, offset, stream);
  return GS_OK;
}

}  // extern "C"
