// Guided-matching depth of new primitives (the paper's appendix on depth
// for Gaussian primitives): per pixel, candidate inverse depths uniform over
// [1/Z* - r, 1/Z* + r] around the monocular depth Z*, one neighbouring frame
// chosen per pixel, the correlation of the pixel's feature vector with the
// neighbour's bilinearly sampled features at each candidate's reprojection,
// the best candidate and a parabola through its neighbours.
//
// Layout: features FP16 channel-last [H][W][C] (a pixel's vector is S = C / 8
// 16-byte segments).  S lanes share a pixel, lane s holding segment s, and
// a workgroup covers 256 / S consecutive pixels of a row, so one load
// instruction of a wave reads the whole vectors of 64 / S neighbouring
// taps (contiguous lines) rather than one segment of 64 scattered vectors.
// A tap's partial inner product is v_dot2_f32_f16 over half2 pairs (FP16
// products are exact in FP32), weighted by the tap's bilinear weight
// (sum_tap w <f_i, F_tap> equals <f_i, sum_tap w F_tap>); the S partials
// are summed across the lanes with xor shuffles, so every lane of a pixel
// holds the same correlation and takes the same decisions.
#include "common.h"

namespace gsmi {
namespace {

constexpr int kMaxNb = 4;

struct DepthArgs {
  int W, H, n_nb, n_cand;
  float fx, fy, cx, cy, r_inv, d_min;
  const uint4 *fi;            // [H][W][C / 8] 16-byte segments
  const uint4 *fj[kMaxNb];
  float R[kMaxNb][9], t[kMaxNb][3];
  const float *zmono;
  float *depth;
  int32_t *best, *choice;
};

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float dot8(const uint4 &a, const uint4 &b, float acc) {
  const uint32_t av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
  for (int q = 0; q < 4; ++q)
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2, av[q]), __builtin_bit_cast(h2, bv[q]), acc, false);
  return acc;
}

// camera-j pixel of the point at inverse depth d on the ray a (= R ray) + t
__device__ __forceinline__ void project_nb(const DepthArgs &A, const float a[3], const float t[3], float d,
                                           float &u, float &v, float &z) {
  const float iz = 1.0f / d;
  const float px = a[0] * iz + t[0], py = a[1] * iz + t[1];
  z = a[2] * iz + t[2];
  u = A.fx * px / z + A.cx;
  v = A.fy * py / z + A.cy;
}

template <int C>
__global__ __launch_bounds__(256) void k_guided_depth(DepthArgs A) {
  constexpr int S = C / 8;    // 16-byte segments per pixel = lanes per pixel
  constexpr int PX = 256 / S; // pixels per workgroup (one row segment)
  const int seg = threadIdx.x % S;
  // workgroups go round-robin to the 8 XCDs: give each XCD a contiguous band of row
  // segments, so the neighbour rows that adjacent rows gather stay in one L2
  const int nx = (A.W + PX - 1) / PX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= nx * A.H) return;
  const int x = (tile % nx) * PX + threadIdx.x / S;
  const int y = tile / nx;
  // lanes past the row end still take part in the shuffles, on a clamped pixel
  const bool live = x < A.W;
  const int xc = live ? x : A.W - 1;
  const int64_t pix = (int64_t)y * A.W + xc;
  const bool lead = live && seg == 0;
  const float zm = A.zmono[pix];
  if (!(zm > 0.f && zm < __builtin_inff())) {  // no monocular depth: no estimate
    if (lead) {
      if (A.choice) A.choice[pix] = -1;
      A.depth[pix] = __builtin_nanf("");
      if (A.best) A.best[pix] = -1;
    }
    return;
  }
  const float inv = 1.0f / zm;
  const float lo = fmaxf(inv - A.r_inv, A.d_min), hi = inv + A.r_inv;
  const float step = (hi - lo) / (float)(A.n_cand - 1);
  const float ray[3] = {((float)xc - A.cx) / A.fx, ((float)y - A.cy) / A.fy, 1.0f};

  // the neighbour whose reprojections of the nearest and farthest candidates
  // lie farthest apart, both inside its image (ties: the lower index)
  int jb = -1;
  float sep_b = -1.0f;
  for (int j = 0; j < A.n_nb; ++j) {
    float a[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) a[r] = A.R[j][3 * r] * ray[0] + A.R[j][3 * r + 1] * ray[1] + A.R[j][3 * r + 2];
    float u0, v0, z0, u1, v1, z1;
    project_nb(A, a, A.t[j], lo, u0, v0, z0);
    project_nb(A, a, A.t[j], hi, u1, v1, z1);
    const auto inside = [&](float u, float v, float z) {
      return z > 0.f && u >= 0.f && u <= (float)(A.W - 1) && v >= 0.f && v <= (float)(A.H - 1);
    };
    const float sep = sqrtf((u1 - u0) * (u1 - u0) + (v1 - v0) * (v1 - v0));
    if (inside(u0, v0, z0) && inside(u1, v1, z1) && sep > sep_b) {
      sep_b = sep;
      jb = j;
    }
  }
  if (lead && A.choice) A.choice[pix] = jb;
  if (jb < 0) {
    if (lead) {
      A.depth[pix] = __builtin_nanf("");
      if (A.best) A.best[pix] = -1;
    }
    return;
  }
  float a[3], t[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    a[r] = A.R[jb][3 * r] * ray[0] + A.R[jb][3 * r + 1] * ray[1] + A.R[jb][3 * r + 2];
    t[r] = A.t[jb][r];
  }
  const uint4 *fj = A.fj[jb] + seg;
  const uint4 f = A.fi[pix * S + seg];

  // streaming argmax (lowest k on ties) with the values beside the best
  const float kNone = -__builtin_inff();
  float cbest = kNone, cleft = kNone, cright = kNone, cprev = kNone;
  int kbest = -1;
#pragma unroll 2
  for (int k = 0; k < A.n_cand; ++k) {
    const float d = lo + step * (float)k;
    float u, v, z;
    project_nb(A, a, t, d, u, v, z);
    float c = kNone;
    if (z > 0.f) {
      // beyond one pixel outside the image every tap is outside: clamp before the
      // conversion to int (u may be huge or infinite for a point near camera j's plane)
      u = fminf(fmaxf(u, -2.0f), (float)A.W + 1.0f);
      v = fminf(fmaxf(v, -2.0f), (float)A.H + 1.0f);
      const float fx0 = floorf(u), fy0 = floorf(v);
      const float ax = u - fx0, ay = v - fy0;
      const int x0 = (int)fx0, y0 = (int)fy0;
      // a tap outside the image reads a clamped pixel with weight 0 (features
      // are finite), so the four loads issue without branches
      float part = 0.f;
#pragma unroll
      for (int tap = 0; tap < 4; ++tap) {
        const int xx = x0 + (tap & 1), yy = y0 + (tap >> 1);
        const bool in = xx >= 0 && xx < A.W && yy >= 0 && yy < A.H;
        const float w = in ? ((tap & 1) ? ax : 1.0f - ax) * ((tap >> 1) ? ay : 1.0f - ay) : 0.0f;
        const int xs = min(max(xx, 0), A.W - 1), ys = min(max(yy, 0), A.H - 1);
        part = __builtin_fmaf(w, dot8(f, fj[((int64_t)ys * A.W + xs) * S], 0.f), part);
      }
      c = part;
#pragma unroll
      for (int o = 1; o < S; o <<= 1) c += __shfl_xor(c, o, 64);
    }
    if (k == kbest + 1 && kbest >= 0) cright = c;
    if (c > cbest) {
      cbest = c;
      kbest = k;
      cleft = cprev;
      cright = kNone;
    }
    cprev = c;
  }
  if (!lead) return;
  if (kbest < 0) {  // no candidate in front of the neighbour
    A.depth[pix] = __builtin_nanf("");
    if (A.best) A.best[pix] = -1;
    return;
  }
  float delta = 0.f;
  if (kbest > 0 && kbest < A.n_cand - 1 && cleft > kNone && cright > kNone) {
    const float den = cleft - 2.0f * cbest + cright;
    if (den < 0.f) delta = 0.5f * (cleft - cright) / den;
  }
  A.depth[pix] = 1.0f / (lo + step * ((float)kbest + delta));
  if (A.best) A.best[pix] = kbest;
}

}  // namespace
}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_guided_depth(int32_t width, int32_t height, int32_t channels, float fx, float fy, float cx, float cy,
                          const void *feat_i, int32_t n_nb, const void *const *feat_nb, const float *rel_poses,
                          const float *zmono, int32_t n_cand, float r_inv, float *depth, int32_t *best,
                          int32_t *choice, void *stream) {
  GS_REQUIRE(width >= 1 && height >= 1 && width <= 16384 && height <= 16384, "gs_guided_depth: bad image size");
  GS_REQUIRE(channels == 8 || channels == 16 || channels == 32 || channels == 64,
             "gs_guided_depth: channels must be 8, 16, 32 or 64");
  GS_REQUIRE(n_nb >= 1 && n_nb <= kMaxNb, "gs_guided_depth: 1..4 neighbouring frames");
  GS_REQUIRE(n_cand >= 3 && n_cand <= 1024, "gs_guided_depth: n_cand must be 3..1024");
  GS_REQUIRE(fx > 0.f && fy > 0.f && r_inv > 0.f, "gs_guided_depth: bad intrinsics or range");
  GS_REQUIRE(feat_i && feat_nb && rel_poses && zmono && depth, "gs_guided_depth: NULL argument");
  DepthArgs A;
  A.W = width; A.H = height; A.n_nb = n_nb; A.n_cand = n_cand;
  A.fx = fx; A.fy = fy; A.cx = cx; A.cy = cy; A.r_inv = r_inv; A.d_min = 1e-3f;
  A.fi = (const uint4 *)feat_i;
  GS_REQUIRE(((uintptr_t)feat_i & 15u) == 0, "gs_guided_depth: features must be 16-byte aligned");
  for (int j = 0; j < kMaxNb; ++j) {
    A.fj[j] = j < n_nb ? (const uint4 *)feat_nb[j] : nullptr;
    if (j < n_nb) GS_REQUIRE(feat_nb[j] && ((uintptr_t)feat_nb[j] & 15u) == 0,
                             "gs_guided_depth: neighbour features NULL or not 16-byte aligned");
    for (int k = 0; k < 9; ++k) A.R[j][k] = j < n_nb ? rel_poses[12 * j + k] : 0.f;
    for (int k = 0; k < 3; ++k) A.t[j][k] = j < n_nb ? rel_poses[12 * j + 9 + k] : 0.f;
  }
  A.zmono = zmono; A.depth = depth; A.best = best; A.choice = choice;
  hipStream_t s = (hipStream_t)stream;
  const auto grid = [&](int c) {  // 256 / (c / 8) pixels of one row per workgroup, padded to 8 XCDs
    const int px = 256 / (c / 8);
    const int64_t tiles = (int64_t)((width + px - 1) / px) * height;
    return dim3((unsigned)((tiles + 7) / 8 * 8));
  };
  switch (channels) {
    case 8: GS_LAUNCH("guided_depth", k_guided_depth<8>, grid(8), 256, 0, s, A); break;
    case 16: GS_LAUNCH("guided_depth", k_guided_depth<16>, grid(16), 256, 0, s, A); break;
    case 32: GS_LAUNCH("guided_depth", k_guided_depth<32>, grid(32), 256, 0, s, A); break;
    default: GS_LAUNCH("guided_depth", k_guided_depth<64>, grid(64), 256, 0, s, A); break;
  }
  return GS_OK;
}

}  // extern "C"
