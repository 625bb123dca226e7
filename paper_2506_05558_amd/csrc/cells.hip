// Spatial cells of a large scene (the scalable construction of section
// 4.4, at the scale of a scene that does not stay resident as a whole):
// Lloyd's k-means over the Gaussians' means in binary64, the cells'
// bounding spheres, and which cells a camera's frustum meets, so that only
// those cells need to be on the device.
//
// * Initial centroids: the means at indices floor((j + 1/2) n / k) (the
//   Gaussians of a capture are seeded frame by frame along the trajectory,
//   so this spreads the centroids along it), or the caller's.
// * Assignment: the nearest centroid by (dx dx + dy dy) + dz dz in binary64
//   on the binary32 means, every operation rounded on its own (no fused
//   multiply-add), ties to the lower centroid.  One lane per mean; the
//   centroids sit in LDS.
// * Update: each workgroup stages a contiguous chunk of 4096 means and
//   their labels in LDS and one lane per cell adds its members in index
//   order (binary64); the per-chunk partial sums are then added in chunk
//   order, one workgroup per cell, so the result does not depend on
//   scheduling.  A cell without members keeps its centroid.
// * Ordering: the means' indices stably sorted by cell (radix sort of the
//   labels), and each cell's first position in that order.
// * Spheres: centre = centroid, radius = the largest centre-to-mean
//   distance of the cell plus a margin times the largest axis scale of its
//   Gaussians (a splat reaches beyond its mean).
// * Visibility: the sphere reaches in front of the near plane and meets the
//   four side planes of the image's frustum widened by the guard band.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace gsmi {
namespace {

constexpr int kMaxCells = 1024;
constexpr int kChunk = 4096;       // means per update workgroup
constexpr int kAssignBlock = 256;

__global__ void k_cells_init(const float *means, int64_t n, int k, double *cent) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const int64_t i = (int64_t)floor(((double)j + 0.5) * (double)n / (double)k);
  for (int a = 0; a < 3; ++a) cent[3 * j + a] = (double)means[a * n + i];
}

__device__ __forceinline__ double sq3(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

__global__ __launch_bounds__(kAssignBlock) void k_cells_assign(const float *means, int64_t n, const double *cent,
                                                               int k, int32_t *labels) {
  __shared__ double c[3 * kMaxCells];
  for (int q = threadIdx.x; q < 3 * k; q += kAssignBlock) c[q] = cent[q];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kAssignBlock + threadIdx.x;
  if (i >= n) return;
  const double x = means[i], y = means[n + i], z = means[2 * n + i];
  double best = INFINITY;
  int bj = 0;
  for (int j = 0; j < k; ++j) {
    const double d = sq3(x - c[3 * j], y - c[3 * j + 1], z - c[3 * j + 2]);
    if (d < best) {  // strict: a tie keeps the lower centroid
      best = d;
      bj = j;
    }
  }
  labels[i] = bj;
}

// Per chunk b: partial[b][j] = (sum x, sum y, sum z, count) of the chunk's
// members of cell j, in index order.
__global__ __launch_bounds__(256) void k_cells_partials(const float *means, int64_t n, const int32_t *labels, int k,
                                                        double *partial) {
  __shared__ float px[kChunk], py[kChunk], pz[kChunk];
  __shared__ int32_t pl[kChunk];
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  const int cnt = (int)std::min<int64_t>(kChunk, n - base);
  for (int q = threadIdx.x; q < cnt; q += 256) {
    px[q] = means[base + q];
    py[q] = means[n + base + q];
    pz[q] = means[2 * n + base + q];
    pl[q] = labels[base + q];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += 256) {
    double sx = 0.0, sy = 0.0, sz = 0.0, c = 0.0;
    for (int q = 0; q < cnt; ++q) {
      if (pl[q] == j) {
        sx += (double)px[q];
        sy += (double)py[q];
        sz += (double)pz[q];
        c += 1.0;
      }
    }
    double *o = partial + ((int64_t)blockIdx.x * k + j) * 4;
    o[0] = sx;
    o[1] = sy;
    o[2] = sz;
    o[3] = c;
  }
}

// One workgroup per cell: the chunk partials in chunk order (each lane a
// strided run, then a fixed tree), the new centroid, the member count.
__global__ __launch_bounds__(256) void k_cells_update(const double *partial, int nchunks, int k, double *cent,
                                                      int64_t *count) {
  const int j = blockIdx.x;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nchunks; b += 256) {
    const double *p = partial + ((int64_t)b * k + j) * 4;
#pragma unroll
    for (int a = 0; a < 4; ++a) s[a] += p[a];
  }
  __shared__ double red[4][256];
#pragma unroll
  for (int a = 0; a < 4; ++a) red[a][threadIdx.x] = s[a];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
#pragma unroll
      for (int a = 0; a < 4; ++a) red[a][threadIdx.x] += red[a][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double c = red[3][0];
    if (cent && c > 0.0)
      for (int a = 0; a < 3; ++a) cent[3 * j + a] = red[a][0] / c;
    if (count) count[j] = (int64_t)c;
  }
}

__global__ void k_iota_labels(const int32_t *labels, int64_t n, uint32_t *keys, uint32_t *vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[i] = (uint32_t)labels[i];
  vals[i] = (uint32_t)i;
}

__global__ void k_offsets(const int64_t *count, int k, int64_t *offsets) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t s = 0;
  for (int j = 0; j < k; ++j) {
    offsets[j] = s;
    s += count[j];
  }
  offsets[k] = s;
}

// Per chunk b and cell j: the largest centre-to-mean distance and the largest
// axis scale of the chunk's members (0 if none), in [b][j][2].
__global__ __launch_bounds__(256) void k_cells_extent(const float *means, const float *log_scales, int64_t n,
                                                      const int32_t *labels, const double *cent, int k,
                                                      double *partial) {
  __shared__ double pd[kChunk / 2];
  __shared__ float ps[kChunk / 2];
  __shared__ int32_t pl[kChunk / 2];
  constexpr int C = kChunk / 2;
  const int64_t base = (int64_t)blockIdx.x * C;
  const int cnt = (int)std::min<int64_t>(C, n - base);
  for (int q = threadIdx.x; q < cnt; q += 256) {
    const int64_t i = base + q;
    const int j = min(max(labels[i], 0), k - 1);  // a label out of range is read as the nearest valid cell
    const double dx = (double)means[i] - cent[3 * j], dy = (double)means[n + i] - cent[3 * j + 1],
                 dz = (double)means[2 * n + i] - cent[3 * j + 2];
    pd[q] = sqrt(sq3(dx, dy, dz));
    ps[q] = fmaxf(fmaxf(log_scales[i], log_scales[n + i]), log_scales[2 * n + i]);
    pl[q] = j;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += 256) {
    double dmax = 0.0;
    float smax = -INFINITY;
    for (int q = 0; q < cnt; ++q)
      if (pl[q] == j) {
        dmax = fmax(dmax, pd[q]);
        smax = fmaxf(smax, ps[q]);
      }
    double *o = partial + ((int64_t)blockIdx.x * k + j) * 2;
    o[0] = dmax;
    o[1] = smax == -INFINITY ? 0.0 : exp((double)smax);
  }
}

__global__ __launch_bounds__(256) void k_cells_radius(const double *partial, int nchunks, int k, double margin,
                                                      double *radius) {
  const int j = blockIdx.x;
  double d = 0.0, s = 0.0;
  for (int b = threadIdx.x; b < nchunks; b += 256) {
    const double *p = partial + ((int64_t)b * k + j) * 2;
    d = fmax(d, p[0]);
    s = fmax(s, p[1]);
  }
  __shared__ double rd[256], rs[256];
  rd[threadIdx.x] = d;
  rs[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      rd[threadIdx.x] = fmax(rd[threadIdx.x], rd[threadIdx.x + off]);
      rs[threadIdx.x] = fmax(rs[threadIdx.x], rs[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) radius[j] = rd[0] + margin * rs[0];
}

struct Frustum {
  double R[9], t[3];
  double xr, xl, yb, yt, near_plane;
};

__global__ void k_cells_visible(const double *cent, const double *radius, int k, const float *pose, Frustum f,
                                int32_t *visible) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double R[9], t[3];
  for (int q = 0; q < 9; ++q) R[q] = (double)pose[q];
  for (int q = 0; q < 3; ++q) t[q] = (double)pose[9 + q];
  double p[3];
  for (int r = 0; r < 3; ++r) p[r] = R[3 * r] * cent[3 * j] + R[3 * r + 1] * cent[3 * j + 1] + R[3 * r + 2] * cent[3 * j + 2] + t[r];
  const double r = radius[j];
  bool vis = p[2] + r > f.near_plane;
  // side planes through the camera centre, outward normals (1, 0, -xr), (-1, 0, -xl), (0, 1, -yb), (0, -1, -yt)
  vis = vis && (p[0] - f.xr * p[2]) <= r * sqrt(1.0 + f.xr * f.xr);
  vis = vis && (-p[0] - f.xl * p[2]) <= r * sqrt(1.0 + f.xl * f.xl);
  vis = vis && (p[1] - f.yb * p[2]) <= r * sqrt(1.0 + f.yb * f.yb);
  vis = vis && (-p[1] - f.yt * p[2]) <= r * sqrt(1.0 + f.yt * f.yt);
  visible[j] = vis ? 1 : 0;
}

inline unsigned grid_of(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }
inline int nchunks_of(int64_t n, int c) { return (int)((n + c - 1) / c); }

int key_bits_of(int k) {
  int b = 1;
  while ((1 << b) < k) ++b;
  return b;
}

struct KmLayout {
  double *partial;
  int64_t *count;
  uint32_t *keys, *vals;
  void *sort_ws;
  size_t bytes;
};

KmLayout km_layout(void *ws, int64_t n, int k) {
  Carve cv(ws);
  KmLayout L;
  const size_t N = (size_t)std::max<int64_t>(n, 1);
  L.partial = cv.take<double>((size_t)nchunks_of(n, kChunk) * (size_t)k * 4);
  L.count = cv.take<int64_t>((size_t)k);
  L.keys = cv.take<uint32_t>(N);
  L.vals = cv.take<uint32_t>(N);
  L.sort_ws = cv.take<char>(sort_pairs_workspace((int64_t)N));
  L.bytes = cv.off;
  return L;
}

}  // namespace
}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_cells_assign(const float *means, int64_t n, const double *centroids, int32_t k, int32_t *labels,
                          void *stream) {
  GS_REQUIRE(n >= 0 && n < (1ll << 31) && k >= 1 && k <= kMaxCells, "gs_cells_assign: need 0 <= n < 2^31, 1 <= k <= %d",
             kMaxCells);
  if (n == 0) return GS_OK;
  GS_REQUIRE(means && centroids && labels, "gs_cells_assign: NULL argument");
  GS_LAUNCH("cells_assign", k_cells_assign, grid_of(n, kAssignBlock), kAssignBlock, 0, (hipStream_t)stream, means, n,
            centroids, (int)k, labels);
  return GS_OK;
}

gs_status gs_cells_kmeans_workspace(int64_t n, int32_t k, size_t *bytes) {
  GS_REQUIRE(bytes && n >= 0 && n < (1ll << 31) && k >= 1 && k <= kMaxCells, "gs_cells_kmeans_workspace: bad argument");
  *bytes = km_layout(nullptr, n, k).bytes;
  return GS_OK;
}

gs_status gs_cells_kmeans(const float *means, int64_t n, int32_t k, int32_t iters, int32_t init, double *centroids,
                          int32_t *labels, int32_t *order, int64_t *offsets, void *ws, size_t ws_bytes,
                          void *stream) {
  GS_REQUIRE(n >= 1 && n < (1ll << 31) && k >= 1 && k <= kMaxCells && k <= n && iters >= 0,
             "gs_cells_kmeans: need 1 <= k <= min(n, %d), n < 2^31, iters >= 0", kMaxCells);
  GS_REQUIRE(means && centroids && labels, "gs_cells_kmeans: NULL argument");
  const KmLayout L = km_layout(ws, n, k);
  if (!ws || ws_bytes < L.bytes) {
    set_error("gs_cells_kmeans: workspace %zu bytes < %zu", ws_bytes, L.bytes);
    return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  if (init) GS_LAUNCH("cells_init", k_cells_init, grid_of(k), 256, 0, s, means, n, (int)k, centroids);
  const int nc = nchunks_of(n, kChunk);
  for (int it = 0; it < iters; ++it) {
    GS_LAUNCH("cells_assign", k_cells_assign, grid_of(n, kAssignBlock), kAssignBlock, 0, s, means, n, centroids,
              (int)k, labels);
    GS_LAUNCH("cells_update", k_cells_partials, nc, 256, 0, s, means, n, labels, (int)k, L.partial);
    GS_LAUNCH("cells_update", k_cells_update, k, 256, 0, s, L.partial, nc, (int)k, centroids, (int64_t *)nullptr);
  }
  // the final assignment, the member counts and the cell order
  GS_LAUNCH("cells_assign", k_cells_assign, grid_of(n, kAssignBlock), kAssignBlock, 0, s, means, n, centroids,
            (int)k, labels);
  if (order || offsets) {
    GS_LAUNCH("cells_update", k_cells_partials, nc, 256, 0, s, means, n, labels, (int)k, L.partial);
    // counts only: the centroids are not moved again
    GS_LAUNCH("cells_count", k_cells_update, k, 256, 0, s, L.partial, nc, (int)k, (double *)nullptr, L.count);
  }
  if (offsets) GS_LAUNCH("cells_offsets", k_offsets, 1, 64, 0, s, L.count, (int)k, offsets);
  if (order) {
    GS_LAUNCH("cells_order", k_iota_labels, grid_of(n), 256, 0, s, labels, n, L.keys, L.vals);
    gs_status st = sort_pairs_u32(L.keys, L.vals, n, key_bits_of(k), L.sort_ws, s);
    if (st != GS_OK) return st;
    GS_CHECK_HIP(hipMemcpyAsync(order, L.vals, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, s),
                 "gs_cells_kmeans order");
  }
  return GS_OK;
}

gs_status gs_cells_spheres_workspace(int64_t n, int32_t k, size_t *bytes) {
  GS_REQUIRE(bytes && n >= 0 && k >= 1 && k <= kMaxCells, "gs_cells_spheres_workspace: bad argument");
  *bytes = align_up(sizeof(double) * 2 * (size_t)k * (size_t)std::max(1, nchunks_of(n, kChunk / 2)));
  return GS_OK;
}

gs_status gs_cells_spheres(const float *means, const float *log_scales, int64_t n, const int32_t *labels,
                           const double *centroids, int32_t k, float margin, double *radius, void *ws,
                           size_t ws_bytes, void *stream) {
  GS_REQUIRE(n >= 1 && n < (1ll << 31) && k >= 1 && k <= kMaxCells && margin >= 0.f,
             "gs_cells_spheres: bad sizes or margin");
  GS_REQUIRE(means && log_scales && labels && centroids && radius, "gs_cells_spheres: NULL argument");
  size_t need = 0;
  gs_cells_spheres_workspace(n, k, &need);
  if (!ws || ws_bytes < need) {
    set_error("gs_cells_spheres: workspace %zu bytes < %zu", ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  const int nc = nchunks_of(n, kChunk / 2);
  GS_LAUNCH("cells_spheres", k_cells_extent, nc, 256, 0, s, means, log_scales, n, labels, centroids, (int)k,
            (double *)ws);
  GS_LAUNCH("cells_spheres", k_cells_radius, k, 256, 0, s, (const double *)ws, nc, (int)k, (double)margin, radius);
  return GS_OK;
}

gs_status gs_cells_visible(const double *centroids, const double *radius, int32_t k, const gs_camera *cam,
                           float guard, int32_t *visible, void *stream) {
  GS_REQUIRE(k >= 1 && k <= kMaxCells && cam && guard > 0.f, "gs_cells_visible: bad argument");
  GS_REQUIRE(centroids && radius && visible && cam->pose, "gs_cells_visible: NULL argument");
  GS_REQUIRE(cam->width > 0 && cam->height > 0 && cam->fx > 0.f && cam->fy > 0.f,
             "gs_cells_visible: bad camera");
  Frustum f;
  f.xr = (double)guard * ((double)cam->width - cam->cx) / cam->fx;
  f.xl = (double)guard * (double)cam->cx / cam->fx;
  f.yb = (double)guard * ((double)cam->height - cam->cy) / cam->fy;
  f.yt = (double)guard * (double)cam->cy / cam->fy;
  f.near_plane = cam->near_plane;
  GS_LAUNCH("cells_visible", k_cells_visible, grid_of(k, 64), 64, 0, (hipStream_t)stream, centroids, radius, (int)k,
            cam->pose, f, visible);
  return GS_OK;
}

}  // extern "C"

// ------------------------------------------------------- cell residency
namespace gsmi {
namespace {
__global__ void k_fill_f32(float *p, int64_t count, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}
}  // namespace
}  // namespace gsmi

extern "C" {

gs_status gs_copy_rows(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                       void *stream) {
  GS_REQUIRE(width <= dpitch && width <= spitch, "gs_copy_rows: a row is wider than its pitch");
  if (width == 0 || height == 0) return GS_OK;
  GS_REQUIRE(dst && src, "gs_copy_rows: NULL argument");
  GS_CHECK_HIP(hipMemcpy2DAsync(dst, dpitch, src, spitch, width, height, hipMemcpyDefault, (hipStream_t)stream),
               "gs_copy_rows");
  return GS_OK;
}

gs_status gs_fill_f32(float *dst, int64_t count, float value, void *stream) {
  GS_REQUIRE(count >= 0, "gs_fill_f32: count < 0");
  if (count == 0) return GS_OK;
  GS_REQUIRE(dst, "gs_fill_f32: NULL argument");
  GS_LAUNCH("fill", k_fill_f32, grid_of(count), 256, 0, (hipStream_t)stream, dst, count, value);
  return GS_OK;
}

}  // extern "C"
