// Metrics and debug checks around the rasterizer.
//
// * gs_psnr: peak signal-to-noise ratio of an image against its target,
//   10 log10(peak^2 / MSE) with the MSE summed in binary64 (the metric the
//   evaluation of section 5 reports; the joint optimisation logs it).
// * Finite checks (GS_CHECK_FINITE=1 in the environment): the entry points
//   that take Gaussians, poses or upstream gradients count the non-finite
//   values of those inputs, and of the images and gradients they produce,
//   and return GS_ERR_NONFINITE naming the first array that holds one.  The
//   count goes through one 8-byte device counter per GPU that the library
//   holds (a file-scope device variable, found with hipGetSymbolAddress);
//   a host mutex serialises the checks, each of which synchronises its
//   stream.  Off by default: then no check launches anything.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "common.h"

namespace gsmi {
namespace {

constexpr int kCheckBlock = 256;
constexpr int kCheckMaxBlocks = 2048;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned long long nonfinite_count;
static std::mutex g_check_mu;
static void *g_count_ptr[kMaxDevices];

__global__ void k_clear_count(unsigned long long *c) { *c = 0ull; }

// One atomic per wave: the ballot's population count of the lanes that saw
// a NaN or an infinity.
__global__ __launch_bounds__(kCheckBlock) void k_count_nonfinite(const float *x, int64_t count,
                                                                 unsigned long long *c) {
  unsigned long long bad = 0;
  const int64_t stride = (int64_t)gridDim.x * kCheckBlock;
  for (int64_t base = (int64_t)blockIdx.x * kCheckBlock; base < count; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool nf = i < count && !isfinite(x[i]);
    bad += (unsigned long long)__popcll(ballot(nf));
  }
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(c, bad);
}

__global__ __launch_bounds__(kCheckBlock) void k_count_nonfinite_d(const double *x, int64_t count,
                                                                   unsigned long long *c) {
  unsigned long long bad = 0;
  const int64_t stride = (int64_t)gridDim.x * kCheckBlock;
  for (int64_t base = (int64_t)blockIdx.x * kCheckBlock; base < count; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool nf = i < count && !isfinite(x[i]);
    bad += (unsigned long long)__popcll(ballot(nf));
  }
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(c, bad);
}

gs_status count_ptr(unsigned long long **out) {
  int dev = -1;
  GS_CHECK_HIP(hipGetDevice(&dev), "hipGetDevice");
  GS_REQUIRE(dev >= 0 && dev < kMaxDevices, "finite check: device %d beyond %d", dev, kMaxDevices);
  if (!g_count_ptr[dev]) {
    void *p = nullptr;
    GS_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(nonfinite_count)), "hipGetSymbolAddress(nonfinite_count)");
    GS_REQUIRE(p != nullptr, "finite check: no device address for the counter");
    g_count_ptr[dev] = p;
  }
  *out = (unsigned long long *)g_count_ptr[dev];
  return GS_OK;
}

unsigned blocks_for(int64_t count) {
  int64_t b = (count + kCheckBlock - 1) / kCheckBlock;
  if (b > kCheckMaxBlocks) b = kCheckMaxBlocks;
  return (unsigned)(b < 1 ? 1 : b);
}

template <class T>
gs_status count_nonfinite_locked(const T *x, int64_t count, hipStream_t s, unsigned long long *bad) {
  unsigned long long *c = nullptr;
  gs_status st = count_ptr(&c);
  if (st != GS_OK) return st;
  hipLaunchKernelGGL(k_clear_count, dim3(1), dim3(1), 0, s, c);
  GS_CHECK_HIP(hipGetLastError(), "finite check clear");
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL(k_count_nonfinite, dim3(blocks_for(count)), dim3(kCheckBlock), 0, s, (const float *)x, count,
                       c);
  else
    hipLaunchKernelGGL(k_count_nonfinite_d, dim3(blocks_for(count)), dim3(kCheckBlock), 0, s, (const double *)x,
                       count, c);
  GS_CHECK_HIP(hipGetLastError(), "finite check count");
  GS_CHECK_HIP(hipMemcpyAsync(bad, c, sizeof(*bad), hipMemcpyDeviceToHost, s), "finite check read");
  GS_CHECK_HIP(hipStreamSynchronize(s), "finite check sync");
  return GS_OK;
}

constexpr int kPsnrBlock = 256;
constexpr int kPsnrMaxBlocks = 1024;

__global__ __launch_bounds__(kPsnrBlock) void k_sq_err(const float *img, const float *tgt, int64_t count,
                                                       double *partials) {
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kPsnrBlock;
  for (int64_t i = (int64_t)blockIdx.x * kPsnrBlock + threadIdx.x; i < count; i += stride) {
    const double d = (double)img[i] - (double)tgt[i];
    s += d * d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  __shared__ double red[kPsnrBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int k = 0; k < kPsnrBlock / 64; ++k) a += red[k];
    partials[blockIdx.x] = a;
  }
}

// out[0] = PSNR in dB (+inf for equal images), out[1] = the MSE
__global__ __launch_bounds__(64) void k_psnr_final(const double *partials, int nparts, int64_t count, double peak,
                                                   double *out) {
  double a = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 64) a += partials[k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
  if (threadIdx.x == 0) {
    const double mse = a / (double)count;
    out[0] = mse > 0.0 ? 10.0 * log10(peak * peak / mse) : INFINITY;
    out[1] = mse;
  }
}

}  // namespace

bool finite_checks_on() {
  const char *e = std::getenv("GS_CHECK_FINITE");
  return e && e[0] && std::strcmp(e, "0") != 0;
}

gs_status check_finite(const float *x, int64_t count, const char *fn, const char *what, hipStream_t s) {
  if (count <= 0 || !x) return GS_OK;
  std::lock_guard<std::mutex> lock(g_check_mu);
  unsigned long long bad = 0;
  gs_status st = count_nonfinite_locked(x, count, s, &bad);
  if (st != GS_OK) return st;
  if (bad) {
    set_error("%s: %llu non-finite values in %s", fn, bad, what);
    return GS_ERR_NONFINITE;
  }
  return GS_OK;
}

gs_status check_finite_d(const double *x, int64_t count, const char *fn, const char *what, hipStream_t s) {
  if (count <= 0 || !x) return GS_OK;
  std::lock_guard<std::mutex> lock(g_check_mu);
  unsigned long long bad = 0;
  gs_status st = count_nonfinite_locked(x, count, s, &bad);
  if (st != GS_OK) return st;
  if (bad) {
    set_error("%s: %llu non-finite values in %s", fn, bad, what);
    return GS_ERR_NONFINITE;
  }
  return GS_OK;
}

gs_status check_finite_gaussians(const gs_gaussians *g, const char *fn, const char *what, hipStream_t s) {
  if (!g || g->n <= 0) return GS_OK;
  const int64_t n = g->n;
  const int nsh = 3 * (g->sh_degree + 1) * (g->sh_degree + 1);
  char name[96];
  const struct {
    const float *p;
    int planes;
    const char *nm;
  } parts[5] = {{g->means, 3, "means"},
                {g->log_scales, 3, "log_scales"},
                {g->quats, 4, "quats"},
                {g->opacity_logits, 1, "opacity_logits"},
                {g->sh, nsh, "sh"}};
  for (const auto &p : parts) {
    std::snprintf(name, sizeof(name), "%s.%s", what, p.nm);
    gs_status st = check_finite(p.p, (int64_t)p.planes * n, fn, name, s);
    if (st != GS_OK) return st;
  }
  return GS_OK;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_count_nonfinite(const float *x, int64_t count, int64_t *n_bad, void *stream) {
  GS_REQUIRE(n_bad && count >= 0, "gs_count_nonfinite: bad argument");
  *n_bad = 0;
  if (count == 0) return GS_OK;
  GS_REQUIRE(x, "gs_count_nonfinite: NULL array");
  std::lock_guard<std::mutex> lock(g_check_mu);
  unsigned long long bad = 0;
  gs_status st = count_nonfinite_locked(x, count, (hipStream_t)stream, &bad);
  if (st != GS_OK) return st;
  *n_bad = (int64_t)bad;
  return GS_OK;
}

gs_status gs_psnr_workspace(int64_t count, size_t *bytes) {
  GS_REQUIRE(bytes && count >= 0, "gs_psnr_workspace: bad argument");
  *bytes = align_up(sizeof(double) * kPsnrMaxBlocks);
  return GS_OK;
}

gs_status gs_psnr(const float *image, const float *target, int64_t count, float peak, double *out, void *ws,
                  size_t ws_bytes, void *stream) {
  GS_REQUIRE(count >= 1 && out && peak > 0.f, "gs_psnr: need count >= 1, an output and peak > 0");
  GS_REQUIRE(image && target, "gs_psnr: NULL image or target");
  size_t need = 0;
  gs_psnr_workspace(count, &need);
  if (!ws || ws_bytes < need) {
    set_error("gs_psnr: workspace %zu bytes < %zu", ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  int64_t blocks = (count + kPsnrBlock - 1) / kPsnrBlock;
  if (blocks > kPsnrMaxBlocks) blocks = kPsnrMaxBlocks;
  GS_LAUNCH("psnr", k_sq_err, blocks, kPsnrBlock, 0, s, image, target, count, (double *)ws);
  GS_LAUNCH("psnr", k_psnr_final, 1, 64, 0, s, (const double *)ws, (int)blocks, count, (double)peak, out);
  return GS_OK;
}

}  // extern "C"
