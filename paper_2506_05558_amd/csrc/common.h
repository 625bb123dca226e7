// Internal helpers shared by the HIP translation units of libgsmi.
// gfx950 only: wave64, DPP cross-lane ops, hardware float atomics.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gs_api.h"

namespace gsmi {

// ---------------------------------------------------------------- host side
void set_error(const char *fmt, ...);
gs_status hip_fail(hipError_t e, const char *what);

// Launch bracket: records profiling events around a kernel when enabled.
struct ProfScope {
  const char *name;
  hipStream_t stream;
  int slot;
  ProfScope(const char *name, hipStream_t s);
  ~ProfScope();
};

// Finite checks (checks.hip): on when GS_CHECK_FINITE is set to anything but
// "0"; each returns GS_ERR_NONFINITE (with the count in gs_last_error) if
// the array holds a NaN or an infinity, and synchronises the stream.
bool finite_checks_on();
gs_status check_finite(const float *x, int64_t count, const char *fn, const char *what, hipStream_t s);
gs_status check_finite_d(const double *x, int64_t count, const char *fn, const char *what, hipStream_t s);
gs_status check_finite_gaussians(const gs_gaussians *g, const char *fn, const char *what, hipStream_t s);

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Launch helper that checks the launch and returns a status.
#define GS_LAUNCH(name, kernel, grid, block, shmem, stream, ...)                   \
  do {                                                                            \
    ::gsmi::ProfScope _ps(name, stream);                                          \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__); \
    hipError_t _e = hipGetLastError();                                            \
    if (_e != hipSuccess) return ::gsmi::hip_fail(_e, name);                      \
  } while (0)

#define GS_CHECK_HIP(call, what)                        \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return ::gsmi::hip_fail(_e, what); \
  } while (0)

#define GS_REQUIRE(cond, ...)              \
  do {                                     \
    if (!(cond)) {                         \
      ::gsmi::set_error(__VA_ARGS__);      \
      return GS_ERR_INVALID_ARG;           \
    }                                      \
  } while (0)

inline int tiles_x_of(int w) { return (w + GS_TILE - 1) / GS_TILE; }
inline int tiles_y_of(int h) { return (h + GS_TILE - 1) / GS_TILE; }

// Workspace carving: bump allocator over a caller buffer.
struct Carve {
  char *base;
  size_t off;
  explicit Carve(void *p) : base((char *)p), off(0) {}
  template <class T>
  T *take(size_t count) {
    T *p = (T *)(base ? base + off : nullptr);
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

// Stable LSD radix sort of (key, value) pairs by the low key_bits bits of
// the keys, in place (binning.hip); ws: sort_pairs_workspace(count) bytes.
size_t sort_pairs_workspace(int64_t count);
gs_status sort_pairs_u32(uint32_t *keys, uint32_t *vals, int64_t count, int key_bits, void *ws, hipStream_t s);

// SplitMix64 (Steele, Lea and Flood 2014): the generator's output for state
// x, the counter-based stream of the library's random draws.
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Scan / radix sort building blocks (binning.hip).
size_t scan_workspace(int64_t count);
gs_status scan_exclusive(const uint32_t *in, uint32_t *out, int64_t count, uint32_t *total, void *ws,
                         hipStream_t s);
gs_status scan_exclusive_u64(const uint64_t *in, uint64_t *out, int64_t count, uint64_t *total, void *ws,
                             hipStream_t s);

// -------------------------------------------------------------- device side
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Lane mask of a predicate straight from the compare result (no round trip
// through a vector register).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK,
                                                               0xf, false));
}

// Sum over the 64 lanes of a wave; the full sum is valid in lane 63.  Every
// lane must be active.  Row (16-lane) rotations first, then the two
// cross-row broadcasts.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v += dpp_mov<0x128, 0xf>(v);  // row_ror:8
  v += dpp_mov<0x124, 0xf>(v);  // row_ror:4
  v += dpp_mov<0x122, 0xf>(v);  // row_ror:2
  v += dpp_mov<0x121, 0xf>(v);  // row_ror:1
  v += dpp_mov<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_mov<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Inclusive tile rect of a support rect, in FP32 with one rounding per
// bound (mean -/+ half-width), then ceil/floor, clipping and integer
// division.  Returns false when the rect holds no pixel of the image.
__device__ __forceinline__ bool tile_rect(float mx, float my, int rx, int ry, int W, int H, int &tx0, int &ty0,
                                          int &tx1, int &ty1) {
  if (rx <= 0 || ry <= 0) return false;
  const float fx = (float)rx, fy = (float)ry;
  const float fu0 = fmaxf(ceilf(__fsub_rn(mx, fx)), 0.0f);
  const float fu1 = fminf(floorf(__fadd_rn(mx, fx)), (float)(W - 1));
  const float fv0 = fmaxf(ceilf(__fsub_rn(my, fy)), 0.0f);
  const float fv1 = fminf(floorf(__fadd_rn(my, fy)), (float)(H - 1));
  if (!(fu0 <= fu1) || !(fv0 <= fv1)) return false;
  tx0 = (int)fu0 / GS_TILE;
  tx1 = (int)fu1 / GS_TILE;
  ty0 = (int)fv0 / GS_TILE;
  ty1 = (int)fv1 / GS_TILE;
  return true;
}

// One Adam update of one element (section 4.3; the formula of
// gs_adam_step): c1 = 1 / (1 - b1^step), c2 = 1 / (1 - b2^step) from
// adam_bias.  Shared by the optimiser kernels and the adjoint that applies
// the step itself; the moment updates are written as explicit FMAs because
// left to contraction the compiler fuses either product of b m + (1 - b) g
// depending on the surrounding code, and the kernels would differ in the
// last bit.
__device__ __forceinline__ void adam_one(float gi, float &mi, float &vi, float &pi, float lr, float b1, float b2,
                                         float eps, float c1, float c2) {
  mi = __builtin_fmaf(b1, mi, (1.f - b1) * gi);
  vi = __builtin_fmaf(b2, vi, (1.f - b2) * gi * gi);
  pi -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}
inline float adam_bias(float beta, int step) {
  return (float)(1.0 / (1.0 - pow((double)beta, (double)step)));
}

// Map workgroup b of a grid of nb to a logical tile so that each of the 8
// XCDs (workgroups are dealt round-robin) walks one contiguous band of tiles
// and neighbouring tiles, which share Gaussians, hit the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int per = nb / 8;  // nb is padded to a multiple of 8
  return (b % 8) * per + b / 8;
}

}  // namespace gsmi
