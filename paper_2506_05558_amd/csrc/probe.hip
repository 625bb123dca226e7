// Measurement probes: the achievable HBM copy rate and the VALU issue rates
// (FP32 FMA, v_exp_f32) on this device, beside the datasheet peaks that the
// roofline fractions use.  Each writes a result the host reads, so no work
// is eliminated.
#include "common.h"

namespace gsmi {
namespace {

constexpr int kChains = 8;  // independent dependency chains per lane (covers VALU latency)

// Each lane moves kCopyUnroll 16-byte vectors per turn (a workgroup's turn
// covers 4 x 4 KiB contiguous), all loads issued before the first store,
// with non-temporal hints: a stream that no cache can hold.
constexpr int kCopyUnroll = 4;
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_probe_copy(const v4f *__restrict__ src, v4f *__restrict__ dst,
                                                    int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * 256 * kCopyUnroll;
  for (int64_t base = (int64_t)blockIdx.x * 256 * kCopyUnroll + threadIdx.x; base < n4; base += stride) {
    v4f v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t i = base + (int64_t)u * 256;
      if (i < n4) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t i = base + (int64_t)u * 256;
      if (i < n4) __builtin_nontemporal_store(v[u], dst + i);
    }
  }
}

// iters x kChains FMAs per lane, all v_fma_f32 (packed FP32 is disabled)
__global__ __launch_bounds__(256) void k_probe_fma(float seed, int iters, float *out) {
  float a[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) a[c] = seed + (float)(threadIdx.x + c);
  const float m = 0.999999f, k = 1e-7f;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = __builtin_fmaf(a[c], m, k);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += a[c];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// iters x kChains v_exp_f32 per lane (each chain feeds its result back)
__global__ __launch_bounds__(256) void k_probe_exp(float seed, int iters, float *out) {
  float a[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) a[c] = 1.0f + 1e-3f * (float)(threadIdx.x + c) + seed;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = __builtin_amdgcn_exp2f(-a[c]);  // the negation is a source modifier
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += a[c];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace
}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_probe_copy(const void *src, void *dst, size_t bytes, void *stream) {
  GS_REQUIRE(bytes % 16 == 0 && ((uintptr_t)src & 15u) == 0 && ((uintptr_t)dst & 15u) == 0,
             "gs_probe_copy: bytes and pointers must be 16-byte multiples");
  if (bytes == 0) return GS_OK;
  GS_REQUIRE(src && dst && src != dst, "gs_probe_copy: bad pointers");
  const int64_t n4 = (int64_t)(bytes / 16);
  // 8 workgroups per CU, grid-stride over the rest
  const int64_t blocks = std::min<int64_t>((n4 + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll), 256 * 8);
  GS_LAUNCH("probe_copy", k_probe_copy, (unsigned)blocks, 256, 0, (hipStream_t)stream, (const v4f *)src,
            (v4f *)dst, n4);
  return GS_OK;
}

gs_status gs_probe_valu(int32_t kind, int32_t blocks, int32_t iters, float *out, void *stream) {
  GS_REQUIRE(kind == 0 || kind == 1, "gs_probe_valu: kind must be 0 (FMA) or 1 (exp)");
  GS_REQUIRE(blocks >= 1 && blocks <= 1 << 20 && iters >= 1, "gs_probe_valu: bad sizes");
  GS_REQUIRE(out, "gs_probe_valu: NULL output");
  if (kind == 0)
    GS_LAUNCH("probe_fma", k_probe_fma, (unsigned)blocks, 256, 0, (hipStream_t)stream, 0.5f, iters, out);
  else
    GS_LAUNCH("probe_exp", k_probe_exp, (unsigned)blocks, 256, 0, (hipStream_t)stream, 0.5f, iters, out);
  return GS_OK;
}

}  // extern "C"
