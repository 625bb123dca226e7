// Learned initialisation of spawned primitives: a 196 -> 64 -> 64 -> 7 MLP
// with exact-erf GELU that predicts, from the 7x7 RGB patch around a spawned
// pixel and its 7x7 depth patch as log(D / D_centre), residuals over the
// direct rule of section 4.2 (three log-scales along the camera-aligned
// axes, the opacity logit, the colour).
//
// Inference runs on the matrix cores: v_mfma_f32_16x16x32_bf16, one wave per
// group of 16 samples (M = 16), weights staged once per workgroup in LDS,
// FP32 accumulation, hidden activations rounded to BF16 between layers.
// The features are gathered from the image and depth planes straight into
// the A operand, so the 196 inputs of a sample never go through HBM.
//
// Training runs in FP32 on the vector ALUs: one workgroup per chunk of 64
// samples keeps the features and all activations in LDS, every weight
// operand of an inner product is wave-uniform (scalar loads), per-chunk
// gradients are summed in a fixed order and the Adam update is fused into
// that sum.
#include <math.h>

#include "common.h"

namespace gsmi {
namespace {

constexpr int kIn = 196, kHid = 64, kOut = 7, kPatch = 7;
constexpr int kNParams = kHid * kIn + kHid + kHid * kHid + kHid + kOut * kHid + kOut;  // 17223
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kOut * kHid;
static_assert(oB3 + kOut == kNParams, "parameter layout");

// ------------------------------------------------------------------ features
// Feature k of the sample at pixel (u, v): k < 147 is channel k % 3 of patch
// position k / 3 (row-major 7x7, replicated borders); 147 <= k < 196 is
// log(D(q) / D(p)) at patch position k - 147.
__device__ __forceinline__ float feature(const float *img, const float *depth, int W, int H, int u, int v,
                                         float log_dc, int k) {
  const int64_t np = (int64_t)W * H;
  if (k < 147) {
    const int q = k / 3, c = k - 3 * q;
    const int y = min(max(v + q / kPatch - 3, 0), H - 1), x = min(max(u + q % kPatch - 3, 0), W - 1);
    return img[c * np + (int64_t)y * W + x];
  }
  const int q = k - 147;
  const int y = min(max(v + q / kPatch - 3, 0), H - 1), x = min(max(u + q % kPatch - 3, 0), W - 1);
  return logf(depth[(int64_t)y * W + x]) - log_dc;
}

__global__ void k_features(const float *img, const float *depth, int W, int H, const int32_t *pixels, int64_t count,
                           float *out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count * kIn) return;
  const int64_t s = e / kIn;
  const int k = (int)(e - s * kIn);
  const int p = pixels[s];
  const int v = p / W, u = p - v * W;
  out[e] = feature(img, depth, W, H, u, v, logf(depth[p]), k);
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ------------------------------------------------------------ BF16 inference
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kK1 = 224;  // 196 inputs padded to 7 MFMA K-steps of 32
// Packed weights (global memory, written by gs_mlp_pack_bf16):
//   W1 bf16 [64][224] (zero beyond 196), W2 bf16 [64][64], W3 bf16 [16][64]
//   (rows >= 7 zero), then b1 f32 [64], b2 f32 [64], b3 f32 [16].
constexpr size_t pW1 = 0, pW2 = pW1 + 64 * kK1 * 2, pW3 = pW2 + 64 * 64 * 2, pB1 = pW3 + 16 * 64 * 2,
                 pB2 = pB1 + 64 * 4, pB3 = pB2 + 64 * 4, kPackedBytes = pB3 + 16 * 4;
// LDS row strides (bf16 elements): padded by 16 bytes so the 16-byte
// fragment reads of 16 consecutive rows fall into different banks.
constexpr int kS1 = kK1 + 8, kS2 = 64 + 8;

__global__ void k_pack_bf16(const float *theta, uint8_t *packed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  __bf16 *w1 = (__bf16 *)(packed + pW1), *w2 = (__bf16 *)(packed + pW2), *w3 = (__bf16 *)(packed + pW3);
  float *b1 = (float *)(packed + pB1), *b2 = (float *)(packed + pB2), *b3 = (float *)(packed + pB3);
  if (i < 64 * kK1) {
    const int n = i / kK1, k = i % kK1;
    w1[i] = (__bf16)(k < kIn ? theta[oW1 + n * kIn + k] : 0.0f);
  }
  if (i < 64 * 64) w2[i] = (__bf16)theta[oW2 + i];
  if (i < 16 * 64) {
    const int n = i / 64;
    w3[i] = (__bf16)(n < kOut ? theta[oW3 + i] : 0.0f);
  }
  if (i < 64) {
    b1[i] = theta[oB1 + i];
    b2[i] = theta[oB2 + i];
  }
  if (i < 16) b3[i] = i < kOut ? theta[oB3 + i] : 0.0f;
}

struct FromArray {  // features given as [count][196] float32
  const float *x;
  __device__ float operator()(int64_t s, int k, const float &) const { return x[s * kIn + k]; }
  __device__ float centre(int64_t) const { return 0.0f; }
};

struct FromImage {  // features gathered at spawned pixels
  const float *img, *depth;
  const int32_t *pixels;
  int W, H;
  __device__ float centre(int64_t s) const { return logf(depth[pixels[s]]); }
  __device__ float operator()(int64_t s, int k, const float &log_dc) const {
    const int p = pixels[s];
    const int v = p / W, u = p - v * W;
    return feature(img, depth, W, H, u, v, log_dc, k);
  }
};

struct ToArray {  // outputs [count][7]
  float *y;
  __device__ void operator()(int64_t s, int n, float val) const { y[s * kOut + n] = val; }
};

struct ToGaussians {  // residuals added onto the rule's parameters at offset + s
  float *log_scales, *opac, *sh;
  int64_t stride, offset;
  __device__ void operator()(int64_t s, int n, float val) const {
    const int64_t o = offset + s;
    if (n < 3)
      log_scales[n * stride + o] += val;
    else if (n == 3)
      opac[o] += val;
    else
      sh[(n - 4) * stride + o] += val * 3.5449077018110318f;  // colour offset -> DC coefficient (2 sqrt(pi))
  }
};

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <class Src, class Sink>
__global__ __launch_bounds__(256) void k_mlp_infer(const uint8_t *packed, Src src, int64_t count, Sink sink) {
  __shared__ __attribute__((aligned(16))) __bf16 sW1[64 * kS1];
  __shared__ __attribute__((aligned(16))) __bf16 sW2[64 * kS2];
  __shared__ __attribute__((aligned(16))) __bf16 sW3[16 * kS2];
  __shared__ __attribute__((aligned(16))) __bf16 sH[4][16 * kS2];
  __shared__ float sB[64 + 64 + 16];
  const int tid = threadIdx.x;
  // stage weights: 16-byte chunks (8 bf16) of each row into padded rows
  for (int c = tid; c < 64 * (kK1 / 8); c += 256) {
    const int r = c / (kK1 / 8), j = c % (kK1 / 8);
    *(uint4 *)&sW1[r * kS1 + j * 8] = *(const uint4 *)(packed + pW1 + (size_t)(r * kK1 + j * 8) * 2);
  }
  for (int c = tid; c < 64 * 8; c += 256) {
    const int r = c / 8, j = c % 8;
    *(uint4 *)&sW2[r * kS2 + j * 8] = *(const uint4 *)(packed + pW2 + (size_t)(r * 64 + j * 8) * 2);
  }
  for (int c = tid; c < 16 * 8; c += 256) {
    const int r = c / 8, j = c % 8;
    *(uint4 *)&sW3[r * kS2 + j * 8] = *(const uint4 *)(packed + pW3 + (size_t)(r * 64 + j * 8) * 2);
  }
  if (tid < 144) sB[tid] = ((const float *)(packed + pB1))[tid];
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int lane = tid % 64, row = lane % 16, quad = lane / 16;
  __bf16 *H = sH[wave];
  const int64_t ngroups = (count + 15) / 16;
  for (int64_t g = (int64_t)blockIdx.x * 4 + wave; g < ngroups; g += (int64_t)gridDim.x * 4) {
    // A operand: lane holds sample g*16 + row, inputs ks*32 + quad*8 + [0, 8)
    const int64_t sa = g * 16 + row;
    const bool va = sa < count;
    const float log_dc = va ? src.centre(sa) : 0.0f;
    f32x4 acc[4];
    for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kK1 / 32; ++ks) {
      bf16x8 a;
      for (int i = 0; i < 8; ++i) {
        const int k = ks * 32 + quad * 8 + i;
        a[i] = (__bf16)((va && k < kIn) ? src(sa, k, log_dc) : 0.0f);
      }
      for (int nb = 0; nb < 4; ++nb) {
        const bf16x8 b = *(const bf16x8 *)&sW1[(nb * 16 + row) * kS1 + ks * 32 + quad * 8];
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nb], 0, 0, 0);
      }
    }
    // D element i of block nb: sample quad*4 + i, unit nb*16 + row
    for (int nb = 0; nb < 4; ++nb)
      for (int i = 0; i < 4; ++i)
        H[(quad * 4 + i) * kS2 + nb * 16 + row] = (__bf16)gelu(acc[nb][i] + sB[nb * 16 + row]);
    wave_lds_fence();
    for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < 2; ++ks) {
      const bf16x8 a = *(const bf16x8 *)&H[row * kS2 + ks * 32 + quad * 8];
      for (int nb = 0; nb < 4; ++nb) {
        const bf16x8 b = *(const bf16x8 *)&sW2[(nb * 16 + row) * kS2 + ks * 32 + quad * 8];
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nb], 0, 0, 0);
      }
    }
    wave_lds_fence();
    for (int nb = 0; nb < 4; ++nb)
      for (int i = 0; i < 4; ++i)
        H[(quad * 4 + i) * kS2 + nb * 16 + row] = (__bf16)gelu(acc[nb][i] + sB[64 + nb * 16 + row]);
    wave_lds_fence();
    f32x4 y = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < 2; ++ks) {
      const bf16x8 a = *(const bf16x8 *)&H[row * kS2 + ks * 32 + quad * 8];
      const bf16x8 b = *(const bf16x8 *)&sW3[row * kS2 + ks * 32 + quad * 8];
      y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, y, 0, 0, 0);
    }
    wave_lds_fence();
    if (row < kOut)
      for (int i = 0; i < 4; ++i) {
        const int64_t s = g * 16 + quad * 4 + i;
        if (s < count) sink(s, row, y[i] + sB[128 + row]);
      }
  }
}

// ----------------------------------------------------------- FP32 training
constexpr int kChunk = 64;    // samples per workgroup (one per lane)
constexpr int kXs = 209;      // LDS row stride of the features (>= 208, odd)
constexpr int kAs = 65;       // LDS row stride of the activations (odd)
constexpr int kK1T = 208;     // inputs padded to 13 x 16 for the weight-gradient tiles

// Transposed weights for wave-uniform (scalar) operand loads in the forward:
// W1t [196][64], W2t [64][64], W3t [64][8] (column 7 zero).
constexpr int tW1 = 0, tW2 = tW1 + kIn * 64, tW3 = tW2 + 64 * 64, kTBytes = (tW3 + 64 * 8) * 4;

__global__ void k_transpose_weights(const float *theta, float *wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kIn * 64) {
    const int k = i / 64, j = i % 64;
    wt[tW1 + i] = theta[oW1 + j * kIn + k];
  }
  if (i < 64 * 64) {
    const int k = i / 64, j = i % 64;
    wt[tW2 + i] = theta[oW2 + j * 64 + k];
  }
  if (i < 64 * 8) {
    const int k = i / 8, o = i % 8;
    wt[tW3 + i] = o < kOut ? theta[oW3 + o * 64 + k] : 0.0f;
  }
}

struct TrainShared {
  float X[kChunk * kXs];
  float h1[kChunk * kAs], g1[kChunk * kAs];  // activation and GELU slope of layer 1 (g1 becomes dz1)
  float h2[kChunk * kAs], g2[kChunk * kAs];  // same for layer 2 (g2 becomes dz2)
  float dy[8 * kChunk];                      // [o][s]
  float loss[4];
};

__global__ __launch_bounds__(256) void k_mlp_train_chunk(const float *theta, const float *wt, const float *X,
                                                         const float *T, int64_t batch, float inv_count,
                                                         float *partials, float *loss_partials) {
  __shared__ TrainShared S;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid / 64);
  const int s = tid % 64;
  const int64_t s0 = (int64_t)blockIdx.x * kChunk;
  const int nvalid = batch - s0 < kChunk ? (int)(batch - s0) : kChunk;
  // features -> LDS (zero for padded inputs and samples past the batch)
  for (int e = tid; e < kChunk * kK1T; e += 256) {
    const int r = e / kK1T, k = e % kK1T;
    S.X[r * kXs + k] = (r < nvalid && k < kIn) ? X[(s0 + r) * kIn + k] : 0.0f;
  }
  __syncthreads();
  const bool valid = s < nvalid;

  // layer 1: wave w computes units 16w .. 16w+15 of its lane's sample
  {
    float acc[16];
    for (int j = 0; j < 16; ++j) acc[j] = theta[oB1 + 16 * w + j];
    for (int k = 0; k < kIn; ++k) {
      const float x = S.X[s * kXs + k];
      const float *wk = wt + tW1 + k * 64 + 16 * w;
      for (int j = 0; j < 16; ++j) acc[j] = fmaf(wk[j], x, acc[j]);
    }
    for (int j = 0; j < 16; ++j) {
      S.h1[s * kAs + 16 * w + j] = gelu(acc[j]);
      S.g1[s * kAs + 16 * w + j] = gelu_grad(acc[j]);
    }
  }
  __syncthreads();
  // layer 2
  {
    float acc[16];
    for (int j = 0; j < 16; ++j) acc[j] = theta[oB2 + 16 * w + j];
    for (int k = 0; k < 64; ++k) {
      const float h = S.h1[s * kAs + k];
      const float *wk = wt + tW2 + k * 64 + 16 * w;
      for (int j = 0; j < 16; ++j) acc[j] = fmaf(wk[j], h, acc[j]);
    }
    for (int j = 0; j < 16; ++j) {
      S.h2[s * kAs + 16 * w + j] = gelu(acc[j]);
      S.g2[s * kAs + 16 * w + j] = gelu_grad(acc[j]);
    }
  }
  __syncthreads();
  // layer 3 and the loss gradient: wave w computes outputs w and w + 4
  {
    float lsum = 0.0f;
    for (int o = w; o < kOut; o += 4) {
      float y = theta[oB3 + o];
      for (int k = 0; k < 64; ++k) y = fmaf(wt[tW3 + k * 8 + o], S.h2[s * kAs + k], y);
      const float d = valid ? y - T[(s0 + s) * kOut + o] : 0.0f;
      lsum += d * d;
      S.dy[o * kChunk + s] = 2.0f * d * inv_count;
    }
    if (w == 3) S.dy[7 * kChunk + s] = 0.0f;
    // wave sum of the squared errors
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (s == 0) S.loss[w] = lsum;
  }
  __syncthreads();
  float *P = partials + (int64_t)blockIdx.x * kNParams;
  if (tid == 0) loss_partials[blockIdx.x] = (S.loss[0] + S.loss[1]) + (S.loss[2] + S.loss[3]);
  // gW3 [7][64], gb3 [7]
  for (int e = tid; e < kOut * 64 + kOut; e += 256) {
    float acc = 0.0f;
    if (e < kOut * 64) {
      const int o = e / 64, k = e % 64;
      for (int r = 0; r < kChunk; ++r) acc = fmaf(S.dy[o * kChunk + r], S.h2[r * kAs + k], acc);
      P[oW3 + e] = acc;
    } else {
      const int o = e - kOut * 64;
      for (int r = 0; r < kChunk; ++r) acc += S.dy[o * kChunk + r];
      P[oB3 + o] = acc;
    }
  }
  // dz2 = (dY W3) * gelu'(z2): wave w, units 16w .. 16w+15 of its lane's sample
  {
    float d[16];
    for (int j = 0; j < 16; ++j) d[j] = 0.0f;
    for (int o = 0; o < kOut; ++o) {
      const float g = S.dy[o * kChunk + s];
      const float *wo = theta + oW3 + o * 64 + 16 * w;
      for (int j = 0; j < 16; ++j) d[j] = fmaf(wo[j], g, d[j]);
    }
    for (int j = 0; j < 16; ++j) S.g2[s * kAs + 16 * w + j] *= d[j];
  }
  __syncthreads();
  // gW2 [64][64] = dz2^T h1 and gb2: thread tile j = 4 (t / 16) + a, k = 4 (t % 16) + b
  {
    const int j0 = 4 * (tid / 16), k0 = 4 * (tid % 16);
    float acc[4][4] = {};
    float gb[4] = {};
    for (int r = 0; r < kChunk; ++r) {
      float dz[4], h[4];
      for (int a = 0; a < 4; ++a) dz[a] = S.g2[r * kAs + j0 + a];
      for (int b = 0; b < 4; ++b) h[b] = S.h1[r * kAs + k0 + b];
      for (int a = 0; a < 4; ++a) {
        gb[a] += dz[a];
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(dz[a], h[b], acc[a][b]);
      }
    }
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) P[oW2 + (j0 + a) * 64 + k0 + b] = acc[a][b];
    if (tid % 16 == 0)
      for (int a = 0; a < 4; ++a) P[oB2 + j0 + a] = gb[a];
  }
  // dz1 = (dz2 W2) * gelu'(z1): wave w, inputs 16w .. 16w+15 of layer 2 for its lane's sample
  {
    float d[16];
    for (int k = 0; k < 16; ++k) d[k] = 0.0f;
    for (int j = 0; j < 64; ++j) {
      const float g = S.g2[s * kAs + j];
      const float *wj = theta + oW2 + j * 64 + 16 * w;
      for (int k = 0; k < 16; ++k) d[k] = fmaf(wj[k], g, d[k]);
    }
    for (int k = 0; k < 16; ++k) S.g1[s * kAs + 16 * w + k] *= d[k];
  }
  __syncthreads();
  // gW1 [64][196] = dz1^T X and gb1: thread tile j = 4 (t / 16) + a, k = (t % 16) + 16 b, b < 13
  {
    const int j0 = 4 * (tid / 16), kb = tid % 16;
    float acc[4][13] = {};
    float gb[4] = {};
    for (int r = 0; r < kChunk; ++r) {
      float dz[4];
      for (int a = 0; a < 4; ++a) dz[a] = S.g1[r * kAs + j0 + a];
      for (int a = 0; a < 4; ++a) gb[a] += dz[a];
      for (int b = 0; b < 13; ++b) {
        const float x = S.X[r * kXs + kb + 16 * b];
        for (int a = 0; a < 4; ++a) acc[a][b] = fmaf(dz[a], x, acc[a][b]);
      }
    }
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 13; ++b) {
        const int k = kb + 16 * b;
        if (k < kIn) P[oW1 + (j0 + a) * kIn + k] = acc[a][b];
      }
    if (kb == 0)
      for (int a = 0; a < 4; ++a) P[oB1 + j0 + a] = gb[a];
  }
}

// Sum of the chunk gradients in chunk order, then one Adam step.
__global__ void k_mlp_reduce_adam(float *theta, float *m, float *v, const float *partials, int nchunks,
                                  const float *loss_partials, float inv_count, float lr, float beta1, float beta2,
                                  float eps, float bc1, float bc2, float *grad_out, float *loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0 && loss) {
    float l = 0.0f;
    for (int c = 0; c < nchunks; ++c) l += loss_partials[c];
    *loss = l * inv_count;
  }
  if (p >= kNParams) return;
  float g = 0.0f;
  for (int c = 0; c < nchunks; ++c) g += partials[(int64_t)c * kNParams + p];
  if (grad_out) grad_out[p] = g;
  if (lr == 0.0f) return;
  const float mm = beta1 * m[p] + (1.0f - beta1) * g;
  const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
  m[p] = mm;
  v[p] = vv;
  theta[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

inline int64_t grid1(int64_t count, int block = 256) { return (count + block - 1) / block; }

struct TrainLayout {
  float *wt, *partials, *loss_partials;
  size_t bytes;
};

TrainLayout train_layout(void *ws, int64_t batch) {
  Carve cv(ws);
  TrainLayout L;
  const int64_t nchunks = (batch + kChunk - 1) / kChunk;
  L.wt = cv.take<float>(kTBytes / 4);
  L.partials = cv.take<float>((size_t)nchunks * kNParams);
  L.loss_partials = cv.take<float>((size_t)nchunks);
  L.bytes = cv.off;
  return L;
}

}  // namespace

gs_status validate_camera(const gs_camera *cam, const char *fn);

}  // namespace gsmi

using namespace gsmi;

extern "C" {

size_t gs_mlp_packed_bytes(void) { return kPackedBytes; }

gs_status gs_mlp_pack_bf16(const float *theta, void *packed, void *stream) {
  GS_REQUIRE(theta && packed, "gs_mlp_pack_bf16: NULL argument");
  GS_LAUNCH("mlp_pack", k_pack_bf16, grid1(64 * kK1), 256, 0, (hipStream_t)stream, theta, (uint8_t *)packed);
  return GS_OK;
}

gs_status gs_mlp_features(const gs_camera *cam, const float *image, const float *depth, const int32_t *pixels,
                          int64_t count, float *features, void *stream) {
  gs_status st = validate_camera(cam, "gs_mlp_features");
  if (st != GS_OK) return st;
  GS_REQUIRE(count >= 0 && count <= (int64_t)1 << 31, "gs_mlp_features: count %lld out of range",
             (long long)count);
  if (count == 0) return GS_OK;
  GS_REQUIRE(image && depth && pixels && features, "gs_mlp_features: NULL argument");
  GS_LAUNCH("mlp_features", k_features, grid1(count * kIn), 256, 0, (hipStream_t)stream, image, depth, cam->width,
            cam->height, pixels, count, features);
  return GS_OK;
}

gs_status gs_mlp_forward_bf16(const void *packed, const float *features, int64_t count, float *out, void *stream) {
  GS_REQUIRE(count >= 0, "gs_mlp_forward_bf16: count < 0");
  if (count == 0) return GS_OK;
  GS_REQUIRE(packed && features && out, "gs_mlp_forward_bf16: NULL argument");
  const int64_t groups = (count + 15) / 16;
  const int64_t grid = std::min<int64_t>((groups + 3) / 4, 4096);
  GS_LAUNCH("mlp_infer", (k_mlp_infer<FromArray, ToArray>), grid, 256, 0, (hipStream_t)stream,
            (const uint8_t *)packed, FromArray{features}, count, ToArray{out});
  return GS_OK;
}

gs_status gs_spawn_mlp(const gs_camera *cam, const float *image, const float *depth, const int32_t *pixels,
                       int64_t count, const void *packed, gs_gaussians *out, int64_t offset, void *stream) {
  gs_status st = validate_camera(cam, "gs_spawn_mlp");
  if (st != GS_OK) return st;
  GS_REQUIRE(out && count >= 0 && offset >= 0, "gs_spawn_mlp: bad argument");
  if (count == 0) return GS_OK;
  GS_REQUIRE(image && depth && pixels && packed, "gs_spawn_mlp: NULL input");
  GS_REQUIRE(out->log_scales && out->opacity_logits && out->sh, "gs_spawn_mlp: NULL output plane");
  if (offset + count > out->n) {
    set_error("gs_spawn_mlp: %lld + %lld exceeds the destination's %lld", (long long)offset, (long long)count,
              (long long)out->n);
    return GS_ERR_CAPACITY;
  }
  const int64_t groups = (count + 15) / 16;
  const int64_t grid = std::min<int64_t>((groups + 3) / 4, 4096);
  FromImage src{image, depth, pixels, cam->width, cam->height};
  ToGaussians sink{out->log_scales, out->opacity_logits, out->sh, out->n, offset};
  GS_LAUNCH("mlp_infer", (k_mlp_infer<FromImage, ToGaussians>), grid, 256, 0, (hipStream_t)stream,
            (const uint8_t *)packed, src, count, sink);
  return GS_OK;
}

gs_status gs_mlp_train_workspace(int64_t batch, size_t *bytes) {
  GS_REQUIRE(bytes && batch >= 0, "gs_mlp_train_workspace: bad argument");
  *bytes = train_layout(nullptr, batch).bytes;
  return GS_OK;
}

gs_status gs_mlp_train_step(float *theta, float *m, float *v, const float *features, const float *targets,
                            int64_t batch, float lr, float beta1, float beta2, float eps, int32_t step, float *loss,
                            float *grad, void *ws, size_t ws_bytes, void *stream) {
  GS_REQUIRE(theta && features && targets, "gs_mlp_train_step: NULL argument");
  GS_REQUIRE(batch > 0 && batch <= (int64_t)1 << 24, "gs_mlp_train_step: batch %lld out of range",
             (long long)batch);
  GS_REQUIRE(lr == 0.0f || (m && v && step >= 1), "gs_mlp_train_step: Adam needs m, v and step >= 1");
  TrainLayout L = train_layout(ws, batch);
  if (!ws || ws_bytes < L.bytes) {
    set_error("gs_mlp_train_step: workspace %zu bytes < %zu", ws_bytes, L.bytes);
    return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  const int nchunks = (int)((batch + kChunk - 1) / kChunk);
  const float inv_count = 1.0f / (float)(batch * kOut);
  GS_LAUNCH("mlp_train", k_transpose_weights, grid1(kIn * 64), 256, 0, s, theta, L.wt);
  GS_LAUNCH("mlp_train", k_mlp_train_chunk, nchunks, 256, 0, s, theta, L.wt, features, targets, batch, inv_count,
            L.partials, L.loss_partials);
  const float bc1 = lr == 0.0f ? 1.0f : 1.0f - powf(beta1, (float)step);
  const float bc2 = lr == 0.0f ? 1.0f : 1.0f - powf(beta2, (float)step);
  GS_LAUNCH("mlp_train", k_mlp_reduce_adam, grid1(kNParams), 256, 0, s, theta, m, v, L.partials, nchunks,
            L.loss_partials, inv_count, lr, beta1, beta2, eps, bc1, bc2, grad, loss);
  return GS_OK;
}

}  // extern "C"
