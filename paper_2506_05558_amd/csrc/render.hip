// Per-tile compositing (forward) and its adjoint.
//
// One 256-lane workgroup (four wave64) per 16x16 tile, one lane per pixel;
// wave w owns the 8x8 quadrant (w & 1, w >> 1) of the tile, and its four
// 16-lane groups the 4x4 sub-blocks of that quadrant.  The tile's
// depth-ordered list is walked in batches (256 entries forward, 120 in the
// adjoint).  Each lane gathers one 64-byte render record, converts it to
// tile-relative form and stages it in LDS with one byte of support box (the
// 4-pixel columns and rows it meets); after a barrier each wave builds, with
// ballots over those bytes, the in-order lists of the batch entries whose box
// meets each of its four sub-blocks.  The four groups of a wave
// walk their own lists side by side (one entry per group per turn), so a
// small Gaussian costs nothing in the sub-blocks it cannot reach.  The
// workgroup leaves once all 256 pixels have stopped; a wave leaves its lists
// once its 64 pixels have.
//
// The 2D Gaussian is evaluated in the log2 domain: with d = pixel - mean,
//   s  = -(A dx^2 + 2 B dx dy + C dy^2) / 2,       alpha = o exp(s)
//   s2 = s log2(e) = ca dx^2 + cb dx dy + cc dy^2,  o exp(s) = 2^(s2 + log2 o)
// with (ca, cb, cc) = -log2(e) (A/2, B, C/2) and log2 o folded in at
// staging.  The skip test alpha >= alpha_min is taken on the exponent,
// s2 + log2 o >= log2 alpha_min, so a pair that no pixel of the wave keeps
// costs seven vector operations and no v_exp_f32.  The forward and the
// adjoint stage, cull and evaluate with the same code and explicit operation
// order, so the adjoint retraces the forward's decisions exactly.
#include <mutex>

#include "common.h"

namespace gsmi {
namespace {

constexpr int kThreads = 256;  // one workgroup per tile, one lane per pixel
constexpr int kBatch = 256;    // forward: tile-list entries staged per round
constexpr int kBwdBatch = 120; // adjoint: small enough for per-wave accumulators (no LDS atomics)
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kFar = 1e30f;  // pixel coordinate of a stopped pixel

struct RenderArgs {
  int W, H, tiles_x, ntiles;
  float bg0, bg1, bg2, alpha_max, alpha_min, t_min;
  const float *rec;
  const uint32_t *values, *ranges;
};

// NB staged entries and the lists of the 16 cull blocks: block 4 q + g is
// the 4x4 sub-block (g & 1, g >> 1) of the 8x8 quadrant (q & 1, q >> 1)
constexpr int kBlocks = 16;
template <int NB>
struct Stage {
  float4 a[NB];               // mean x, y relative to the tile origin, ca, cb
  float4 b[NB];               // cc, log2 opacity, depth, colour r
  float2 c[NB];               // colour g, b
  uint8_t box[NB];            // the 4-pixel columns (bits 0-3) and rows (bits 4-7) the support box meets
  uint8_t list[kBlocks][NB];  // per cull block: batch entries whose box meets it, in order
};

// The tile-list value (Gaussian index) lane t stages for the batch at base,
// loaded one batch ahead so that its latency overlaps the walk.
template <int NB>
__device__ __forceinline__ uint32_t batch_gid(const RenderArgs &a, uint32_t base, uint32_t end) {
  const uint32_t j = base + threadIdx.x;
  return threadIdx.x < NB && j < end ? a.values[j] : 0u;
}

// Stages entries [base, end) of the tile list (at most NB; lane t's value
// gid from batch_gid), then each wave builds the lists of its own four
// sub-blocks (read only by that wave).  Called by all 256 lanes; contains
// one barrier.  Returns the length of the calling lane's sub-block list.
template <int NB>
__device__ __forceinline__ int stage_batch(const RenderArgs &a, uint32_t base, uint32_t end, float ox, float oy,
                                           Stage<NB> &S, uint32_t gid) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4;
  const uint32_t j = base + t;
  if (t < NB) {
    unsigned box = 0;  // an entry past the end meets nothing
    if (j < end) {
      const float4 *r = (const float4 *)(a.rec + (size_t)gid * GS_REC_FLOATS);
      const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
      // integer part minus tile origin is exact; one rounding adds the fraction
      const float mx = __fadd_rn(__fsub_rn(r0.x, ox), r0.z);
      const float my = __fadd_rn(__fsub_rn(r0.y, oy), r0.w);
      S.a[t] = make_float4(mx, my, __fmul_rn(-0.5f * kLog2e, r1.x), __fmul_rn(-kLog2e, r1.y));
      S.b[t] = make_float4(__fmul_rn(-0.5f * kLog2e, r1.z), __builtin_amdgcn_logf(r1.w), r2.w, r2.x);
      S.c[t] = make_float2(r2.y, r2.z);
      // support box, widened so that FP32 rounding can never cull a pixel the
      // per-pixel test would accept
      const float hx = r3.x * (1.0f + 1e-4f) + 1e-3f, hy = r3.y * (1.0f + 1e-4f) + 1e-3f;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        box |= (unsigned)(mx - hx <= 4.0f * c + 3.0f && mx + hx >= 4.0f * c) << c;
        box |= (unsigned)(my - hy <= 4.0f * c + 3.0f && my + hy >= 4.0f * c) << (4 + c);
      }
    }
    S.box[t] = (uint8_t)box;
  }
  __syncthreads();
  // wave w's sub-blocks g = 0..3 lie in the 4-pixel columns 2 (w & 1) + (g & 1)
  // and rows 2 (w >> 1) + (g >> 1); entries in ascending order, 64 per round
  const int sx = 2 * (w & 1), sy = 4 + 2 * (w >> 1);
  const uint64_t lt = lanemask_lt();
  int n[4] = {0, 0, 0, 0};  // wave-uniform list lengths
#pragma unroll
  for (int r = 0; r < (NB + 63) / 64; ++r) {
    const int k = r * 64 + lane;
    const unsigned bx = k < NB ? S.box[k] : 0u;
    const unsigned cm = (bx >> sx) & 3u, rm = (bx >> sy) & 3u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool in = ((cm >> (q & 1)) & (rm >> (q >> 1)) & 1u) != 0;
      const uint64_t bal = ballot(in);
      if (in) S.list[4 * w + q][n[q] + __popcll(bal & lt)] = (uint8_t)k;
      n[q] += __popcll(bal);
    }
  }
  return g == 0 ? n[0] : g == 1 ? n[1] : g == 2 ? n[2] : n[3];
}

// log2-domain exponent of the 2D Gaussian at offset (dx, dy).
__device__ __forceinline__ float splat_s2(float ca, float cb, float cc, float dx, float dy) {
  const float t = __fmaf_rn(ca, dx, __fmul_rn(cb, dy));
  return __fmaf_rn(dx, t, __fmul_rn(__fmul_rn(cc, dy), dy));
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// min(alpha_max, raw) for raw = 2^x >= 0 (never NaN): one v_med3_f32
__device__ __forceinline__ float clamp_alpha(float raw, float alpha_max) {
  return __builtin_amdgcn_fmed3f(raw, 0.0f, alpha_max);
}

struct Pixel {
  int px, py, u, v;
  bool inside;
};

// The lanes 16 g .. 16 g + 15 of wave w are the 4x4 sub-block g of
// quadrant w, lane l its pixel (l & 3, (l >> 2) & 3).
__device__ __forceinline__ Pixel pixel_of(int tile, int tiles_x, int W, int H) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63, g = l >> 4;
  Pixel p;
  p.px = (w & 1) * 8 + (g & 1) * 4 + (l & 3);
  p.py = (w >> 1) * 8 + (g >> 1) * 4 + ((l >> 2) & 3);
  p.u = (tile % tiles_x) * GS_TILE + p.px;
  p.v = (tile / tiles_x) * GS_TILE + p.py;
  p.inside = p.u < W && p.v < H;
  return p;
}

// ------------------------------------------------------------------ forward
struct FwdOut {
  float *image, *depth, *alpha, *final_t;
  int32_t *n_contrib, *stats;
  // the fused L1 loss (LOSS): target image, gradient scale, dL/dimage and
  // per-tile partial sums [tile][2] of |image - target| and its square
  const float *target;
  float loss_scale;
  float *g_image;
  double *partials;
};

// LOSS: the L1 photometric loss is formed in the epilogue (the gradient
// and the tile's partial sums) while the pixel's colour is in registers.
template <bool STATS, bool LOSS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(STATS ? 1 : 8))) void k_render_fwd(RenderArgs a, FwdOut o) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= a.ntiles) return;  // uniform over the workgroup
  const int w = threadIdx.x >> 6;
  const Pixel P = pixel_of(tile, a.tiles_x, a.W, a.H);
  const uint32_t s = a.ranges[2 * tile], e = a.ranges[2 * tile + 1];
  const float ox = (float)((tile % a.tiles_x) * GS_TILE), oy = (float)((tile / a.tiles_x) * GS_TILE);
  // a pixel that has stopped (or lies outside the image) is moved far away:
  // its exponent is then -inf and it takes nothing more
  float fpx = P.inside ? (float)P.px : kFar;
  const float fpy = (float)P.py;
  const float l2min = __builtin_amdgcn_logf(a.alpha_min);

  __shared__ Stage<kBatch> S;

  float T = 1.0f, c0 = 0.f, c1 = 0.f, c2 = 0.f, D = 0.f;
  int last = 0, nev = 0, nsup = 0, ncomp = 0;
  int ntile = (int)(e - s);  // tile-list entries up to and including the stop
  const int blk = w * 4 + (threadIdx.x & 63) / 16;  // this lane's 4x4 cull block

  uint32_t gid = batch_gid<kBatch>(a, s, e);
  for (uint32_t base = s; base < e; base += kBatch) {
    if (__syncthreads_count(fpx == kFar) == kThreads) break;
    // the length of this lane's sub-block list (the same over its 16 lanes)
    const int cnt = stage_batch(a, base, e, ox, oy, S, gid);
    gid = batch_gid<kBatch>(a, base + kBatch, e);
    if (ballot(fpx != kFar) == 0) continue;
    const int idx0 = (int)(base - s);
    // the four sub-blocks of a wave walk their own lists side by side, four
    // entries per turn: all exponents first, then the four compositing steps
    // predicated per lane (a pixel that stops takes nothing more), and one
    // ballot per turn for the stops; a sub-block whose list is done or whose
    // pixels have all stopped sits out
    // four list entries per 32-bit read, the next turn's read issued a turn ahead
    int qn = cnt > 0 ? *(const int *)&S.list[blk][0] : 0;
    for (int i = 0;; i += 4) {
      const bool act = i < cnt && fpx != kFar;
      if (ballot(act) == 0) break;
      const int qd = qn;
      qn = i + 4 < cnt ? *(const int *)&S.list[blk][i + 4] : 0;
      int kk[4];
      float4 BB[4];
      float2 CC[4];
      float lg[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        kk[j] = i + j < cnt ? (qd >> (8 * j)) & 255 : (qd & 255);
        const float4 A = S.a[kk[j]];
        BB[j] = S.b[kk[j]];
        CC[j] = S.c[kk[j]];
        lg[j] = __fadd_rn(splat_s2(A.z, A.w, BB[j].x, __fsub_rn(fpx, A.x), __fsub_rn(fpy, A.y)), BB[j].y);
      }
      bool stopped = false;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // bitwise conditions: no branches inside a turn
        const bool live = act & (i + j < cnt) & !stopped;
        if (STATS) nev += live ? 1 : 0;
        const bool take = live & (lg[j] >= l2min);
        const float alpha = clamp_alpha(exp2_fast(lg[j]), a.alpha_max);
        const float2 C = CC[j];
        const float Tn = __fmul_rn(T, __fsub_rn(1.0f, alpha));
        const bool stop = take & (Tn < a.t_min);
        const bool comp = take & !stop;
        const float wgt = comp ? __fmul_rn(alpha, T) : 0.0f;
        c0 = __fmaf_rn(BB[j].w, wgt, c0);
        c1 = __fmaf_rn(C.x, wgt, c1);
        c2 = __fmaf_rn(C.y, wgt, c2);
        D = __fmaf_rn(BB[j].z, wgt, D);
        T = comp ? Tn : T;
        last = comp ? idx0 + kk[j] + 1 : last;
        if (STATS) {
          nsup += take ? 1 : 0;
          ncomp += comp ? 1 : 0;
          ntile = stop ? idx0 + kk[j] + 1 : ntile;
        }
        stopped = stopped | stop;
      }
      if (ballot(stopped) != 0) {
        fpx = stopped ? kFar : fpx;
        if (ballot(fpx != kFar) == 0) break;
      }
    }
  }
  const int64_t pix = (int64_t)P.v * a.W + P.u, np = (int64_t)a.W * a.H;
  const float v[3] = {__fmaf_rn(T, a.bg0, c0), __fmaf_rn(T, a.bg1, c1), __fmaf_rn(T, a.bg2, c2)};
  if (P.inside) {
    o.image[pix] = v[0];
    o.image[np + pix] = v[1];
    o.image[2 * np + pix] = v[2];
    o.depth[pix] = D;
    o.alpha[pix] = 1.0f - T;
    o.final_t[pix] = T;
    o.n_contrib[pix] = last;
    if (STATS) {
      o.stats[pix] = ntile;
      o.stats[np + pix] = nev;
      o.stats[2 * np + pix] = nsup;
      o.stats[3 * np + pix] = ncomp;
    }
  }
  if (LOSS) {
    // d = image - target as gs_loss_l1 forms it (the same binary32 values),
    // dL/dimage = scale sign(d) with exact zeros; the tile's sums of |d| and
    // d^2 in FP64, in a fixed order
    double s1 = 0.0, s2 = 0.0;
    if (P.inside) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float d = v[c] - o.target[c * np + pix];
        s1 += fabs((double)d);
        s2 += (double)d * (double)d;
        o.g_image[c * np + pix] = d > 0.f ? o.loss_scale : (d < 0.f ? -o.loss_scale : 0.f);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s1 += __shfl_down(s1, off, 64);
      s2 += __shfl_down(s2, off, 64);
    }
    __shared__ double red[4][2];
    if ((threadIdx.x & 63) == 0) {
      red[w][0] = s1;
      red[w][1] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      o.partials[2 * tile] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
      o.partials[2 * tile + 1] = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    }
  }
}

// Sum of the per-tile loss partials in a fixed order: 1024 lanes each add
// every 1024-th tile, then a wave tree and the 16 wave sums in order.
constexpr int kSumBlock = 1024;
__global__ __launch_bounds__(kSumBlock) void k_tile_loss_sums(const double *partials, int ntiles, double *sums) {
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < ntiles; k += kSumBlock) {
    a += partials[2 * k];
    b += partials[2 * k + 1];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  __shared__ double red[kSumBlock / 64][2];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w][0] = a;
    red[w][1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0.0, y = 0.0;
    for (int k = 0; k < kSumBlock / 64; ++k) {
      x += red[k][0];
      y += red[k][1];
    }
    sums[0] = x;
    sums[1] = y;
  }
}

// ------------------------------------------------------------------ adjoint
struct BwdIn {
  const float *image, *depth, *final_t;
  const int32_t *n_contrib;
  const float *g_image, *g_depth, *g_alpha;
  const uint32_t *slots;  // emission index of each sorted pair
  float *pair_grad;       // [M][12] per (Gaussian, tile) pair: the ten 2D gradients
};

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

constexpr int kChunk = 8;          // wave iterations handed from phase 1 to phase 2
constexpr uint8_t kNoEntry = 0xff;  // chunk slot of a sub-block that had no entry

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Per-wave chunk table, slot-major with the lane index XOR-ed by the slot:
// phase 1 (all lanes, one slot) writes a permutation of one row; phase 2
// (lane = sub-block g, slot e, half h) reads [e][(16 g + 8 h + i) ^ e], one
// lane per bank.
struct BwdShared {
  float gs[4][kChunk][64];  // per wave, chunk slot, lane ^ slot: d L / d s  (natural-log exponent)
  float wt[4][kChunk][64];  // per wave, chunk slot, lane ^ slot: blending weight alpha T
};

// Phase 2 of the adjoint for one wave: the sums of a chunk.  A chunk slot holds one entry per
// 4x4 sub-block (the four sub-blocks of a wave walk their own lists), so
// the lanes are (sub-block g = lane / 16, slot e, half h = lane % 2); each
// lane sums the 8 pixels of rows 2 h, 2 h + 1 of its sub-block, the two
// halves are combined with one DPP add, and the two lanes add the sums (five
// each) to the wave's own accumulator of that entry:
//   sum gs, gs dx, gs dy, gs dx^2, gs dx dy, gs dy^2 (the mean, conic and
//   opacity gradients are linear in these: d s / d mean = (A dx + B dy,
//   B dx + C dy), d alpha / d o = alpha / o), sum w G_c and sum w G_depth
//   (the colour and depth gradients).
// The lane's entry k (kNoEntry: the slot holds none) and its mean (mx, my)
// come from the sub-block's list: slot e of a chunk is list position
// 8 c + e, since every list entry takes a slot.  BwdCommit adds the sums to
// the accumulator.
// The values a lane adds in the five rounds of BwdCommit (round r: value
// (r + g) mod 5 of the lane's five).
struct Rot5 {
  float r0, r1, r2, r3, r4;
};

__device__ __forceinline__ float pick4(int g, float a, float b, float c, float d) {
  return g == 0 ? a : g == 1 ? b : g == 2 ? c : d;
}

template <bool DEPTH>
__device__ __forceinline__ Rot5 bwd_sums(BwdShared &B, int w, int k, float mx_, float my_, const float (&Gr)[4][8]) {
  constexpr int NQ = DEPTH ? 10 : 9;
  const int lane = threadIdx.x & 63, g = lane >> 4, e = (lane >> 1) & 7, h = lane & 1;
  float v[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) v[q] = 0.f;
  if (k != kNoEntry) {
    // pixel i of the lane sits at (x0 + ix, y0 + iy) from the mean, ix = i % 4, iy = i / 4
    const float x0 = (float)((w & 1) * 8 + (g & 1) * 4) - mx_;
    const float y0 = (float)((w >> 1) * 8 + (g >> 1) * 4 + 2 * h) - my_;
    float m0 = 0.f, mx = 0.f, my = 0.f, mxx = 0.f, mxy = 0.f, s0 = 0.f, s1 = 0.f, s2 = 0.f, sd = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int p = g * 16 + h * 8 + i;
      const float gs = B.gs[w][e][p ^ e], wt = B.wt[w][e][p ^ e];
      const int ix = i & 3, iy = i >> 2;
      if (i == 0) {  // the sums start at the first term (no add of zero)
        m0 = gs;
        s0 = wt * Gr[0][0];
        s1 = wt * Gr[1][0];
        s2 = wt * Gr[2][0];
        if (DEPTH) sd = wt * Gr[3][0];
        continue;
      }
      m0 += gs;
      if (ix == 1) mx = i == 1 ? gs : mx + gs;
      if (ix > 1) mx = __fmaf_rn(gs, (float)ix, mx);
      if (ix == 1) mxx = i == 1 ? gs : mxx + gs;
      if (ix > 1) mxx = __fmaf_rn(gs, (float)(ix * ix), mxx);
      if (iy) my = i == 4 ? gs : my + gs;
      if (iy && ix == 1) mxy = gs;
      if (iy && ix > 1) mxy = __fmaf_rn(gs, (float)ix, mxy);
      s0 = __fmaf_rn(wt, Gr[0][i], s0);
      s1 = __fmaf_rn(wt, Gr[1][i], s1);
      s2 = __fmaf_rn(wt, Gr[2][i], s2);
      if (DEPTH) sd = __fmaf_rn(wt, Gr[3][i], sd);
    }
    // about the mean: dx = x0 + ix, dy = y0 + iy (iy^2 = iy)
    v[0] = m0;
    v[1] = __fmaf_rn(x0, m0, mx);                                               // sum gs dx
    v[2] = __fmaf_rn(y0, m0, my);                                               // sum gs dy
    v[3] = __fmaf_rn(x0, __fmaf_rn(x0, m0, 2.0f * mx), mxx);                    // sum gs dx^2
    v[4] = __fmaf_rn(x0, __fmaf_rn(y0, m0, my), __fmaf_rn(y0, mx, mxy));        // sum gs dx dy
    v[5] = __fmaf_rn(y0, __fmaf_rn(y0, m0, 2.0f * my), my);                     // sum gs dy^2
    v[6] = s0;
    v[7] = s1;
    v[8] = s2;
    v[9] = sd;
  }
  // the two halves of a (sub-block, slot) are neighbouring lanes
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] += dpp_mov<0xb1, 0xf>(v[q]);  // quad_perm [1,0,3,2]
  // both lanes of a (sub-block, slot) hold the sums: lane h adds sums
  // 5 h .. 5 h + 4, in the order of the rounds
  const float u0 = h ? v[5] : v[0], u1 = h ? v[6] : v[1], u2 = h ? v[7] : v[2], u3 = h ? v[8] : v[3];
  const float u4 = h ? (NQ > 9 ? v[9] : 0.f) : v[4];
  Rot5 o;
  o.r0 = pick4(g, u0, u1, u2, u3);
  o.r1 = pick4(g, u1, u2, u3, u4);
  o.r2 = pick4(g, u2, u3, u4, u0);
  o.r3 = pick4(g, u3, u4, u0, u1);
  o.r4 = pick4(g, u4, u0, u1, u2);
  return o;
}

typedef __attribute__((address_space(3))) float lds_float;

// One lane's part of adding a chunk's sums (bwd_sums: entry k, rotated
// values) to the wave's accumulator, in five rounds of one read-modify-write:
// in round r the lane of sub-block g adds its value (r + g) mod 5, so the
// four sub-blocks of a round always write different rows and two lanes of a
// round never share an address, even where sub-blocks hold the same entry;
// no other wave writes this accumulator.
// The accesses are volatile, so the rounds stay in order (an address written
// in one round may be read in a later one); the caller spreads them over a
// turn's arithmetic to hide their latency.  A lane with nothing to add in a
// round reads and writes its own cell `dummy` instead, which no other lane
// touches and which the caller overwrites before it reads it.
template <bool DEPTH>
struct BwdCommit {
  volatile lds_float *p[5];
  float val[5];
  __device__ __forceinline__ BwdCommit(float (*acc)[kBwdBatch], int k, const Rot5 &c, float *dummy) {
    constexpr int NQ = DEPTH ? 10 : 9;
    const int lane = threadIdx.x & 63, g = lane >> 4, h = lane & 1;
    const bool has = k != kNoEntry;
    lds_float *col = (lds_float *)&acc[5 * h][has ? k : 0];
    lds_float *dum = (lds_float *)dummy;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      const int q = r + g >= 5 ? r + g - 5 : r + g;
      p[r] = has && 5 * h + q < NQ ? col + q * kBwdBatch : dum;
    }
    val[0] = c.r0;
    val[1] = c.r1;
    val[2] = c.r2;
    val[3] = c.r3;
    val[4] = c.r4;
  }
  __device__ __forceinline__ float read(int r) const { return *p[r]; }
  __device__ __forceinline__ void write(int r, float old) const { *p[r] = old + val[r]; }
};

// DEPTH: a depth gradient is given (without one, the depth sums are skipped)
template <bool DEPTH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DEPTH ? 3 : 4))) void k_render_bwd(RenderArgs a, BwdIn bi) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= a.ntiles) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, g = lane >> 4, blk = w * 4 + g;
  const Pixel P = pixel_of(tile, a.tiles_x, a.W, a.H);
  const uint32_t s = a.ranges[2 * tile], e = a.ranges[2 * tile + 1];
  const float ox = (float)((tile % a.tiles_x) * GS_TILE), oy = (float)((tile / a.tiles_x) * GS_TILE);
  const float fpx = (float)P.px, fpy = (float)P.py;

  constexpr int NQ = DEPTH ? 10 : 9;  // accumulated sums per entry
  __shared__ Stage<kBwdBatch> S;
  __shared__ float sAcc[4][NQ][kBwdBatch];  // per wave
  __shared__ BwdShared B;
  __shared__ int sMax;

  const int64_t pix = (int64_t)P.v * a.W + P.u, np = (int64_t)a.W * a.H;
  int ncon = 0;
  float G0 = 0.f, G1 = 0.f, G2 = 0.f, GD = 0.f, GA = 0.f, GI = 0.f, Tf = 1.f;
  if (P.inside) {
    ncon = bi.n_contrib[pix];
    G0 = bi.g_image[pix];
    G1 = bi.g_image[np + pix];
    G2 = bi.g_image[2 * np + pix];
    GD = DEPTH ? bi.g_depth[pix] : 0.f;
    GA = bi.g_alpha ? bi.g_alpha[pix] : 0.f;
    // G . (everything the pixel outputs): colour incl. background, and depth
    GI = G0 * bi.image[pix] + G1 * bi.image[np + pix] + G2 * bi.image[2 * np + pix] +
         (DEPTH ? GD * bi.depth[pix] : 0.f);
    Tf = bi.final_t[pix];
  }
  B.gs[w][0][lane] = G0;  // staged in the (not yet used) chunk table
  B.gs[w][1][lane] = G1;
  B.gs[w][2][lane] = G2;
  B.gs[w][3][lane] = GD;
  if (t == 0) sMax = 0;
  {  // the accumulators start at zero; afterwards each batch's writer clears what it read
    float4 *z = (float4 *)&sAcc[0][0][0];
    for (int i = t; i < 4 * NQ * kBwdBatch / 4; i += kThreads) z[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();
  // the phase 2 lane (sub-block g, half h) sums over the lanes 16 g + 8 h ..
  // 16 g + 8 h + 7 of its wave: their upstream gradients stay in registers
  float Gr[4][8];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int i = 0; i < 8; ++i) Gr[c][i] = B.gs[w][c][g * 16 + (lane & 1) * 8 + i];
  // the last contributor of any pixel of the sub-block, and of the tile
  int gmax = ncon;
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) gmax = max(gmax, __shfl_xor(gmax, off, 64));
  const int wmax = __builtin_amdgcn_readfirstlane(wave_max(gmax));
  if (lane == 0 && wmax > 0) atomicMax(&sMax, wmax);
  __syncthreads();
  const uint32_t stop = min(s + (uint32_t)sMax, e);

  // T: transmittance before the entry; GP: G . (colour, depth) composited so far.
  // d alpha_k = T_k (G . c_k) - (G . suffix_k) / (1 - alpha_k) + G_alpha T_final / (1 - alpha_k)
  // with G . suffix_k = GI - GP_k (GP_k includes entry k).
  float T = 1.0f, GP = 0.f;
  const float GAT = GA * Tf;
  const float l2min = __builtin_amdgcn_logf(a.alpha_min);

  // No barrier opens a batch: lane t stages entry t and is also the lane that wrote out
  // entry t of the previous batch and cleared its accumulator column, so its own program
  // order covers those; the other lanes' accumulator writes come after the staging
  // barrier, and the walk of the previous batch (with its wave's list building) ended at
  // the barrier before its write-out.
  const int pe = (lane >> 1) & 7;  // this lane's phase 2 chunk slot
  // the values and pair slots of the next batch are loaded during the walk of this one
  uint32_t gid = batch_gid<kBwdBatch>(a, s, stop);
  uint32_t slot = t < kBwdBatch && s + t < stop ? bi.slots[s + t] : 0u;
  for (uint32_t base = s; base < stop; base += kBwdBatch) {
    // the length of this lane's sub-block list (the same over its 16 lanes)
    const int cnt = stage_batch(a, base, stop, ox, oy, S, gid);
    const uint32_t my_slot = slot;
    gid = batch_gid<kBwdBatch>(a, base + kBwdBatch, stop);
    slot = t < kBwdBatch && base + kBwdBatch + t < stop ? bi.slots[base + kBwdBatch + t] : 0u;
    const int idx0 = (int)(base - s);
    const int nrel = ncon - idx0;  // batch entries below nrel come before this pixel's last contributor
    // Every list entry takes a chunk slot, so a chunk is two turns.  The
    // sums of a chunk are added to the accumulator at the start of the next
    // (or after the walk), where the adds overlap that turn's arithmetic.
    int ck = kNoEntry;  // the pending sums: entry and values
    Rot5 cu = {0.f, 0.f, 0.f, 0.f, 0.f};
    // one turn: entries i .. i + 3 of the sub-block list into slots e0 .. e0 + 3
    // four list entries per 32-bit read, the next turn's read issued a turn ahead
    int qn = cnt > 0 ? *(const int *)&S.list[blk][0] : 0;
    auto turn = [&](int i, int e0, bool commit_first) -> bool {
      const int qd = qn;
      qn = i + 4 < cnt ? *(const int *)&S.list[blk][i + 4] : 0;
      const bool act = i < cnt && idx0 + (qd & 255) < gmax;  // lists ascend
      if (ballot(act) == 0) return false;
      int kk[4];
      float4 BB[4];
      float2 CC[4];
      float lg[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        kk[j] = i + j < cnt ? (qd >> (8 * j)) & 255 : (qd & 255);
        const float4 A = S.a[kk[j]];
        BB[j] = S.b[kk[j]];
        CC[j] = S.c[kk[j]];
        lg[j] = __fadd_rn(splat_s2(A.z, A.w, BB[j].x, __fsub_rn(fpx, A.x), __fsub_rn(fpy, A.y)), BB[j].y);
      }
      // the pending sums: round j is read before body j and written after it, round 4 after
      // body 3; a lane's dummy cell is the one its own body of slot 7 writes
      const BwdCommit<DEPTH> cm(sAcc[w], commit_first ? ck : (int)kNoEntry, cu, &B.wt[w][7][lane ^ 7]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float old = commit_first ? cm.read(j) : 0.f;
        // bitwise conditions: no branches in a turn, so that its parts can interleave
        const bool live = act & (i + j < cnt);
        const bool take = live & (kk[j] < nrel) & (lg[j] >= l2min);
        const float4 &Bv = BB[j];
        const float raw = exp2_fast(lg[j]);
        // alpha where the pixel takes the entry, else 0 (then the weight is 0 and T stays)
        const float ae = take ? clamp_alpha(raw, a.alpha_max) : 0.0f;
        const float2 C = CC[j];
        const float wgt = __fmul_rn(ae, T);
        const float om = __fsub_rn(1.0f, ae);
        const float gc = DEPTH ? G0 * Bv.w + G1 * C.x + G2 * C.y + GD * Bv.z : G0 * Bv.w + G1 * C.x + G2 * C.y;
        GP = __fmaf_rn(wgt, gc, GP);
        const float inv = __builtin_amdgcn_rcpf(om);
        const float dalpha = T * gc + (GAT - GI + GP) * inv;
        const bool livegrad = take & (raw < a.alpha_max);  // the clamp passes no gradient
        // row e0 + j, column lane ^ (e0 + j): flat index lane ^ (65 (e0 + j))
        const int sw = lane ^ ((e0 + j) * 65);
        (&B.gs[w][0][0])[sw] = livegrad ? dalpha * raw : 0.0f;  // d alpha / d s = alpha
        (&B.wt[w][0][0])[sw] = wgt;
        T = __fmul_rn(T, om);
        if (commit_first) cm.write(j, old);
      }
      if (commit_first) cm.write(4, cm.read(4));
      return true;
    };
    for (int i = 0;; i += 8) {
      // this lane's phase 2 entry: list position i + pe of its sub-block (every list entry
      // takes a slot), read ahead of the two turns, and that entry's mean
      const bool pin = i + pe < cnt;
      const int pw = *(const int *)&S.list[blk][i + (pe & 4)];
      const int pkk = pin ? (pw >> (8 * (pe & 3))) & 255 : 0;
      const float2 pm = *(const float2 *)&S.a[pkk];
      if (!turn(i, 0, true)) break;  // the previous chunk's sums are added here
      const bool more = turn(i + 4, 4, false);
      // a slot of a turn that did not run holds no entry; one that ran for the wave but not
      // for this sub-block holds zeros
      const int pk = pin && (pe < 4 || more) ? pkk : (int)kNoEntry;
      cu = bwd_sums<DEPTH>(B, w, pk, pm.x, pm.y, Gr);
      ck = pk;
      if (!more) break;
    }
    {
      const BwdCommit<DEPTH> cm(sAcc[w], ck, cu, &B.wt[w][7][lane ^ 7]);
#pragma unroll
      for (int r = 0; r < 5; ++r) cm.write(r, cm.read(r));
    }
    __syncthreads();
    // one plain store per (tile, entry): the pair's slot is owned by this tile.
    // From the sums (gs, gs dx, gs dy, gs dx^2, gs dx dy, gs dy^2, w G_c, w G_depth):
    // with A = -2 ca ln2, B = -cb ln2, C = -2 cc ln2,
    //   d mean = -(A sum gs dx + B sum gs dy, B sum gs dx + C sum gs dy)
    //   d (A, B, C) = -(sum gs dx^2 / 2, sum gs dx dy, sum gs dy^2 / 2)
    //   d o = sum gs / o   (d alpha / d o = alpha / o)
    //   d colour = sum w G_c for a channel above 0; 0 for one the projection clamped at 0
    //   (the colour is max(SH value, 0): such a channel passes nothing to the SH terms)
    if (t < kBwdBatch && base + t < stop) {
      float v[10];
#pragma unroll
      for (int q = 0; q < 10; ++q)
        v[q] = q < NQ ? (sAcc[0][q][t] + sAcc[1][q][t]) + (sAcc[2][q][t] + sAcc[3][q][t]) : 0.f;
      const float4 A = S.a[t], Bb = S.b[t];
      const float2 Cc = S.c[t];
      float4 *dst = (float4 *)(bi.pair_grad + (size_t)my_slot * 12);
      dst[0] = make_float4(-kLn2 * (2.0f * A.z * v[1] + A.w * v[2]), -kLn2 * (A.w * v[1] + 2.0f * Bb.x * v[2]),
                           -0.5f * v[3], -v[4]);
      dst[1] = make_float4(-0.5f * v[5], v[0] * exp2_fast(-Bb.y), Bb.w > 0.f ? v[6] : 0.f, Cc.x > 0.f ? v[7] : 0.f);
      dst[2] = make_float4(Cc.y > 0.f ? v[8] : 0.f, v[9], 0.f, 0.f);
    }
    if (t < kBwdBatch) {  // clear column t of the four accumulators for the next batch
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        sAcc[0][q][t] = 0.f;
        sAcc[1][q][t] = 0.f;
        sAcc[2][q][t] = 0.f;
        sAcc[3][q][t] = 0.f;
      }
    }
  }
  // entries past the last contributor of every pixel receive nothing from this tile
  for (uint32_t j = stop + t; j < e; j += kThreads) {
    float4 *dst = (float4 *)(bi.pair_grad + (size_t)bi.slots[j] * 12);
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    dst[0] = z;
    dst[1] = z;
    dst[2] = z;
  }
}

}  // namespace

gs_status validate_camera(const gs_camera *cam, const char *fn);
gs_status validate_gaussians(const gs_gaussians *g, const char *fn);

static RenderArgs render_args(const gs_camera *cam, const gs_raster_params *rp, const gs_projected *proj,
                              const uint32_t *values, const uint32_t *ranges) {
  RenderArgs a;
  a.W = cam->width;
  a.H = cam->height;
  a.tiles_x = tiles_x_of(cam->width);
  a.ntiles = a.tiles_x * tiles_y_of(cam->height);
  a.bg0 = cam->bg[0];
  a.bg1 = cam->bg[1];
  a.bg2 = cam->bg[2];
  a.alpha_max = rp->alpha_max;
  a.alpha_min = rp->alpha_min;
  a.t_min = rp->t_min;
  a.rec = proj->rec;
  a.values = values;
  a.ranges = ranges;
  return a;
}

static int padded_grid(int ntiles) { return (ntiles + 7) / 8 * 8; }

// GS_CHECK_FINITE: the image and depth a render wrote
static gs_status check_frame(const gs_camera *cam, const float *image, const float *depth, const char *fn,
                             hipStream_t s) {
  if (!finite_checks_on()) return GS_OK;
  const int64_t np = (int64_t)cam->width * cam->height;
  gs_status st = check_finite(image, 3 * np, fn, "image", s);
  if (st != GS_OK) return st;
  return check_finite(depth, np, fn, "depth", s);
}

// ---------------------------------------------- fixed scratch (no allocation)
// The per-tile loss partials of gs_render_fwd_l1_noalloc live in a
// file-scope device array: each GPU the library runs on holds its own copy
// (2 doubles per tile, 1 MiB) until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in symbol):
// its device address is looked up once per device with hipGetSymbolAddress
// and kept in g_scratch_ptr.
constexpr int kNoAllocMaxTiles = 65536;
static __device__ __align__(256) double scratch[2 * kNoAllocMaxTiles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// The current device's address of `scratch`, looked up on the first call on
// that device.
static gs_status noalloc_scratch(double **out) {
  int dev = -1;
  GS_CHECK_HIP(hipGetDevice(&dev), "hipGetDevice");
  GS_REQUIRE(dev >= 0 && dev < kMaxDevices, "gs_render_fwd_l1_noalloc: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    GS_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    GS_REQUIRE(ptr != nullptr, "gs_render_fwd_l1_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = (double *)g_scratch_ptr[dev];
  return GS_OK;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_render_fwd(const gs_camera *cam, const gs_raster_params *rp, const gs_projected *proj,
                        const uint32_t *values, const uint32_t *ranges, float *image, float *depth, float *alpha,
                        float *final_t, int32_t *n_contrib, int32_t *stats, void *stream) {
  gs_status st = validate_camera(cam, "gs_render_fwd");
  if (st != GS_OK) return st;
  GS_REQUIRE(rp && proj && ranges && image && depth && alpha && final_t && n_contrib,
             "gs_render_fwd: NULL argument");
  GS_REQUIRE(rp->alpha_max > 0.f && rp->alpha_max < 1.f && rp->t_min > 0.f && rp->t_min < 1.f,
             "gs_render_fwd: raster params out of range");
  RenderArgs a = render_args(cam, rp, proj, values, ranges);
  FwdOut o{image, depth, alpha, final_t, n_contrib, stats, nullptr, 0.f, nullptr, nullptr};
  if (stats)
    GS_LAUNCH("render_fwd", (k_render_fwd<true, false>), padded_grid(a.ntiles), 256, 0, (hipStream_t)stream, a, o);
  else
    GS_LAUNCH("render_fwd", (k_render_fwd<false, false>), padded_grid(a.ntiles), 256, 0, (hipStream_t)stream, a, o);
  return check_frame(cam, image, depth, "gs_render_fwd", (hipStream_t)stream);
}

gs_status gs_render_fwd_l1_workspace(int32_t width, int32_t height, size_t *bytes) {
  GS_REQUIRE(bytes && width > 0 && height > 0, "gs_render_fwd_l1_workspace: bad argument");
  *bytes = align_up(2 * sizeof(double) * (size_t)tiles_x_of(width) * (size_t)tiles_y_of(height));
  return GS_OK;
}

gs_status gs_render_fwd_l1(const gs_camera *cam, const gs_raster_params *rp, const gs_projected *proj,
                           const uint32_t *values, const uint32_t *ranges, float *image, float *depth, float *alpha,
                           float *final_t, int32_t *n_contrib, const float *target, float grad_scale,
                           float *dL_dimage, double *sums, void *ws, size_t ws_bytes, void *stream) {
  gs_status st = validate_camera(cam, "gs_render_fwd_l1");
  if (st != GS_OK) return st;
  GS_REQUIRE(rp && proj && ranges && image && depth && alpha && final_t && n_contrib && target && dL_dimage && sums,
             "gs_render_fwd_l1: NULL argument");
  GS_REQUIRE(rp->alpha_max > 0.f && rp->alpha_max < 1.f && rp->t_min > 0.f && rp->t_min < 1.f,
             "gs_render_fwd_l1: raster params out of range");
  size_t need = 0;
  gs_render_fwd_l1_workspace(cam->width, cam->height, &need);
  if (ws_bytes < need || !ws) {
    set_error("gs_render_fwd_l1: workspace %zu bytes < %zu", ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  RenderArgs a = render_args(cam, rp, proj, values, ranges);
  FwdOut o{image, depth, alpha, final_t, n_contrib, nullptr, target, grad_scale, dL_dimage, (double *)ws};
  GS_LAUNCH("render_fwd", (k_render_fwd<false, true>), padded_grid(a.ntiles), 256, 0, (hipStream_t)stream, a, o);
  GS_LAUNCH("loss_final", k_tile_loss_sums, 1, kSumBlock, 0, (hipStream_t)stream, (const double *)ws, a.ntiles,
            sums);
  return check_frame(cam, image, depth, "gs_render_fwd_l1", (hipStream_t)stream);
}

gs_status gs_render_fwd_l1_noalloc(const gs_camera *cam, const gs_raster_params *rp, const gs_projected *proj,
                                   const uint32_t *values, const uint32_t *ranges, float *image, float *depth,
                                   float *alpha, float *final_t, int32_t *n_contrib, const float *target,
                                   float grad_scale, float *dL_dimage, double *sums, void *stream) {
  gs_status st = validate_camera(cam, "gs_render_fwd_l1_noalloc");
  if (st != GS_OK) return st;
  GS_REQUIRE(rp && proj && ranges && image && depth && alpha && final_t && n_contrib && target && dL_dimage && sums,
             "gs_render_fwd_l1_noalloc: NULL argument");
  GS_REQUIRE(rp->alpha_max > 0.f && rp->alpha_max < 1.f && rp->t_min > 0.f && rp->t_min < 1.f,
             "gs_render_fwd_l1_noalloc: raster params out of range");
  const int64_t ntiles = (int64_t)tiles_x_of(cam->width) * tiles_y_of(cam->height);
  GS_REQUIRE(ntiles <= kNoAllocMaxTiles, "gs_render_fwd_l1_noalloc: %lld tiles exceed the fixed scratch of %d tiles",
             (long long)ntiles, kNoAllocMaxTiles);
  double *partials = nullptr;
  if ((st = noalloc_scratch(&partials)) != GS_OK) return st;
  RenderArgs a = render_args(cam, rp, proj, values, ranges);
  FwdOut o{image, depth, alpha, final_t, n_contrib, nullptr, target, grad_scale, dL_dimage, partials};
  // launched without the profiling bracket (its events are created on demand)
  // every tile writes its own two partials: nothing in the scratch needs clearing
  hipLaunchKernelGGL((k_render_fwd<false, true>), dim3(padded_grid(a.ntiles)), dim3(256), 0, (hipStream_t)stream, a,
                     o);
  GS_CHECK_HIP(hipGetLastError(), "render_fwd");
  hipLaunchKernelGGL(k_tile_loss_sums, dim3(1), dim3(kSumBlock), 0, (hipStream_t)stream, (const double *)partials,
                     a.ntiles, sums);
  GS_CHECK_HIP(hipGetLastError(), "loss_final");
  return GS_OK;
}

gs_status gs_render_bwd_pairs(const gs_camera *cam, const gs_raster_params *rp, const gs_projected *proj,
                              const uint32_t *values, const uint32_t *slots, const uint32_t *ranges,
                              int64_t n_instances, const float *image, const float *depth, const float *final_t,
                              const int32_t *n_contrib, const float *dL_dimage, const float *dL_ddepth,
                              const float *dL_dalpha, float *pair_grad, void *stream) {
  gs_status st = validate_camera(cam, "gs_render_bwd_pairs");
  if (st != GS_OK) return st;
  GS_REQUIRE(rp && proj && ranges && image && depth && final_t && n_contrib && dL_dimage,
             "gs_render_bwd_pairs: NULL argument");
  GS_REQUIRE(n_instances >= 0, "gs_render_bwd_pairs: n_instances < 0");
  if (n_instances > 0) GS_REQUIRE(values && slots && pair_grad, "gs_render_bwd_pairs: NULL list argument");
  RenderArgs a = render_args(cam, rp, proj, values, ranges);
  BwdIn bi{image, depth, final_t, n_contrib, dL_dimage, dL_ddepth, dL_dalpha, slots, pair_grad};
  if (dL_ddepth)
    GS_LAUNCH("render_bwd", k_render_bwd<true>, padded_grid(a.ntiles), 256, 0, (hipStream_t)stream, a, bi);
  else
    GS_LAUNCH("render_bwd", k_render_bwd<false>, padded_grid(a.ntiles), 256, 0, (hipStream_t)stream, a, bi);
  return GS_OK;
}

gs_status gs_render_bwd_workspace(int64_t n, int64_t n_instances, size_t *bytes) {
  GS_REQUIRE(bytes && n >= 0 && n_instances >= 0, "gs_render_bwd_workspace: bad argument");
  size_t pose = 0;
  gs_project_bwd_views_workspace(n, 1, &pose);
  *bytes = align_up(sizeof(float) * 12 * (size_t)n_instances) + pose;
  return GS_OK;
}

gs_status gs_render_bwd(const gs_camera *cam, const gs_raster_params *rp, const gs_gaussians *g,
                        const gs_projected *proj, const uint32_t *values, const uint32_t *slots,
                        const uint32_t *ranges, const uint32_t *first_slot, int64_t n_instances, const float *image,
                        const float *depth, const float *final_t, const int32_t *n_contrib, const float *dL_dimage,
                        const float *dL_ddepth, const float *dL_dalpha, gs_gaussians *grads, double *dL_dpose,
                        double *dL_dtwist, void *ws, size_t ws_bytes, void *stream) {
  gs_status st = validate_camera(cam, "gs_render_bwd");
  if (st != GS_OK) return st;
  if ((st = validate_gaussians(g, "gs_render_bwd")) != GS_OK) return st;
  if ((st = validate_gaussians(grads, "gs_render_bwd(grads)")) != GS_OK) return st;
  GS_REQUIRE(grads->n == g->n && grads->sh_degree == g->sh_degree, "gs_render_bwd: grads shape differs from g");
  GS_REQUIRE(rp && proj && ranges && image && depth && final_t && n_contrib && dL_dimage,
             "gs_render_bwd: NULL argument");
  GS_REQUIRE(n_instances >= 0, "gs_render_bwd: n_instances < 0");
  if (n_instances > 0) GS_REQUIRE(values && slots && first_slot, "gs_render_bwd: NULL list argument");
  size_t need = 0;
  gs_render_bwd_workspace(g->n, n_instances, &need);
  if (ws_bytes < need || (need && !ws)) {
    set_error("gs_render_bwd: workspace %zu bytes < %zu", ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  const bool checks = finite_checks_on();
  const int64_t np = (int64_t)cam->width * cam->height;
  hipStream_t hs = (hipStream_t)stream;
  if (checks) {
    if ((st = check_finite(dL_dimage, 3 * np, "gs_render_bwd", "dL_dimage", hs)) != GS_OK) return st;
    if ((st = check_finite(dL_ddepth, np, "gs_render_bwd", "dL_ddepth", hs)) != GS_OK) return st;
    if ((st = check_finite(dL_dalpha, np, "gs_render_bwd", "dL_dalpha", hs)) != GS_OK) return st;
  }
  Carve cv(ws);
  float *pair_grad = cv.take<float>(12 * (size_t)n_instances);
  size_t pose_bytes = 0;
  gs_project_bwd_views_workspace(g->n, 1, &pose_bytes);
  void *pose_ws = cv.take<char>(pose_bytes);
  if ((st = gs_render_bwd_pairs(cam, rp, proj, values, slots, ranges, n_instances, image, depth, final_t,
                                n_contrib, dL_dimage, dL_ddepth, dL_dalpha, pair_grad, stream)) != GS_OK)
    return st;
  // Without a (Gaussian, tile) pair no pixel depends on any Gaussian or on the
  // pose: every gradient this call would add is zero, and the accumulating
  // outputs stay as they are.  (The projection adjoint reads a first slot per
  // Gaussian, which the caller need not provide in that case.)
  if (g->n == 0 || n_instances == 0) return GS_OK;
  gs_view view;
  view.cam = *cam;
  view.proj = *proj;
  view.pair_grad = pair_grad;
  view.first_slot = first_slot;
  view.dL_dpose = dL_dpose;
  view.dL_dtwist = dL_dtwist;
  if ((st = gs_project_bwd_views(1, &view, rp, g, grads, pose_ws, pose_bytes, stream)) != GS_OK) return st;
  if (checks) {
    if ((st = check_finite_gaussians(grads, "gs_render_bwd", "grads", hs)) != GS_OK) return st;
    if ((st = check_finite_d(dL_dpose, 12, "gs_render_bwd", "dL_dpose", hs)) != GS_OK) return st;
    if ((st = check_finite_d(dL_dtwist, 6, "gs_render_bwd", "dL_dtwist", hs)) != GS_OK) return st;
  }
  return GS_OK;
}

}  // extern "C"
