// Per-tile compositing (forward) and its adjoint.
//
// One 256-lane workgroup (four wave64) per 16x16 tile, one lane per pixel;
// wave w owns the 8x8 quadrant (w & 1, w >> 1) of the tile.  The tile's
// depth-ordered list is walked in batches of 256 entries.  Each lane gathers
// one 64-byte render record, converts it to tile-relative form and stages it
// in LDS, and tests the entry's support box against the four quadrants;
// ballots then build, per quadrant, the in-order list of the batch entries
// whose box meets it.  Each wave walks only its own list, reading staged
// entries with broadcast LDS loads, so a small Gaussian costs nothing in the
// quadrants it cannot reach.  The workgroup leaves once all 256 pixels have
// stopped; a wave leaves its list once its 64 pixels have.
//
// The 2D Gaussian is evaluated in the log2 domain: with d = pixel - mean,
//   s  = -(A dx^2 + 2 B dx dy + C dy^2) / 2,       alpha = o exp(s)
//   s2 = s log2(e) = ca dx^2 + cb dx dy + cc dy^2,  exp(s) = 2^s2
// with (ca, cb, cc) = -log2(e) (A/2, B, C/2) folded in at staging, so one
// v_exp_f32 per pair.  The forward and the adjoint stage, cull and evaluate
// with the same code and explicit operation order, so the adjoint retraces
// the forward's decisions exactly.
#include "common.h"

namespace gsmi {
namespace {

constexpr int kBatch = 256;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

struct RenderArgs {
  int W, H, tiles_x, ntiles;
  float bg0, bg1, bg2, alpha_max, alpha_min, t_min;
  const float *rec;
  const uint32_t *values, *ranges;
};

struct Stage {
  float4 a[kBatch];         // mean x, y relative to the tile origin, ca, cb
  float4 b[kBatch];         // cc, opacity, depth, -
  float4 c[kBatch];         // colour r, g, b, -
  uint8_t list[4][kBatch];  // per quadrant: batch entries whose box meets it, in order
  int cnt[4][4];            // [entry wave][quadrant] entries
};

// Stages entries [base, end) of the tile list (at most kBatch) and builds the
// per-quadrant lists.  Called by all 256 lanes; contains two barriers.
__device__ __forceinline__ void stage_batch(const RenderArgs &a, uint32_t base, uint32_t end, float ox, float oy,
                                            Stage &S, uint32_t *gid_out) {
  const int t = threadIdx.x, lane = t & 63, ew = t >> 6;
  const uint32_t j = base + t;
  unsigned mask = 0;
  if (j < end) {
    const uint32_t gid = a.values[j];
    const float4 *r = (const float4 *)(a.rec + (size_t)gid * GS_REC_FLOATS);
    const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
    // integer part minus tile origin is exact; one rounding adds the fraction
    const float mx = __fadd_rn(__fsub_rn(r0.x, ox), r0.z);
    const float my = __fadd_rn(__fsub_rn(r0.y, oy), r0.w);
    S.a[t] = make_float4(mx, my, __fmul_rn(-0.5f * kLog2e, r1.x), __fmul_rn(-kLog2e, r1.y));
    S.b[t] = make_float4(__fmul_rn(-0.5f * kLog2e, r1.z), r1.w, r2.w, 0.0f);
    S.c[t] = make_float4(r2.x, r2.y, r2.z, 0.0f);
    if (gid_out) gid_out[t] = gid;
    // support box, widened so that FP32 rounding can never cull a pixel the
    // per-pixel test would accept
    const float hx = r3.x * (1.0f + 1e-4f) + 1e-3f, hy = r3.y * (1.0f + 1e-4f) + 1e-3f;
    const bool x0 = mx - hx <= 7.0f && mx + hx >= 0.0f;
    const bool x1 = mx - hx <= 15.0f && mx + hx >= 8.0f;
    const bool y0 = my - hy <= 7.0f && my + hy >= 0.0f;
    const bool y1 = my - hy <= 15.0f && my + hy >= 8.0f;
    mask = (unsigned)(x0 && y0) | (unsigned)(x1 && y0) << 1 | (unsigned)(x0 && y1) << 2 | (unsigned)(x1 && y1) << 3;
  }
  const uint64_t lt = lanemask_lt();
  int rank[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint64_t bal = __ballot((mask >> q) & 1u);
    rank[q] = __popcll(bal & lt);
    if (lane == 0) S.cnt[ew][q] = __popcll(bal);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if ((mask >> q) & 1u) {
      int off = rank[q];
      for (int w = 0; w < ew; ++w) off += S.cnt[w][q];
      S.list[q][off] = (uint8_t)t;
    }
  }
  __syncthreads();
}

// log2-domain exponent of the 2D Gaussian at offset (dx, dy).
__device__ __forceinline__ float splat_s2(float ca, float cb, float cc, float dx, float dy) {
  const float t = __fmaf_rn(ca, dx, __fmul_rn(cb, dy));
  return __fmaf_rn(dx, t, __fmul_rn(__fmul_rn(cc, dy), dy));
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

struct Pixel {
  int px, py, u, v;
  bool inside;
};

__device__ __forceinline__ Pixel pixel_of(int tile, int tiles_x, int W, int H) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  Pixel p;
  p.px = (w & 1) * 8 + (l & 7);
  p.py = (w >> 1) * 8 + (l >> 3);
  p.u = (tile % tiles_x) * GS_TILE + p.px;
  p.v = (tile / tiles_x) * GS_TILE + p.py;
  p.inside = p.u < W && p.v < H;
  return p;
}

// ------------------------------------------------------------------ forward
struct FwdOut {
  float *image, *depth, *alpha, *final_t;
  int32_t *n_contrib, *stats;
};

__global__ __launch_bounds__(256) void k_render_fwd(RenderArgs a, FwdOut o) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= a.ntiles) return;  // uniform over the workgroup
  const int w = threadIdx.x >> 6;
  const Pixel P = pixel_of(tile, a.tiles_x, a.W, a.H);
  const uint32_t s = a.ranges[2 * tile], e = a.ranges[2 * tile + 1];
  const float ox = (float)((tile % a.tiles_x) * GS_TILE), oy = (float)((tile / a.tiles_x) * GS_TILE);
  const float fpx = (float)P.px, fpy = (float)P.py;

  __shared__ Stage S;

  float T = 1.0f, c0 = 0.f, c1 = 0.f, c2 = 0.f, D = 0.f;
  int last = 0, nev = 0, nsup = 0, ncomp = 0;
  int ntile = (int)(e - s);  // tile-list entries up to and including the stop
  bool done = !P.inside;

  for (uint32_t base = s; base < e; base += kBatch) {
    if (__syncthreads_count(done) == kBatch) break;
    stage_batch(a, base, e, ox, oy, S, nullptr);
    const int cnt = S.cnt[0][w] + S.cnt[1][w] + S.cnt[2][w] + S.cnt[3][w];
    if (__ballot(!done) == 0) continue;
    const int idx0 = (int)(base - s);
    for (int i = 0; i < cnt; ++i) {
      const int k = S.list[w][i];
      const float4 A = S.a[k];
      const float4 B = S.b[k];
      const float dx = __fsub_rn(fpx, A.x), dy = __fsub_rn(fpy, A.y);
      const float ex = exp2_fast(splat_s2(A.z, A.w, B.x, dx, dy));
      const float alpha = fminf(a.alpha_max, __fmul_rn(B.y, ex));
      nev += done ? 0 : 1;
      const bool take = !done && alpha >= a.alpha_min;
      if (__ballot(take) == 0) continue;
      const float4 C = S.c[k];
      const float Tn = __fmul_rn(T, __fsub_rn(1.0f, alpha));
      const bool stop = take && Tn < a.t_min;
      const bool comp = take && !stop;
      const float wgt = comp ? __fmul_rn(alpha, T) : 0.0f;
      c0 = __fmaf_rn(C.x, wgt, c0);
      c1 = __fmaf_rn(C.y, wgt, c1);
      c2 = __fmaf_rn(C.z, wgt, c2);
      D = __fmaf_rn(B.z, wgt, D);
      T = comp ? Tn : T;
      last = comp ? idx0 + k + 1 : last;
      nsup += take ? 1 : 0;
      ncomp += comp ? 1 : 0;
      ntile = stop ? idx0 + k + 1 : ntile;
      done = done || stop;
      if (__ballot(!done) == 0) break;
    }
  }
  if (!P.inside) return;
  const int64_t pix = (int64_t)P.v * a.W + P.u, np = (int64_t)a.W * a.H;
  o.image[pix] = __fmaf_rn(T, a.bg0, c0);
  o.image[np + pix] = __fmaf_rn(T, a.bg1, c1);
  o.image[2 * np + pix] = __fmaf_rn(T, a.bg2, c2);
  o.depth[pix] = D;
  o.alpha[pix] = 1.0f - T;
  o.final_t[pix] = T;
  o.n_contrib[pix] = last;
  if (o.stats) {
    o.stats[pix] = ntile;
    o.stats[np + pix] = nev;
    o.stats[2 * np + pix] = nsup;
    o.stats[3 * np + pix] = ncomp;
  }
}

// ------------------------------------------------------------------ adjoint
struct BwdIn {
  const float *image, *depth, *final_t;
  const int32_t *n_contrib;
  const float *g_image, *g_depth, *g_alpha;
  float *g2d;  // [n][12] accumulated per-Gaussian 2D gradients
};

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

// Per (wave, list entry) the ten partial gradients are summed over the 64
// lanes with DPP, lane 63 adds them to the batch's LDS accumulator, and
// after the batch one lane per entry issues the global float atomics.
__global__ __launch_bounds__(256) void k_render_bwd(RenderArgs a, BwdIn bi) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= a.ntiles) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const Pixel P = pixel_of(tile, a.tiles_x, a.W, a.H);
  const uint32_t s = a.ranges[2 * tile], e = a.ranges[2 * tile + 1];
  const float ox = (float)((tile % a.tiles_x) * GS_TILE), oy = (float)((tile / a.tiles_x) * GS_TILE);
  const float fpx = (float)P.px, fpy = (float)P.py;

  __shared__ Stage S;
  __shared__ uint32_t sGid[kBatch];
  __shared__ float sAcc[10][kBatch];
  __shared__ int sMax;

  const int64_t pix = (int64_t)P.v * a.W + P.u, np = (int64_t)a.W * a.H;
  int ncon = 0;
  float G0 = 0.f, G1 = 0.f, G2 = 0.f, GD = 0.f, GA = 0.f, I0 = 0.f, I1 = 0.f, I2 = 0.f, ID = 0.f, Tf = 1.f;
  if (P.inside) {
    ncon = bi.n_contrib[pix];
    G0 = bi.g_image[pix];
    G1 = bi.g_image[np + pix];
    G2 = bi.g_image[2 * np + pix];
    GD = bi.g_depth ? bi.g_depth[pix] : 0.f;
    GA = bi.g_alpha ? bi.g_alpha[pix] : 0.f;
    I0 = bi.image[pix];
    I1 = bi.image[np + pix];
    I2 = bi.image[2 * np + pix];
    ID = bi.depth[pix];
    Tf = bi.final_t[pix];
  }
  if (t == 0) sMax = 0;
  __syncthreads();
  const int wmax = wave_max(ncon);
  if (lane == 0 && wmax > 0) atomicMax(&sMax, wmax);
  __syncthreads();
  const uint32_t stop = min(s + (uint32_t)sMax, e);

  float T = 1.0f, P0 = 0.f, P1 = 0.f, P2 = 0.f, PD = 0.f;
  const float GAT = GA * Tf;

  for (uint32_t base = s; base < stop; base += kBatch) {
    __syncthreads();  // the previous batch's flush is done with sAcc / sGid
#pragma unroll
    for (int q = 0; q < 10; ++q) sAcc[q][t] = 0.f;
    stage_batch(a, base, stop, ox, oy, S, sGid);
    const int cnt = S.cnt[0][w] + S.cnt[1][w] + S.cnt[2][w] + S.cnt[3][w];
    const int idx0 = (int)(base - s);
    for (int i = 0; i < cnt; ++i) {
      const int k = S.list[w][i];
      if (idx0 + k >= wmax) break;  // lists ascend: no pixel of this wave reaches further
      const float4 A = S.a[k];
      const float4 B = S.b[k];
      const float dx = __fsub_rn(fpx, A.x), dy = __fsub_rn(fpy, A.y);
      const float ex = exp2_fast(splat_s2(A.z, A.w, B.x, dx, dy));
      const float raw = __fmul_rn(B.y, ex);
      const float alpha = fminf(a.alpha_max, raw);
      const bool take = idx0 + k < ncon && alpha >= a.alpha_min;
      if (__ballot(take) == 0) continue;
      const float4 C = S.c[k];
      const float z = B.z;
      const float wgt = take ? __fmul_rn(alpha, T) : 0.0f;
      P0 = __fmaf_rn(C.x, wgt, P0);
      P1 = __fmaf_rn(C.y, wgt, P1);
      P2 = __fmaf_rn(C.z, wgt, P2);
      PD = __fmaf_rn(z, wgt, PD);
      // suffix sums: everything composited after this entry plus T_final bg
      const float S0 = I0 - P0, S1 = I1 - P1, S2 = I2 - P2, SD = ID - PD;
      const float inv = 1.0f / (1.0f - alpha);
      const float dalpha = G0 * (C.x * T - S0 * inv) + G1 * (C.y * T - S1 * inv) + G2 * (C.z * T - S2 * inv) +
                           GD * (z * T - SD * inv) + GAT * inv;
      const bool live = take && raw < a.alpha_max;  // the clamp passes no gradient
      const float gs = live ? dalpha * raw : 0.0f;    // d alpha / d s (natural log domain)
      float g[10];
      // d s / d mean = (A dx + B dy, B dx + C dy), A = -2 ca ln2, B = -cb ln2, C = -2 cc ln2
      const float gl = -gs * kLn2;
      g[0] = gl * (2.0f * A.z * dx + A.w * dy);
      g[1] = gl * (A.w * dx + 2.0f * B.x * dy);
      g[2] = -0.5f * gs * dx * dx;
      g[3] = -gs * dx * dy;
      g[4] = -0.5f * gs * dy * dy;
      g[5] = live ? dalpha * ex : 0.0f;  // d alpha / d o
      g[6] = G0 * wgt;
      g[7] = G1 * wgt;
      g[8] = G2 * wgt;
      g[9] = GD * wgt;
      T = take ? __fmul_rn(T, __fsub_rn(1.0f, alpha)) : T;
#pragma unroll
      for (int q = 0; q < 10; ++q) g[q] = wave_sum_to_lane63(g[q]);
      if (lane == 63) {
#pragma unroll
        for (int q = 0; q < 10; ++q)
          if (g[q] != 0.f) atomicAdd(&sAcc[q][k], g[q]);
      }
    }
    __syncthreads();
    if (base + t < stop) {
      float *dst = bi.g2d + (size_t)sGid[t] * 12;
#pragma unroll
      for (int q = 0; q < 10; ++q) {
        const float r = sAcc[q][t];
        if (r != 0.f) unsafeAtomicAdd(dst + q, r);
      }
    }
  }
}

}  // namespace

gs_status validate_camera(const gs_camera *cam, const char *fn);
gs_status validate_gaussians(const gs_gaussians *g, const char *fn);
size_t project_bwd_workspace(int64_t n);
gs_status project_bwd(const gs_camera *cam, const gs_raster_params *rp, const gs_gaussians *g,
                      const gs_projected *proj, const float *g2d, gs_gaussians *grads, double *d_pose,
                      double *d_twist, void *ws, hipStream_t s);
gs_status zero_f32(float *p, int64_t count, hipStream_t s);

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
  FwdOut o{image, depth, alpha, final_t, n_contrib, stats};
  GS_LAUNCH("render_fwd", k_render_fwd, padded_grid(a.ntiles), 256, 0, (hipStream_t)stream, a, o);
  return GS_OK;
}

gs_status gs_render_bwd_workspace(int64_t n, size_t *bytes) {
  GS_REQUIRE(bytes && n >= 0, "gs_render_bwd_workspace: bad argument");
  *bytes = align_up(sizeof(float) * 12 * (size_t)n) + project_bwd_workspace(n);
  return GS_OK;
}

gs_status gs_render_bwd(const gs_camera *cam, const gs_raster_params *rp, const gs_gaussians *g,
                        const gs_projected *proj, const uint32_t *values, const uint32_t *ranges, const float *image,
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
  size_t need = 0;
  gs_render_bwd_workspace(g->n, &need);
  if (ws_bytes < need || (need && !ws)) {
    set_error("gs_render_bwd: workspace %zu bytes < %zu", ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  Carve cv(ws);
  float *g2d = cv.take<float>(12 * (size_t)g->n);
  void *pose_ws = cv.take<char>(project_bwd_workspace(g->n));
  if ((st = zero_f32(g2d, 12 * g->n, s)) != GS_OK) return st;
  RenderArgs a = render_args(cam, rp, proj, values, ranges);
  BwdIn bi{image, depth, final_t, n_contrib, dL_dimage, dL_ddepth, dL_dalpha, g2d};
  GS_LAUNCH("render_bwd", k_render_bwd, padded_grid(a.ntiles), 256, 0, s, a, bi);
  return project_bwd(cam, rp, g, proj, g2d, grads, dL_dpose, dL_dtwist, pose_ws, s);
}

}  // extern "C"
