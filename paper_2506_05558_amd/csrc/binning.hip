// Tile binning: the per-tile lists of (Gaussian, tile) pairs in
// (tile, depth, index) order.
//
// Instead of sorting M 64-bit (tile | depth) keys, the visible Gaussians are
// first sorted by depth (32-bit keys, N of them), pairs are emitted in that
// order, and the M pairs are then sorted by tile id alone (ceil(log2 T)
// bits).  Both sorts are stable LSD radix sorts, so the result is exactly the
// order of a stable sort of (tile << 32 | depth bits) over pairs emitted in
// Gaussian-index order, at about a third of the key traffic.
//
// Radix pass layout: every wave owns a contiguous chunk of kChunk keys.  The
// histogram kernel counts each chunk's digits; an exclusive scan over the
// digit-major table [digit][chunk] gives every (digit, chunk) its output
// base; the scatter kernel walks its chunk 64 keys at a time in order, finds
// the lanes holding the same digit with one ballot per digit bit, and places
// each key at base + running count + rank among its peers.  All of this is
// wave-private, so the scatter needs no workgroup barriers and is stable.
#include "common.h"

namespace gsmi {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;  // 4096
constexpr int kChunk = 1024;                        // keys per wave in a radix pass
constexpr int kRadixBlock = 256;                    // 4 waves
constexpr int kWaves = kRadixBlock / 64;

// ------------------------------------------------------------------- scan
template <class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const int lane = __lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over the workgroup; returns the
// workgroup total through *total.
template <class T>
__device__ __forceinline__ T block_excl_scan(T x, T *total) {
  __shared__ T wsum[kScanBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const T inc = wave_incl_scan<T>(x);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kScanBlock / 64; ++i) {
    if (i < w) before += wsum[i];
    all += wsum[i];
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const T *in, int64_t count, T *partials) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < count) sum += in[base + k];
  T total;
  block_excl_scan<T>(sum, &total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the partials in place, total -> *total.
template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_spine(T *partials, int64_t nparts, T *total) {
  T carry = 0;
  for (int64_t base = 0; base < nparts; base += kScanTile) {
    const int64_t i0 = base + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = (i0 + k < nparts) ? partials[i0 + k] : (T)0;
      sum += v[k];
    }
    T tot;
    T run = carry + block_excl_scan<T>(sum, &tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (i0 + k < nparts) partials[i0 + k] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const T *in, T *out, int64_t count, const T *partials) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems], sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < count) ? in[base + k] : (T)0;
    sum += v[k];
  }
  T tot;
  T run = partials[blockIdx.x] + block_excl_scan<T>(sum, &tot);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < count) out[base + k] = run;
    run += v[k];
  }
}

template <class T>
__global__ void k_fill(T *p, int64_t count, T value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

// ------------------------------------------------------------- radix sort
__device__ __forceinline__ uint64_t peers_of(uint32_t digit, int bits, bool valid) {
  uint64_t peers = __ballot(valid);
  for (int b = 0; b < bits; ++b) {
    const bool bit = (digit >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

__global__ __launch_bounds__(kRadixBlock) void k_radix_hist(const uint32_t *keys, const uint32_t *count_dev,
                                                            uint32_t count_max, int shift, int bits,
                                                            int64_t nchunks, uint32_t *hist) {
  __shared__ uint32_t cnt[kWaves][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t chunk = (int64_t)blockIdx.x * kWaves + w;
  const int ndig = 1 << bits;
  for (int d = lane; d < 256; d += 64) cnt[w][d] = 0;
  if (chunk >= nchunks) return;  // wave-uniform; no workgroup barriers below
  const uint32_t count = count_dev ? min(*count_dev, count_max) : count_max;
  const int64_t c0 = chunk * kChunk;
  const uint32_t mask = (uint32_t)ndig - 1u;
  const uint64_t lt = lanemask_lt();
  for (int it = 0; it < kChunk / 64; ++it) {
    const int64_t i = c0 + it * 64 + lane;
    const bool valid = i < (int64_t)count;
    if (__ballot(valid) == 0) break;
    const uint32_t d = valid ? (keys[i] >> shift) & mask : 0u;
    const uint64_t peers = peers_of(d, bits, valid);
    const uint64_t higher = peers & ~(lt | (1ull << lane));
    if (valid && higher == 0) cnt[w][d] += (uint32_t)__popcll(peers);  // highest lane of the group
  }
  for (int d = lane; d < ndig; d += 64) hist[(int64_t)d * nchunks + chunk] = cnt[w][d];
}

template <bool TWO>
__global__ __launch_bounds__(kRadixBlock) void k_radix_scatter(const uint32_t *kin, const uint32_t *vin,
                                                               const uint32_t *win, uint32_t *kout, uint32_t *vout,
                                                               uint32_t *wout, const uint32_t *count_dev,
                                                               uint32_t count_max, int shift, int bits,
                                                               int64_t nchunks, const uint32_t *offsets) {
  __shared__ uint32_t run[kWaves][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t chunk = (int64_t)blockIdx.x * kWaves + w;
  if (chunk >= nchunks) return;
  const int ndig = 1 << bits;
  for (int d = lane; d < ndig; d += 64) run[w][d] = offsets[(int64_t)d * nchunks + chunk];
  const uint32_t count = count_dev ? min(*count_dev, count_max) : count_max;
  const int64_t c0 = chunk * kChunk;
  const uint32_t mask = (uint32_t)ndig - 1u;
  const uint64_t lt = lanemask_lt();
  for (int it = 0; it < kChunk / 64; ++it) {
    const int64_t i = c0 + it * 64 + lane;
    const bool valid = i < (int64_t)count;
    if (__ballot(valid) == 0) break;
    uint32_t key = 0, val = 0, val2 = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
      if (TWO) val2 = win[i];
    }
    const uint32_t d = (key >> shift) & mask;
    const uint64_t peers = peers_of(d, bits, valid);
    if (valid) {
      const uint32_t base = run[w][d];
      const uint32_t pos = base + (uint32_t)__popcll(peers & lt);
      kout[pos] = key;
      vout[pos] = val;
      if (TWO) wout[pos] = val2;
      const uint64_t higher = peers & ~(lt | (1ull << lane));
      if (higher == 0) run[w][d] = base + (uint32_t)__popcll(peers);
    }
  }
}

// ------------------------------------------------------------ binning steps
__global__ void k_visible_flags(const int32_t *tiles, int64_t n, uint32_t *flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = tiles[i] > 0 ? 1u : 0u;
}

__global__ void k_compact(const uint32_t *flags, const uint32_t *pos, const float *rec, int64_t n, uint32_t *keys,
                          uint32_t *vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flags[i]) return;
  const uint32_t p = pos[i];
  keys[p] = __float_as_uint(rec[i * GS_REC_FLOATS + 11]);  // depth > 0: bits order like values
  vals[p] = (uint32_t)i;
}

__global__ void k_gather_counts(const uint32_t *order, const uint32_t *count_dev, const int32_t *tiles, int64_t n,
                                uint32_t *cnt) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  cnt[j] = j < (int64_t)*count_dev ? (uint32_t)tiles[order[j]] : 0u;
}

// Emits the pairs of the j-th Gaussian in depth order at its offset: tile
// id, Gaussian index and the pair's emission index ("slot"); the pairs of a
// Gaussian occupy slots [first_slot[g], first_slot[g] + tiles_touched[g]).
__global__ void k_duplicate(const uint32_t *order, const uint32_t *count_dev, const uint32_t *offs, const float *rec,
                            const int32_t *radius, int64_t n, int W, int H, int tiles_x, uint32_t capacity,
                            uint32_t *tile_keys, uint32_t *vals, uint32_t *slots, uint32_t *first_slot) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= (int64_t)*count_dev) return;
  const uint32_t g = order[j];
  first_slot[g] = offs[j];
  const float4 r0 = *(const float4 *)(rec + (size_t)g * GS_REC_FLOATS);
  int tx0, ty0, tx1, ty1;
  if (!tile_rect(__fadd_rn(r0.x, r0.z), __fadd_rn(r0.y, r0.w), radius[g], radius[n + g], W, H, tx0, ty0, tx1,
                 ty1))
    return;
  uint32_t o = offs[j];
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx) {
      if (o >= capacity) return;
      tile_keys[o] = (uint32_t)(ty * tiles_x + tx);
      vals[o] = g;
      slots[o] = o;
      ++o;
    }
}


__global__ void k_ranges(const uint32_t *tile_keys, uint32_t M, uint32_t *ranges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const uint32_t t = tile_keys[i];
  if (i == 0 || tile_keys[i - 1] != t) ranges[2 * t] = (uint32_t)i;
  if (i == (int64_t)M - 1 || tile_keys[i + 1] != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
}

inline int64_t nchunks_of(int64_t count) { return (count + kChunk - 1) / kChunk; }
inline int64_t grid1(int64_t count, int block = 256) { return (count + block - 1) / block; }

// Passes of at most 8 bits covering [0, total_bits), as equal as possible.
int plan_passes(int total_bits, int shifts[8], int widths[8]) {
  if (total_bits <= 0) return 0;
  const int np = (total_bits + 7) / 8;
  int at = 0;
  for (int p = 0; p < np; ++p) {
    const int wdt = (total_bits - at + (np - p) - 1) / (np - p);
    shifts[p] = at;
    widths[p] = wdt;
    at += wdt;
  }
  return np;
}

struct RadixWs {
  uint32_t *hist;  // [256][nchunks(count_max)]
  void *scan_ws;
};

size_t radix_hist_elems(int64_t count_max) { return 256 * (size_t)nchunks_of(count_max); }

// Sorts (k[0], v[0]) by the given passes, ping-ponging with (k[1], v[1]).
// Returns the index (0 or 1) of the buffer pair holding the result.
gs_status radix_sort(uint32_t *k[2], uint32_t *v[2], uint32_t *v2[2], const uint32_t *count_dev, int64_t count_max,
                     int npasses, const int *shifts, const int *widths, const RadixWs &rw, hipStream_t s,
                     int *result) {
  int cur = 0;
  const int64_t nch = nchunks_of(count_max);
  const int64_t blocks = (nch + kWaves - 1) / kWaves;
  for (int p = 0; p < npasses; ++p) {
    if (count_max == 0) break;
    GS_LAUNCH("radix_hist", k_radix_hist, blocks, kRadixBlock, 0, s, k[cur], count_dev, (uint32_t)count_max,
              shifts[p], widths[p], nch, rw.hist);
    gs_status st = scan_exclusive(rw.hist, rw.hist, (int64_t)(1 << widths[p]) * nch, nullptr, rw.scan_ws, s);
    if (st != GS_OK) return st;
    if (v2)
      GS_LAUNCH("radix_scatter", k_radix_scatter<true>, blocks, kRadixBlock, 0, s, k[cur], v[cur], v2[cur],
                k[1 - cur], v[1 - cur], v2[1 - cur], count_dev, (uint32_t)count_max, shifts[p], widths[p], nch,
                rw.hist);
    else
      GS_LAUNCH("radix_scatter", k_radix_scatter<false>, blocks, kRadixBlock, 0, s, k[cur], v[cur], nullptr,
                k[1 - cur], v[1 - cur], nullptr, count_dev, (uint32_t)count_max, shifts[p], widths[p], nch,
                rw.hist);
    cur = 1 - cur;
  }
  *result = cur;
  return GS_OK;
}

}  // namespace

size_t scan_workspace(int64_t count) {
  const int64_t nparts = (count + kScanTile - 1) / kScanTile;
  return align_up(sizeof(uint64_t) * (size_t)(nparts + 1));
}

template <class T>
static gs_status scan_exclusive_t(const T *in, T *out, int64_t count, T *total, void *ws, hipStream_t s) {
  if (count <= 0) {
    if (total) GS_LAUNCH("fill", k_fill<T>, 1, 64, 0, s, total, 1, (T)0);
    return GS_OK;
  }
  const int64_t nparts = (count + kScanTile - 1) / kScanTile;
  T *partials = (T *)ws;
  GS_LAUNCH("scan", k_scan_reduce<T>, nparts, kScanBlock, 0, s, in, count, partials);
  GS_LAUNCH("scan", k_scan_spine<T>, 1, kScanBlock, 0, s, partials, nparts, total);
  GS_LAUNCH("scan", k_scan_apply<T>, nparts, kScanBlock, 0, s, in, out, count, (const T *)partials);
  return GS_OK;
}

// Exclusive scan; in may equal out.  total (device, may be NULL) receives the sum.
gs_status scan_exclusive(const uint32_t *in, uint32_t *out, int64_t count, uint32_t *total, void *ws,
                         hipStream_t s) {
  return scan_exclusive_t<uint32_t>(in, out, count, total, ws, s);
}
gs_status scan_exclusive_u64(const uint64_t *in, uint64_t *out, int64_t count, uint64_t *total, void *ws,
                             hipStream_t s) {
  return scan_exclusive_t<uint64_t>(in, out, count, total, ws, s);
}

}  // namespace gsmi

using namespace gsmi;

namespace {

struct BinLayout {
  uint32_t *flags, *pos, *kA, *vA, *kB, *vB, *cnt, *offs, *hist, *scalars, *ktmp, *vtmp, *stmp;
  void *scan_ws;
  size_t bytes;
};

BinLayout bin_layout(void *ws, int64_t n, int64_t capacity) {
  Carve cv(ws);
  BinLayout L;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  const size_t cc = (size_t)(capacity > 0 ? capacity : 1);
  L.flags = cv.take<uint32_t>(nn);
  L.pos = cv.take<uint32_t>(nn);
  L.kA = cv.take<uint32_t>(nn);
  L.vA = cv.take<uint32_t>(nn);
  L.kB = cv.take<uint32_t>(nn);
  L.vB = cv.take<uint32_t>(nn);
  L.cnt = cv.take<uint32_t>(nn);
  L.offs = cv.take<uint32_t>(nn);
  const int64_t big = n > capacity ? n : capacity;
  L.hist = cv.take<uint32_t>(radix_hist_elems(big));
  L.scan_ws = cv.take<char>(scan_workspace((int64_t)radix_hist_elems(big) > big ? (int64_t)radix_hist_elems(big) : big));
  L.scalars = cv.take<uint32_t>(4);
  L.ktmp = cv.take<uint32_t>(cc);
  L.vtmp = cv.take<uint32_t>(cc);
  L.stmp = cv.take<uint32_t>(cc);
  L.bytes = cv.off;
  return L;
}

}  // namespace

namespace gsmi {
gs_status validate_camera(const gs_camera *cam, const char *fn);
}

extern "C" {

gs_status gs_bin_sort_workspace(int64_t n, int64_t capacity, size_t *bytes) {
  GS_REQUIRE(bytes && n >= 0 && capacity >= 0, "gs_bin_sort_workspace: bad argument");
  GS_REQUIRE(n < (int64_t(1) << 31) && capacity < (int64_t(1) << 32) - 1, "gs_bin_sort_workspace: size too large");
  *bytes = bin_layout(nullptr, n, capacity).bytes;
  return GS_OK;
}

gs_status gs_bin_sort(const gs_camera *cam, const gs_projected *proj, int64_t n, int64_t capacity, void *ws,
                      size_t ws_bytes, uint32_t *tile_ids, uint32_t *values, uint32_t *slots, uint32_t *ranges,
                      uint32_t *first_slot, int64_t *n_instances, void *stream) {
  gs_status st = validate_camera(cam, "gs_bin_sort");
  if (st != GS_OK) return st;
  GS_REQUIRE(proj && ranges && n_instances, "gs_bin_sort: NULL argument");
  GS_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "gs_bin_sort: n out of range");
  GS_REQUIRE(capacity >= 0 && capacity < (int64_t(1) << 32) - 1, "gs_bin_sort: capacity out of range");
  if (n > 0) GS_REQUIRE(proj->rec && proj->radius && proj->tiles_touched, "gs_bin_sort: NULL projection plane");
  if (capacity > 0) GS_REQUIRE(tile_ids && values && slots, "gs_bin_sort: NULL list output");
  if (n > 0) GS_REQUIRE(first_slot, "gs_bin_sort: NULL first_slot");
  size_t need = 0;
  gs_bin_sort_workspace(n, capacity, &need);
  if (ws_bytes < need || !ws) {
    set_error("gs_bin_sort: workspace %zu bytes < %zu", ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  const int W = cam->width, H = cam->height;
  const int tx = tiles_x_of(W), T = tx * tiles_y_of(H);
  BinLayout L = bin_layout(ws, n, capacity);
  RadixWs rw{L.hist, L.scan_ws};
  uint32_t *V = L.scalars, *Mdev = L.scalars + 1;

  uint32_t M = 0;
  int order_buf = 0;
  if (n > 0) {
    // 1. compact the visible Gaussians with their depth keys
    GS_LAUNCH("bin_flags", k_visible_flags, grid1(n), 256, 0, s, proj->tiles_touched, n, L.flags);
    if ((st = scan_exclusive(L.flags, L.pos, n, V, L.scan_ws, s)) != GS_OK) return st;
    GS_LAUNCH("bin_compact", k_compact, grid1(n), 256, 0, s, L.flags, L.pos, proj->rec, n, L.kA, L.vA);
    // 2. stable sort by depth (31 significant bits of a positive float)
    int shifts[8], widths[8];
    const int np = plan_passes(31, shifts, widths);
    uint32_t *kk[2] = {L.kA, L.kB}, *vv[2] = {L.vA, L.vB};
    if ((st = radix_sort(kk, vv, nullptr, V, n, np, shifts, widths, rw, s, &order_buf)) != GS_OK) return st;
    const uint32_t *order = vv[order_buf];
    // 3. pair offsets in depth order
    GS_LAUNCH("bin_counts", k_gather_counts, grid1(n), 256, 0, s, order, V, proj->tiles_touched, n, L.cnt);
    if ((st = scan_exclusive(L.cnt, L.offs, n, Mdev, L.scan_ws, s)) != GS_OK) return st;
    GS_CHECK_HIP(hipMemcpyAsync(&M, Mdev, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read M");
    GS_CHECK_HIP(hipStreamSynchronize(s), "sync M");
  }
  *n_instances = M;
  if ((int64_t)M > capacity) {
    set_error("gs_bin_sort: %u pairs exceed capacity %lld", M, (long long)capacity);
    return GS_ERR_CAPACITY;
  }
  GS_LAUNCH("bin_fill", k_fill<uint32_t>, grid1(2 * (int64_t)T), 256, 0, s, ranges, 2 * (int64_t)T, 0u);
  if (M == 0) return GS_OK;

  // 4. emit pairs in depth order, 5. stable sort by tile, 6. ranges
  int tb = 0;
  while ((1 << tb) < T) ++tb;
  int shifts[8], widths[8];
  const int np = plan_passes(tb, shifts, widths);
  // start in the buffer pair that makes the final pass land in the caller's arrays
  uint32_t *kk[2], *vv[2], *ss[2];
  if (np % 2 == 0) {
    kk[0] = tile_ids; vv[0] = values; ss[0] = slots; kk[1] = L.ktmp; vv[1] = L.vtmp; ss[1] = L.stmp;
  } else {
    kk[0] = L.ktmp; vv[0] = L.vtmp; ss[0] = L.stmp; kk[1] = tile_ids; vv[1] = values; ss[1] = slots;
  }
  const uint32_t *order = order_buf ? L.vB : L.vA;
  GS_LAUNCH("bin_duplicate", k_duplicate, grid1(n), 256, 0, s, order, V, L.offs, proj->rec, proj->radius, n, W, H, tx,
            (uint32_t)capacity, kk[0], vv[0], ss[0], first_slot);
  int res = 0;
  if ((st = radix_sort(kk, vv, ss, nullptr, M, np, shifts, widths, rw, s, &res)) != GS_OK) return st;
  GS_LAUNCH("bin_ranges", k_ranges, grid1(M), 256, 0, s, tile_ids, M, ranges);
  return GS_OK;
}

}  // extern "C"
