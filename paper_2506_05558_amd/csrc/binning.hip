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
// Radix pass layout: every workgroup (8 waves) owns 2048 consecutive keys,
// each wave a contiguous run of 256.  The histogram kernel counts each
// block's digits into the digit-major table [digit][block]; one workgroup
// per digit scans its row in place and records the row total.  The scatter
// kernel ranks each wave's keys in order (the lanes holding the same digit
// are found with one ballot per digit bit), combines the waves' digit counts
// into block-local positions, adds the row-total prefix to the row scan to
// get each digit's output base, reorders the block in LDS and writes each
// digit's keys as one contiguous run -- stable, and with coalesced stores.
#include <algorithm>

#include "common.h"

namespace gsmi {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;  // 4096
// 8 waves of 256 keys: short per-wave ranking chains, and small enough LDS
// (24-32 KB) that the sorts of one view run beside another view's renders
constexpr int kRadixBlock = 512;                    // 8 waves
constexpr int kWaves = kRadixBlock / 64;
constexpr int kWaveKeys = 256;                      // keys per wave in a radix pass
constexpr int kBlockKeys = kWaves * kWaveKeys;      // keys per workgroup (2048)

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

// The elements a scan reads: in[i] (ArrayLoad), or the binning's 64-bit
// visibility record formed from a Gaussian's tile count (TilesLoad).
template <class T>
struct ArrayLoad {
  const T *in;
  __device__ __forceinline__ T operator()(int64_t i) const { return in[i]; }
};

// One 64-bit value per Gaussian whose exclusive prefix sum gives both its
// position among the visible Gaussians (low word: visibility flag) and its
// first slot (high word: tiles touched).  Neither total can carry into the
// high word: n < 2^31 and the pair count < 2^32.
__device__ __forceinline__ uint64_t visibility_record(int32_t t) {
  return t > 0 ? (1ull | (uint64_t)(uint32_t)t << 32) : 0ull;
}
struct TilesLoad {
  const int32_t *tiles;
  __device__ __forceinline__ uint64_t operator()(int64_t i) const { return visibility_record(tiles[i]); }
};

// A workgroup's tile of kScanTile elements is read and written with
// coalesced accesses (element k * kScanBlock + thread), and handed between
// that order and the thread-contiguous order of the serial scan through LDS
// padded by one element per 16, so that both orders are free of bank
// conflicts.
__device__ __forceinline__ int scan_pad(int e) { return e + (e >> 4); }
constexpr int kScanLds = kScanTile + kScanTile / 16;

template <class T, class L>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(L load, int64_t count, T *partials) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  T sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanBlock;
    if (i < count) sum += load(i);
  }
  T total;
  block_excl_scan<T>(sum, &total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// Applies the scan to one tile.  The tile's offset is the sum of the tile
// totals before it, which every workgroup adds up itself from the (few,
// cached) partials -- no separate spine launch.  The last workgroup also
// writes the grand total.
template <class T, class L>
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(L load, T *out, int64_t count, const T *partials,
                                                           T *total) {
  __shared__ T s_off;
  __shared__ T tile[kScanLds];
  {
    T part = 0;
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kScanBlock) part += partials[b];
    T all;
    block_excl_scan<T>(part, &all);
    if (threadIdx.x == 0) {
      s_off = all;
      if (total && blockIdx.x == gridDim.x - 1) *total = all + partials[blockIdx.x];
    }
  }
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int e = k * kScanBlock + threadIdx.x;
    tile[scan_pad(e)] = base + e < count ? load(base + e) : (T)0;
  }
  __syncthreads();
  T v[kScanItems], sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = tile[scan_pad(threadIdx.x * kScanItems + k)];
    sum += v[k];
  }
  T tot;
  T run = s_off + block_excl_scan<T>(sum, &tot);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    tile[scan_pad(threadIdx.x * kScanItems + k)] = run;
    run += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int e = k * kScanBlock + threadIdx.x;
    if (base + e < count) out[base + e] = tile[scan_pad(e)];
  }
}

// Single-workgroup exclusive scan for arrays of up to one workgroup tile
// (8192 elements): one launch instead of three.  Longer arrays take the
// three-kernel path: one workgroup streaming 100k+ elements is slower than
// two extra launches.
constexpr int kSmallBlock = 1024;
constexpr int kSmallItems = 8;
constexpr int64_t kSmallScan = kSmallBlock * kSmallItems;

template <class T>
__device__ __forceinline__ T big_block_excl_scan(T x, T *total) {
  __shared__ T wsum[kSmallBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const T inc = wave_incl_scan<T>(x);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    const T v = lane < kSmallBlock / 64 ? wsum[lane] : (T)0;
    const T vi = wave_incl_scan<T>(v);
    if (lane < kSmallBlock / 64) wsum[lane] = vi - v;  // exclusive wave offsets
    if (lane == kSmallBlock / 64 - 1) wsum[kSmallBlock / 64 - 1] = vi - v, *total = vi;
  }
  __syncthreads();
  const T before = wsum[w];
  __syncthreads();
  return before + inc - x;
}

template <class T, class L>
__global__ __launch_bounds__(kSmallBlock) void k_scan_small(L load, T *out, int64_t count, T *total) {
  __shared__ T tot;
  T carry = 0;
  for (int64_t base = 0; base < count; base += (int64_t)kSmallBlock * kSmallItems) {
    const int64_t i0 = base + (int64_t)threadIdx.x * kSmallItems;
    T v[kSmallItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kSmallItems; ++k) {
      v[k] = (i0 + k < count) ? load(i0 + k) : (T)0;
      sum += v[k];
    }
    T run = carry + big_block_excl_scan<T>(sum, &tot);
#pragma unroll
    for (int k = 0; k < kSmallItems; ++k) {
      if (i0 + k < count) out[i0 + k] = run;
      run += v[k];
    }
    carry += tot;  // tot is read after the scan's last barrier and rewritten only after the next one
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <class T>
__global__ void k_fill(T *p, int64_t count, T value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

// ------------------------------------------------------------- radix sort
__device__ __forceinline__ uint64_t peers_of(uint32_t digit, int bits, bool valid) {
  uint64_t peers = ballot(valid);
  for (int b = 0; b < bits; ++b) {
    const bool bit = (digit >> b) & 1u;
    const uint64_t m = ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Pass layout: each workgroup owns kBlockKeys consecutive keys, each of its
// waves a contiguous run of kWaveKeys.  The count kernel gives the digit
// histogram of every block, hist[digit][block].
__global__ __launch_bounds__(kRadixBlock) void k_radix_hist(const uint32_t *keys, const uint32_t *count_dev,
                                                            uint32_t count_max, int shift, int bits,
                                                            int64_t nblocks, uint32_t *hist) {
  __shared__ uint32_t cnt[kWaves][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ndig = 1 << bits;
  for (int d = lane; d < 256; d += 64) cnt[w][d] = 0;  // each wave owns its row
  const uint32_t count = count_dev ? min(*count_dev, count_max) : count_max;
  const int64_t c0 = (int64_t)blockIdx.x * kBlockKeys + (int64_t)w * kWaveKeys;
  const uint32_t mask = (uint32_t)ndig - 1u;
  const uint64_t lt = lanemask_lt();
  for (int it = 0; it < kWaveKeys / 64; ++it) {
    const int64_t i = c0 + it * 64 + lane;
    const bool valid = i < (int64_t)count;
    if (ballot(valid) == 0) break;  // wave-uniform
    const uint32_t d = valid ? (keys[i] >> shift) & mask : 0u;
    const uint64_t peers = peers_of(d, bits, valid);
    const uint64_t higher = peers & ~(lt | (1ull << lane));
    if (valid && higher == 0) cnt[w][d] += (uint32_t)__popcll(peers);  // highest lane of the group
  }
  __syncthreads();
  for (int d = threadIdx.x; d < ndig; d += kRadixBlock) {
    uint32_t sum = 0;
#pragma unroll
    for (int v = 0; v < kWaves; ++v) sum += cnt[v][d];
    hist[(int64_t)d * nblocks + blockIdx.x] = sum;
  }
}

// Exclusive scan of one digit's row hist[d][0 .. nblocks) in place (one
// workgroup per digit); the row total goes to rowtot[d].
constexpr int kRowItems = 4;
__global__ __launch_bounds__(kScanBlock) void k_radix_rowscan(uint32_t *hist, int64_t nblocks, uint32_t *rowtot) {
  uint32_t *row = hist + (int64_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  for (int64_t base = 0; base < nblocks; base += kScanBlock * kRowItems) {
    const int64_t i0 = base + (int64_t)threadIdx.x * kRowItems;
    uint32_t v[kRowItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) {
      v[k] = i0 + k < nblocks ? row[i0 + k] : 0u;
      sum += v[k];
    }
    uint32_t tot;
    uint32_t run = carry + block_excl_scan<uint32_t>(sum, &tot);
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) {
      if (i0 + k < nblocks) row[i0 + k] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) rowtot[blockIdx.x] = carry;
}

// Stable scatter of one block: each wave ranks its run in key order with
// ballot peer matching (rank = earlier keys of the same digit), the block
// turns per-wave digit counts into local positions (digit-major, then wave,
// then rank), the keys are reordered in LDS, and consecutive lanes then
// write consecutive local positions, so each digit's keys leave as one
// contiguous run.  Digit d of block b starts at the exclusive prefix of the
// row totals (rowtot) plus the row scan (rows[d][b]).
template <bool TWO>
__global__ __launch_bounds__(kRadixBlock) void k_radix_scatter(const uint32_t *kin, const uint32_t *vin,
                                                               const uint32_t *win, uint32_t *kout, uint32_t *vout,
                                                               uint32_t *wout, const uint32_t *count_dev,
                                                               uint32_t count_max, int shift, int bits,
                                                               int64_t nblocks, const uint32_t *rows,
                                                               const uint32_t *rowtot) {
  constexpr int kIt = kWaveKeys / 64;
  __shared__ uint32_t run[kWaves][256];
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t dsum[2][4];
  __shared__ uint32_t sk[kBlockKeys];
  __shared__ uint32_t sv[kBlockKeys];
  __shared__ uint32_t sw[TWO ? kBlockKeys : 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ndig = 1 << bits;
  const uint32_t mask = (uint32_t)ndig - 1u;
  for (int d = lane; d < 256; d += 64) run[w][d] = 0;
  const uint32_t count = count_dev ? min(*count_dev, count_max) : count_max;
  const int64_t b0 = (int64_t)blockIdx.x * kBlockKeys;
  const int64_t c0 = b0 + (int64_t)w * kWaveKeys;
  const uint64_t lt = lanemask_lt();
  uint32_t key[kIt], val[kIt], val2[kIt], rk[kIt];
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int64_t i = c0 + it * 64 + lane;
    const bool valid = i < (int64_t)count;
    key[it] = valid ? kin[i] : 0u;
    val[it] = valid ? vin[i] : 0u;
    val2[it] = (TWO && valid) ? win[i] : 0u;
    const uint32_t d = (key[it] >> shift) & mask;
    const uint64_t peers = peers_of(d, bits, valid);
    rk[it] = 0xffffffffu;
    if (valid) {
      const uint32_t base = run[w][d];
      rk[it] = (base + (uint32_t)__popcll(peers & lt)) | (d << 16);  // rank < 2^16
      const uint64_t higher = peers & ~(lt | (1ull << lane));
      if (higher == 0) run[w][d] = base + (uint32_t)__popcll(peers);
    }
  }
  __syncthreads();
  // the first four waves, one digit per lane: local digit starts (exclusive
  // scan of the block's digit totals), the digit's global start (exclusive
  // scan of the row totals), and the per-wave starts within each digit
  const int d = threadIdx.x;
  uint32_t tot = 0, rt = 0, inc = 0, rinc = 0;
  if (d < 256) {
#pragma unroll
    for (int v = 0; v < kWaves; ++v) tot += run[v][d];
    rt = d < ndig ? rowtot[d] : 0u;
    inc = wave_incl_scan<uint32_t>(tot);
    rinc = wave_incl_scan<uint32_t>(rt);
    if (lane == 63) dsum[0][w] = inc, dsum[1][w] = rinc;
  }
  __syncthreads();
  if (d < 256) {
    uint32_t before = 0, rbefore = 0;
    for (int i = 0; i < w; ++i) before += dsum[0][i], rbefore += dsum[1][i];
    const uint32_t start = before + inc - tot;
    gbase[d] = (d < ndig ? rbefore + rinc - rt + rows[(int64_t)d * nblocks + blockIdx.x] : 0u) - start;
    uint32_t acc = start;
#pragma unroll
    for (int v = 0; v < kWaves; ++v) {
      const uint32_t n = run[v][d];
      run[v][d] = acc;
      acc += n;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    if (rk[it] != 0xffffffffu) {
      const uint32_t lp = run[w][rk[it] >> 16] + (rk[it] & 0xffffu);
      sk[lp] = key[it];
      sv[lp] = val[it];
      if (TWO) sw[lp] = val2[it];
    }
  }
  __syncthreads();
  const int64_t nvalid64 = (int64_t)count - b0;
  const int nvalid = nvalid64 <= 0 ? 0 : (nvalid64 >= kBlockKeys ? kBlockKeys : (int)nvalid64);
  for (int idx = threadIdx.x; idx < nvalid; idx += kRadixBlock) {
    const uint32_t k = sk[idx];
    const uint32_t pos = gbase[(k >> shift) & mask] + (uint32_t)idx;
    kout[pos] = k;
    vout[pos] = sv[idx];
    if (TWO) wout[pos] = sw[idx];
  }
}

// ------------------------------------------------------------ binning steps
constexpr uint32_t kNoSlot = 0xffffffffu;

// Visible Gaussians in index order: depth key, index, a 16-byte record for
// the pair emission -- the tile rect packed as (tx0 | ty0 << 16,
// tx1 | ty1 << 16) and the first slot -- and the first slot itself.  A
// Gaussian whose slots do not all fit (an asynchronous call short of
// capacity) gets no first slot, so its adjoint reads no pair.  With bin
// (the projection's binning inputs) the depth and the rect come from one
// 16-byte read; otherwise from the record's line and the radii.
__global__ void k_compact(const int32_t *tiles, const uint64_t *pos, const float *rec, const int32_t *radius,
                          const uint4 *bin, int64_t n, int W, int H, uint32_t capacity, uint32_t *keys,
                          uint32_t *vals, uint4 *rect, uint32_t *first_slot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || tiles[i] <= 0) return;
  const uint64_t ps = pos[i];
  const uint32_t p = (uint32_t)ps;
  uint32_t key, rx, ry;
  if (bin) {
    const uint4 b = bin[i];
    key = b.x;
    rx = b.y;
    ry = b.z;
  } else {
    const float4 r0 = *(const float4 *)(rec + i * GS_REC_FLOATS);
    key = __float_as_uint(rec[i * GS_REC_FLOATS + 11]);
    int tx0 = 0, ty0 = 0, tx1 = -1, ty1 = -1;
    tile_rect(__fadd_rn(r0.x, r0.z), __fadd_rn(r0.y, r0.w), radius[i], radius[n + i], W, H, tx0, ty0, tx1, ty1);
    rx = (uint32_t)tx0 | (uint32_t)ty0 << 16;
    ry = (uint32_t)tx1 | (uint32_t)ty1 << 16;
  }
  keys[p] = key;  // depth > 0: bits order like values
  vals[p] = (uint32_t)i;
  const uint32_t s0 = (uint32_t)(ps >> 32);
  rect[i] = make_uint4(rx, ry, s0, 0u);
  const uint32_t npairs = ((ry & 0xffffu) - (rx & 0xffffu) + 1u) * ((ry >> 16) - (rx >> 16) + 1u);
  first_slot[i] = (uint64_t)s0 + npairs <= capacity ? s0 : kNoSlot;
}

// The visible Gaussians' emission records in depth order: the index-order
// record with the Gaussian index in its spare word, so the emission reads
// coalesced records; and the pair count of every block of kDupBlock
// consecutive Gaussians, whose exclusive scan gives each block its first
// pair.
constexpr int kDupBlock = 256;
__global__ __launch_bounds__(kDupBlock) void k_depth_records(const uint32_t *order, const uint32_t *count_dev,
                                                             const uint4 *rect, int64_t n, uint4 *drec,
                                                             uint32_t *block_pairs) {
  const int64_t j = (int64_t)blockIdx.x * kDupBlock + threadIdx.x;
  uint32_t np = 0;
  if (j < (int64_t)*count_dev) {
    const uint32_t g = order[j];
    uint4 r = rect[g];
    np = ((r.y & 0xffffu) - (r.x & 0xffffu) + 1u) * ((r.y >> 16) - (r.x >> 16) + 1u);
    r.w = g;
    drec[j] = r;
  }
  uint32_t total;
  block_excl_scan<uint32_t>(np, &total);
  if (threadIdx.x == 0) block_pairs[blockIdx.x] = total;
}

// Emits the pairs of the visible Gaussians in depth order: tile id,
// Gaussian index and the pair's slot.  A workgroup takes kDupBlock
// consecutive Gaussians of the depth order, scans their pair counts on top
// of the block's first pair, stages offsets and rects in LDS, and its lanes
// then walk the workgroup's pair range together, one pair per lane (the
// owning Gaussian by binary search over the staged offsets), so the stores
// are coalesced and a Gaussian with many tiles is spread over many lanes.
// Slots are numbered in Gaussian index order (islot = exclusive prefix sum
// of tiles_touched), so the projection adjoint, one lane per Gaussian,
// reads the per-pair gradients of a wave's Gaussians from one contiguous
// range.  Pairs at or past capacity are dropped; a Gaussian whose slots do
// not all fit writes its pairs to slot 0 (in bounds; such lists are to be
// redone anyway).
__global__ __launch_bounds__(kDupBlock) void k_duplicate(const uint4 *drec, const uint32_t *count_dev,
                                                         const uint32_t *block_first, int tiles_x,
                                                         uint32_t capacity, uint32_t *tile_keys, uint32_t *vals,
                                                         uint32_t *slots) {
  __shared__ uint32_t sOff[kDupBlock + 1];
  __shared__ uint32_t sG[kDupBlock], sSlot[kDupBlock];
  __shared__ uint32_t sX[kDupBlock], sY[kDupBlock];
  const uint32_t V = *count_dev;
  const int64_t j0 = (int64_t)blockIdx.x * kDupBlock;
  if (j0 >= (int64_t)V) return;  // uniform over the workgroup
  const int nj = (int)min((int64_t)kDupBlock, (int64_t)V - j0);
  const int t = threadIdx.x;
  uint32_t np = 0;
  if (t < nj) {
    const uint4 r = drec[j0 + t];
    np = ((r.y & 0xffffu) - (r.x & 0xffffu) + 1u) * ((r.y >> 16) - (r.x >> 16) + 1u);
    sG[t] = r.w;
    sSlot[t] = (uint64_t)r.z + np <= capacity ? r.z : kNoSlot;
    sX[t] = r.x;
    sY[t] = r.y;
  }
  uint32_t total;
  const uint32_t first = block_first[blockIdx.x];
  sOff[t] = first + block_excl_scan<uint32_t>(np, &total);
  if (t == 0) sOff[nj] = first + total;
  __syncthreads();
  const uint32_t p0 = sOff[0], p1 = min(sOff[nj], capacity);
  for (uint32_t p = p0 + t; p < p1; p += kDupBlock) {
    // the last Gaussian k with sOff[k] <= p (offsets ascend; a run of equal
    // offsets ends at the Gaussian that owns the pairs)
    int lo = 0, hi = nj - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sOff[mid] <= p) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t local = p - sOff[lo];
    const uint32_t rx = sX[lo], ry = sY[lo];
    const uint32_t tx0 = rx & 0xffffu, ty0 = rx >> 16, w = (ry & 0xffffu) - tx0 + 1u;
    const uint32_t dy = local / w, dx = local - dy * w;
    tile_keys[p] = (ty0 + dy) * (uint32_t)tiles_x + tx0 + dx;
    vals[p] = sG[lo];
    slots[p] = sSlot[lo] == kNoSlot ? 0u : sSlot[lo] + local;
  }
}

__global__ void k_ranges(const uint32_t *tile_keys, const uint32_t *count_dev, uint32_t count_max,
                         uint32_t *ranges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t M = count_dev ? min(*count_dev, count_max) : count_max;
  if (i >= M) return;
  const uint32_t t = tile_keys[i];
  if (i == 0 || tile_keys[i - 1] != t) ranges[2 * t] = (uint32_t)i;
  if (i == (int64_t)M - 1 || tile_keys[i + 1] != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
}

inline int64_t nblocks_of(int64_t count) { return (count + kBlockKeys - 1) / kBlockKeys; }
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
  uint32_t *hist;    // [256][nblocks(count_max)]
  uint32_t *rowtot;  // [256]
};

size_t radix_hist_elems(int64_t count_max) { return 256 * (size_t)nblocks_of(count_max); }

// Sorts (k[0], v[0]) by the given passes, ping-ponging with (k[1], v[1]).
// Returns the index (0 or 1) of the buffer pair holding the result.
gs_status radix_sort(uint32_t *k[2], uint32_t *v[2], uint32_t *v2[2], const uint32_t *count_dev, int64_t count_max,
                     int npasses, const int *shifts, const int *widths, const RadixWs &rw, hipStream_t s,
                     int *result) {
  int cur = 0;
  const int64_t blocks = nblocks_of(count_max);
  for (int p = 0; p < npasses; ++p) {
    if (count_max == 0) break;
    GS_LAUNCH("radix_hist", k_radix_hist, blocks, kRadixBlock, 0, s, k[cur], count_dev, (uint32_t)count_max,
              shifts[p], widths[p], blocks, rw.hist);
    GS_LAUNCH("scan", k_radix_rowscan, 1 << widths[p], kScanBlock, 0, s, rw.hist, blocks, rw.rowtot);
    if (v2)
      GS_LAUNCH("radix_scatter", k_radix_scatter<true>, blocks, kRadixBlock, 0, s, k[cur], v[cur], v2[cur],
                k[1 - cur], v[1 - cur], v2[1 - cur], count_dev, (uint32_t)count_max, shifts[p], widths[p], blocks,
                rw.hist, rw.rowtot);
    else
      GS_LAUNCH("radix_scatter", k_radix_scatter<false>, blocks, kRadixBlock, 0, s, k[cur], v[cur], nullptr,
                k[1 - cur], v[1 - cur], nullptr, count_dev, (uint32_t)count_max, shifts[p], widths[p], blocks,
                rw.hist, rw.rowtot);
    cur = 1 - cur;
  }
  *result = cur;
  return GS_OK;
}

}  // namespace

size_t sort_pairs_workspace(int64_t count) {
  return 2 * align_up(sizeof(uint32_t) * (size_t)std::max<int64_t>(count, 1)) +
         align_up(sizeof(uint32_t) * radix_hist_elems(std::max<int64_t>(count, 1))) + align_up(sizeof(uint32_t) * 256);
}

gs_status sort_pairs_u32(uint32_t *keys, uint32_t *vals, int64_t count, int key_bits, void *ws, hipStream_t s) {
  if (count <= 1 || key_bits <= 0) return GS_OK;
  Carve cv(ws);
  uint32_t *k_alt = cv.take<uint32_t>((size_t)count), *v_alt = cv.take<uint32_t>((size_t)count);
  RadixWs rw{cv.take<uint32_t>(radix_hist_elems(count)), cv.take<uint32_t>(256)};
  int shifts[8], widths[8];
  const int np = plan_passes(key_bits, shifts, widths);
  uint32_t *kk[2] = {keys, k_alt}, *vv[2] = {vals, v_alt};
  int res = 0;
  gs_status st = radix_sort(kk, vv, nullptr, nullptr, count, np, shifts, widths, rw, s, &res);
  if (st != GS_OK) return st;
  if (res == 1) {
    GS_CHECK_HIP(hipMemcpyAsync(keys, k_alt, sizeof(uint32_t) * count, hipMemcpyDeviceToDevice, s), "sort copy");
    GS_CHECK_HIP(hipMemcpyAsync(vals, v_alt, sizeof(uint32_t) * count, hipMemcpyDeviceToDevice, s), "sort copy");
  }
  return GS_OK;
}

size_t scan_workspace(int64_t count) {
  const int64_t nparts = (count + kScanTile - 1) / kScanTile;
  return align_up(sizeof(uint64_t) * (size_t)(nparts + 1));
}

template <class T, class L>
static gs_status scan_exclusive_t(L load, T *out, int64_t count, T *total, void *ws, hipStream_t s) {
  if (count <= 0) {
    if (total) GS_LAUNCH("fill", k_fill<T>, 1, 64, 0, s, total, 1, (T)0);
    return GS_OK;
  }
  if (count <= kSmallScan) {
    GS_LAUNCH("scan", (k_scan_small<T, L>), 1, kSmallBlock, 0, s, load, out, count, total);
    return GS_OK;
  }
  const int64_t nparts = (count + kScanTile - 1) / kScanTile;
  T *partials = (T *)ws;
  GS_LAUNCH("scan", (k_scan_reduce<T, L>), nparts, kScanBlock, 0, s, load, count, partials);
  GS_LAUNCH("scan", (k_scan_apply<T, L>), nparts, kScanBlock, 0, s, load, out, count, (const T *)partials, total);
  return GS_OK;
}

// Exclusive scan; in may equal out.  total (device, may be NULL) receives the sum.
gs_status scan_exclusive(const uint32_t *in, uint32_t *out, int64_t count, uint32_t *total, void *ws,
                         hipStream_t s) {
  return scan_exclusive_t<uint32_t>(ArrayLoad<uint32_t>{in}, out, count, total, ws, s);
}
gs_status scan_exclusive_u64(const uint64_t *in, uint64_t *out, int64_t count, uint64_t *total, void *ws,
                             hipStream_t s) {
  return scan_exclusive_t<uint64_t>(ArrayLoad<uint64_t>{in}, out, count, total, ws, s);
}

}  // namespace gsmi

using namespace gsmi;

namespace {

struct BinLayout {
  uint32_t *kA, *vA, *kB, *vB, *block_pairs, *hist, *rowtot, *scalars, *ktmp, *vtmp, *stmp;
  uint64_t *total64;
  uint64_t *pos64;
  uint4 *rect, *drec;
  void *scan_ws;
  size_t bytes;
};

BinLayout bin_layout(void *ws, int64_t n, int64_t capacity) {
  Carve cv(ws);
  BinLayout L;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  const size_t cc = (size_t)(capacity > 0 ? capacity : 1);
  L.pos64 = cv.take<uint64_t>(nn);
  L.kA = cv.take<uint32_t>(nn);
  L.vA = cv.take<uint32_t>(nn);
  L.kB = cv.take<uint32_t>(nn);
  L.vB = cv.take<uint32_t>(nn);
  L.block_pairs = cv.take<uint32_t>((nn + kDupBlock - 1) / kDupBlock);
  L.rect = cv.take<uint4>(nn);
  L.drec = cv.take<uint4>(nn);
  const int64_t big = n > capacity ? n : capacity;
  L.hist = cv.take<uint32_t>(radix_hist_elems(big));
  L.rowtot = cv.take<uint32_t>(256);
  L.scan_ws = cv.take<char>(scan_workspace(big));
  L.scalars = cv.take<uint32_t>(4);
  L.total64 = cv.take<uint64_t>(1);
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

// The binning pipeline.  With n_dev == NULL the pair count M is read back
// (one stream synchronisation) and checked against capacity before the
// pairs are emitted; with n_dev it is left on the device (*n_dev) and every
// later kernel takes its count from there, clamped to capacity.
static gs_status bin_sort_impl(const gs_camera *cam, const gs_projected *proj, int64_t n, int64_t capacity, void *ws,
                               size_t ws_bytes, uint32_t *tile_ids, uint32_t *values, uint32_t *slots,
                               uint32_t *ranges, uint32_t *first_slot, int64_t *n_instances, uint32_t *n_dev,
                               hipStream_t s, const char *fn) {
  gs_status st = validate_camera(cam, fn);
  if (st != GS_OK) return st;
  GS_REQUIRE(proj && ranges && (n_instances || n_dev), "%s: NULL argument", fn);
  GS_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "%s: n out of range", fn);
  GS_REQUIRE(capacity >= 0 && capacity < (int64_t(1) << 32) - 1, "%s: capacity out of range", fn);
  if (n > 0) GS_REQUIRE(proj->rec && proj->radius && proj->tiles_touched, "%s: NULL projection plane", fn);
  GS_REQUIRE(((uintptr_t)proj->bin & 15u) == 0, "%s: bin must be 16-byte aligned", fn);
  if (capacity > 0) GS_REQUIRE(tile_ids && values && slots, "%s: NULL list output", fn);
  if (n > 0) GS_REQUIRE(first_slot, "%s: NULL first_slot", fn);
  size_t need = 0;
  gs_bin_sort_workspace(n, capacity, &need);
  if (ws_bytes < need || !ws) {
    set_error("%s: workspace %zu bytes < %zu", fn, ws_bytes, need);
    return GS_ERR_WORKSPACE;
  }
  const int W = cam->width, H = cam->height;
  const int tx = tiles_x_of(W), T = tx * tiles_y_of(H);
  BinLayout L = bin_layout(ws, n, capacity);
  RadixWs rw{L.hist, L.rowtot};
  // V: the visible count, the low word of the 64-bit scan total (little endian)
  uint32_t *V = (uint32_t *)L.total64, *Mdev = n_dev ? n_dev : L.scalars + 1;

  uint32_t M = 0;
  int order_buf = 0;
  if (n > 0) {
    // 1. compact the visible Gaussians with their depth keys
    //    (one 64-bit scan gives the visible positions and the index-order first slots;
    //    the visible count V is the low word of its total)
    if ((st = scan_exclusive_t<uint64_t>(TilesLoad{proj->tiles_touched}, L.pos64, n, L.total64, L.scan_ws, s)) !=
        GS_OK)
      return st;
    GS_LAUNCH("bin_compact", k_compact, grid1(n), 256, 0, s, proj->tiles_touched, L.pos64, proj->rec, proj->radius,
              (const uint4 *)proj->bin, n, W, H, (uint32_t)capacity, L.kA, L.vA, L.rect, first_slot);
    // 2. stable sort by depth (31 significant bits of a positive float)
    int shifts[8], widths[8];
    const int np = plan_passes(31, shifts, widths);
    uint32_t *kk[2] = {L.kA, L.kB}, *vv[2] = {L.vA, L.vB};
    if ((st = radix_sort(kk, vv, nullptr, V, n, np, shifts, widths, rw, s, &order_buf)) != GS_OK) return st;
    const uint32_t *order = vv[order_buf];
    // 3. emission records in depth order; the first pair of every block of them
    const int64_t dblocks = grid1(n, kDupBlock);
    GS_LAUNCH("bin_counts", k_depth_records, dblocks, kDupBlock, 0, s, order, V, L.rect, n, L.drec, L.block_pairs);
    if ((st = scan_exclusive(L.block_pairs, L.block_pairs, dblocks, Mdev, L.scan_ws, s)) != GS_OK) return st;
    if (!n_dev) {
      GS_CHECK_HIP(hipMemcpyAsync(&M, Mdev, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read M");
      GS_CHECK_HIP(hipStreamSynchronize(s), "sync M");
    }
  } else if (n_dev) {
    GS_LAUNCH("bin_fill", k_fill<uint32_t>, 1, 64, 0, s, n_dev, 1, 0u);
  }
  if (!n_dev) {
    *n_instances = M;
    if ((int64_t)M > capacity) {
      set_error("%s: %u pairs exceed capacity %lld", fn, M, (long long)capacity);
      return GS_ERR_CAPACITY;
    }
  }
  GS_LAUNCH("bin_fill", k_fill<uint32_t>, grid1(2 * (int64_t)T), 256, 0, s, ranges, 2 * (int64_t)T, 0u);
  // the number of pairs the later kernels size their grids for
  const int64_t mmax = n_dev ? capacity : (int64_t)M;
  if (n == 0 || mmax == 0) return GS_OK;

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
  GS_LAUNCH("bin_duplicate", k_duplicate, grid1(n, kDupBlock), kDupBlock, 0, s, L.drec, V, L.block_pairs, tx,
            (uint32_t)capacity, kk[0], vv[0], ss[0]);
  int res = 0;
  const uint32_t *mcount = n_dev ? n_dev : nullptr;
  if ((st = radix_sort(kk, vv, ss, mcount, mmax, np, shifts, widths, rw, s, &res)) != GS_OK) return st;
  GS_LAUNCH("bin_ranges", k_ranges, grid1(mmax), 256, 0, s, tile_ids, mcount, (uint32_t)mmax, ranges);
  return GS_OK;
}

gs_status gs_bin_sort(const gs_camera *cam, const gs_projected *proj, int64_t n, int64_t capacity, void *ws,
                      size_t ws_bytes, uint32_t *tile_ids, uint32_t *values, uint32_t *slots, uint32_t *ranges,
                      uint32_t *first_slot, int64_t *n_instances, void *stream) {
  return bin_sort_impl(cam, proj, n, capacity, ws, ws_bytes, tile_ids, values, slots, ranges, first_slot,
                       n_instances, nullptr, (hipStream_t)stream, "gs_bin_sort");
}

gs_status gs_bin_sort_async(const gs_camera *cam, const gs_projected *proj, int64_t n, int64_t capacity, void *ws,
                            size_t ws_bytes, uint32_t *tile_ids, uint32_t *values, uint32_t *slots,
                            uint32_t *ranges, uint32_t *first_slot, uint32_t *n_instances_dev, void *stream) {
  GS_REQUIRE(n_instances_dev, "gs_bin_sort_async: NULL n_instances_dev");
  return bin_sort_impl(cam, proj, n, capacity, ws, ws_bytes, tile_ids, values, slots, ranges, first_slot, nullptr,
                       n_instances_dev, (hipStream_t)stream, "gs_bin_sort_async");
}

}  // extern "C"
