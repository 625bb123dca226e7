// Clustering and primitive merging of the scalable construction (section
// 4.4): when an anchor is created, a random share 1/(k+1) of the primitives
// that look smaller than a pixel is selected, each selected primitive is
// merged with its k nearest neighbours among the other too-fine primitives
// (k = 3 in the paper), and every other primitive is kept.  The merged set,
// in the original order, becomes the new active set.
//
// Plan (gs_anchor_merge_plan):
//   * classes: a fine primitive i is selected iff the top 24 bits of
//     SplitMix64(seed + i) fall below floor(2^24 / (k+1)) (a counter-based
//     Bernoulli draw), else it is a candidate;
//   * neighbours: the candidates are hashed into a uniform grid (1024 cells
//     per axis at most, the cell edge h from the candidates' bounding box
//     and count) and sorted by cell; each selected primitive scans the 3x3x3
//     cells around its own, one contiguous key range per (y, z) row, keeping
//     its k best (d2, index) in registers.  Every candidate outside the
//     scanned block is more than R h away, so the result is exact once the
//     k-th distance is below R h (with a relative margin for the rounding of
//     the cell coordinates); otherwise the 5x5x5 block is scanned, and a
//     selected primitive whose neighbours are still farther scans all
//     candidates.  d2 = (dx dx + dy dy) + dz dz in binary64 on the binary32
//     means (dx exact), ties to the lower index: the k nearest are those of
//     a brute-force search, bit for bit;
//   * ownership: a candidate claimed by several selected primitives joins
//     the claim with the smallest (binary32 d2, selected index), one 64-bit
//     atomic minimum per claim;
//   * the new active set: the ascending indices of the primitives that are
//     not absorbed, and every primitive's new index.
// Apply (gs_anchor_merge_apply): the kept primitives are gathered, then each
// selected primitive with at least one neighbour is overwritten by the merge
// of its group (hierarchical-3DGS style, in FP64): weights w = o s_x s_y s_z,
// the weighted mean, the weighted second moment about it (covariances plus
// spreads), SH coefficients averaged with the same weights, opacity
// min(0.99, W / sqrt(det Sigma)); Sigma is diagonalised by cyclic Jacobi
// rotations into the rotation quaternion and log-scales.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace gsmi {
namespace {

constexpr int kMaxK = 8;
constexpr int kCellBits = 10;
constexpr int kCells = 1 << kCellBits;  // per axis
constexpr int kClsOther = 0, kClsSeed = 1, kClsCand = 2;
constexpr int kBoxBlocks = 512;

__global__ void k_merge_classes(const int32_t *fine, int64_t n, uint32_t thr, uint64_t seed, int32_t *cls,
                                uint32_t *seed_flag, uint32_t *cand_flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = kClsOther;
  if (fine[i]) c = (uint32_t)(splitmix64(seed + (uint64_t)i) >> 40) < thr ? kClsSeed : kClsCand;
  cls[i] = c;
  seed_flag[i] = c == kClsSeed ? 1u : 0u;
  cand_flag[i] = c == kClsCand ? 1u : 0u;
}

__global__ void k_flag_index(const uint32_t *flag, const uint32_t *pos, int64_t n, uint32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = (uint32_t)i;
}

// per-workgroup min / max of the candidates' means: partials [block][6]
__global__ __launch_bounds__(256) void k_cand_box(const uint32_t *cand, int64_t nc, const float *means, int64_t n,
                                                  float *partials) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < nc; t += (int64_t)gridDim.x * 256) {
    const int64_t j = cand[t];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float x = means[a * n + j];
      lo[a] = fminf(lo[a], x);
      hi[a] = fmaxf(hi[a], x);
    }
  }
  __shared__ float red[6][256];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    red[a][threadIdx.x] = lo[a];
    red[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + off]);
        red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + off]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) partials[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

struct Grid {
  double ox, oy, oz, inv_h, h;
};

__device__ __forceinline__ int64_t cell_of(double x, double o, double inv_h) {
  const double c = floor((x - o) * inv_h);
  return (int64_t)fmin(fmax(c, -1048576.0), 1048576.0);
}

__device__ __forceinline__ uint32_t cell_key(int64_t cx, int64_t cy, int64_t cz) {
  return (uint32_t)cx | ((uint32_t)cy << kCellBits) | ((uint32_t)cz << (2 * kCellBits));
}

__global__ void k_cell_keys(const uint32_t *cand, int64_t nc, const float *means, int64_t n, Grid gr,
                            uint32_t *keys, uint32_t *vals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc) return;
  const int64_t j = cand[t];
  const int64_t cx = min<int64_t>(max<int64_t>(cell_of(means[j], gr.ox, gr.inv_h), 0), kCells - 1);
  const int64_t cy = min<int64_t>(max<int64_t>(cell_of(means[n + j], gr.oy, gr.inv_h), 0), kCells - 1);
  const int64_t cz = min<int64_t>(max<int64_t>(cell_of(means[2 * n + j], gr.oz, gr.inv_h), 0), kCells - 1);
  keys[t] = cell_key(cx, cy, cz);
  vals[t] = (uint32_t)j;
}

// (d2, index) order
__device__ __forceinline__ bool before(double d, uint32_t j, double e, uint32_t k) {
  return d < e || (d == e && j < k);
}

// the K best (d2, index), ascending, in registers (K a compile-time
// constant so that no array is indexed at run time)
template <int K>
struct TopK {
  double d[K];
  uint32_t j[K];
  __device__ __forceinline__ void reset() {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      d[t] = INFINITY;
      j[t] = 0xffffffffu;
    }
  }
  // insertion without branches: from the top down, entry t takes entry
  // t - 1 if the new pair precedes that one, else the new pair if it
  // precedes entry t, else stays
  __device__ __forceinline__ void insert(double dd, uint32_t jj) {
    if (!before(dd, jj, d[K - 1], j[K - 1])) return;
#pragma unroll
    for (int t = K - 1; t >= 0; --t) {
      const bool up = t > 0 && before(dd, jj, d[t > 0 ? t - 1 : 0], j[t > 0 ? t - 1 : 0]);
      const bool here = before(dd, jj, d[t], j[t]);
      const double nd = up ? d[t > 0 ? t - 1 : 0] : (here ? dd : d[t]);
      const uint32_t nj = up ? j[t > 0 ? t - 1 : 0] : (here ? jj : j[t]);
      d[t] = nd;
      j[t] = nj;
    }
  }
};

// binary64 squared distance, (dx dx + dy dy) + dz dz, each operation rounded
// (contraction off: no product is fused into an add)
__device__ __forceinline__ double sq_dist(double x, double y, double z, const float *means, int64_t n, int64_t j) {
#pragma clang fp contract(off)
  const double dx = (double)means[j] - x, dy = (double)means[n + j] - y, dz = (double)means[2 * n + j] - z;
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ uint32_t lower_bound(const uint32_t *a, uint32_t n, uint32_t key) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// One lane per selected primitive.  kk = min(K, candidates) neighbours are
// kept; with fewer than K candidates every candidate is a neighbour.
template <int K>
__global__ __launch_bounds__(256) void k_knn(const uint32_t *seeds, int64_t ns, const uint32_t *keys,
                                             const uint32_t *vals, int64_t nc, const float *means, int64_t n,
                                             Grid gr, int32_t *nbr, unsigned long long *claim) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  const int64_t s = seeds[t];
  const double x = means[s], y = means[n + s], z = means[2 * n + s];
  const int64_t cx = cell_of(x, gr.ox, gr.inv_h), cy0 = cell_of(y, gr.oy, gr.inv_h),
                cz0 = cell_of(z, gr.oz, gr.inv_h);
  TopK<K> best;
  // the K-th entry once K candidates exist; with fewer, the last one there is
  const int last = (int)min<int64_t>(K, nc) - 1;
  bool done = false;
  for (int R = 1; R <= 2 && !done; ++R) {
    best.reset();
    const int64_t x0 = max<int64_t>(cx - R, 0), x1 = min<int64_t>(cx + R, kCells - 1);
    const int64_t y0 = max<int64_t>(cy0 - R, 0), y1 = min<int64_t>(cy0 + R, kCells - 1);
    const int64_t z0 = max<int64_t>(cz0 - R, 0), z1 = min<int64_t>(cz0 + R, kCells - 1);
    if (x0 <= x1) {
      for (int64_t cz = z0; cz <= z1; ++cz)
        for (int64_t cy = y0; cy <= y1; ++cy) {
          const uint32_t b = lower_bound(keys, (uint32_t)nc, cell_key(x0, cy, cz));
          const uint32_t e = lower_bound(keys, (uint32_t)nc, cell_key(x1, cy, cz) + 1u);
          for (uint32_t q = b; q < e; ++q) {
            const uint32_t j = vals[q];
            best.insert(sq_dist(x, y, z, means, n, j), j);
          }
        }
    }
    // every candidate outside the block is more than R h away
    const double lim = (double)R * gr.h * (1.0 - 1e-9);
    double dl = INFINITY;
    uint32_t jl = 0xffffffffu;
#pragma unroll
    for (int u = 0; u < K; ++u)
      if (u == last) dl = best.d[u], jl = best.j[u];
    done = jl != 0xffffffffu && dl < lim * lim;
  }
  if (!done) {  // brute force over every candidate
    best.reset();
    for (int64_t q = 0; q < nc; ++q) {
      const uint32_t j = vals[q];
      best.insert(sq_dist(x, y, z, means, n, j), j);
    }
  }
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const bool have = u <= last && best.j[u] != 0xffffffffu;
    nbr[s * K + u] = have ? (int32_t)best.j[u] : -1;
    if (have) {
      const float d32 = (float)best.d[u];
      const unsigned long long key = ((unsigned long long)__float_as_uint(d32) << 32) | (unsigned long long)s;
      atomicMin(claim + best.j[u], key);
    }
  }
}

__global__ void k_owners(const unsigned long long *claim, int64_t n, int32_t *owner, uint32_t *keep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long c = claim[i];
  const bool absorbed = c != ~0ull;
  owner[i] = absorbed ? (int32_t)(c & 0xffffffffull) : -1;
  keep[i] = absorbed ? 0u : 1u;
}

__global__ void k_new_index(const uint32_t *keep, const uint32_t *pos, int64_t n, int32_t *new_index,
                            int32_t *keep_index) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  new_index[i] = keep[i] ? (int32_t)pos[i] : -1;
  if (keep[i]) keep_index[pos[i]] = (int32_t)i;
}

// ----------------------------------------------------------------- merge
__device__ void quat_to_rot(double w, double x, double y, double z, double R[9]) {
  const double nrm = sqrt(w * w + x * x + y * y + z * z);
  w /= nrm, x /= nrm, y /= nrm, z /= nrm;
  R[0] = 1 - 2 * (y * y + z * z), R[1] = 2 * (x * y - w * z), R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z), R[4] = 1 - 2 * (x * x + z * z), R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y), R[7] = 2 * (y * z + w * x), R[8] = 1 - 2 * (x * x + y * y);
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix A (row-major):
// on return A is diagonal (the eigenvalues) and V (row-major) holds the
// eigenvectors as columns, A_in = V diag V^T.
__device__ void jacobi3(double A[9], double V[9]) {
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    const double dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (off <= 1e-34 * dia) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double apq = A[3 * p + q];
      if (fabs(apq) <= 1e-300) continue;
      const double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
      const double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double cs = 1.0 / sqrt(tt * tt + 1.0), sn = tt * cs;
      // A <- J^T A J with J the rotation in the (p, q) plane
      for (int r = 0; r < 3; ++r) {  // columns p, q
        const double arp = A[3 * r + p], arq = A[3 * r + q];
        A[3 * r + p] = cs * arp - sn * arq;
        A[3 * r + q] = sn * arp + cs * arq;
      }
      for (int r = 0; r < 3; ++r) {  // rows p, q
        const double apr = A[3 * p + r], aqr = A[3 * q + r];
        A[3 * p + r] = cs * apr - sn * aqr;
        A[3 * q + r] = sn * apr + cs * aqr;
      }
      for (int r = 0; r < 3; ++r) {
        const double vrp = V[3 * r + p], vrq = V[3 * r + q];
        V[3 * r + p] = cs * vrp - sn * vrq;
        V[3 * r + q] = sn * vrp + cs * vrq;
      }
    }
  }
}

// unit quaternion (w, x, y, z) of a rotation matrix (row-major)
__device__ void rot_to_quat(const double R[9], double q[4]) {
  const double tr = R[0] + R[4] + R[8];
  if (tr > 0.0) {
    const double S = sqrt(tr + 1.0) * 2.0;
    q[0] = 0.25 * S, q[1] = (R[7] - R[5]) / S, q[2] = (R[2] - R[6]) / S, q[3] = (R[3] - R[1]) / S;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    const double S = sqrt(1.0 + R[0] - R[4] - R[8]) * 2.0;
    q[0] = (R[7] - R[5]) / S, q[1] = 0.25 * S, q[2] = (R[1] + R[3]) / S, q[3] = (R[2] + R[6]) / S;
  } else if (R[4] > R[8]) {
    const double S = sqrt(1.0 + R[4] - R[0] - R[8]) * 2.0;
    q[0] = (R[2] - R[6]) / S, q[1] = (R[1] + R[3]) / S, q[2] = 0.25 * S, q[3] = (R[5] + R[7]) / S;
  } else {
    const double S = sqrt(1.0 + R[8] - R[0] - R[4]) * 2.0;
    q[0] = (R[3] - R[1]) / S, q[1] = (R[2] + R[6]) / S, q[2] = (R[5] + R[7]) / S, q[3] = 0.25 * S;
  }
}

struct MergeArgs {
  const float *means, *log_scales, *quats, *logits, *sh;
  int64_t n;
  int nsh;  // SH coefficients per Gaussian (3 (d + 1)^2)
  const int32_t *cls, *nbr, *owner, *new_index;
  int k;
  float *o_means, *o_log_scales, *o_quats, *o_logits, *o_sh;
  int64_t m;  // size of the new set (the output planes' stride)
  int32_t *merged;
};

__global__ __launch_bounds__(128) void k_merge_apply(MergeArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n || a.cls[s] != kClsSeed) return;
  const int64_t n = a.n;
  int64_t mem[kMaxK + 1];
  int nm = 0;
  mem[nm++] = s;
  for (int u = 0; u < a.k; ++u) {
    const int32_t j = a.nbr[s * a.k + u];
    if (j >= 0 && a.owner[j] == (int32_t)s) mem[nm++] = j;
  }
  if (nm == 1) return;  // no neighbour joined: kept as it is (gathered)
  // the members in ascending index order after the selected one
  for (int i = 2; i < nm; ++i)
    for (int j = i; j > 1 && mem[j - 1] > mem[j]; --j) {
      const int64_t t = mem[j];
      mem[j] = mem[j - 1];
      mem[j - 1] = t;
    }
  double w[kMaxK + 1], W = 0.0, mu[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < nm; ++c) {
    const int64_t i = mem[c];
    const double o = 1.0 / (1.0 + exp(-(double)a.logits[i]));
    w[c] = o * exp((double)a.log_scales[i] + (double)a.log_scales[n + i] + (double)a.log_scales[2 * n + i]);
    W += w[c];
    for (int d = 0; d < 3; ++d) mu[d] += w[c] * (double)a.means[d * n + i];
  }
  for (int d = 0; d < 3; ++d) mu[d] /= W;
  double S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int c = 0; c < nm; ++c) {
    const int64_t i = mem[c];
    double R[9];
    quat_to_rot(a.quats[i], a.quats[n + i], a.quats[2 * n + i], a.quats[3 * n + i], R);
    double s2[3], dv[3];
    for (int d = 0; d < 3; ++d) {
      s2[d] = exp(2.0 * (double)a.log_scales[d * n + i]);
      dv[d] = (double)a.means[d * n + i] - mu[d];
    }
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) {
        double v = dv[r] * dv[q];
        for (int e = 0; e < 3; ++e) v += R[3 * r + e] * s2[e] * R[3 * q + e];
        S[3 * r + q] += w[c] * v;
      }
  }
  for (int e = 0; e < 9; ++e) S[e] /= W;
  const double det = S[0] * (S[4] * S[8] - S[5] * S[7]) - S[1] * (S[3] * S[8] - S[5] * S[6]) +
                     S[2] * (S[3] * S[7] - S[4] * S[6]);
  const double op = fmin(0.99, W / sqrt(fmax(det, 1e-300)));
  double A[9], V[9];
  for (int e = 0; e < 9; ++e) A[e] = S[e];
  jacobi3(A, V);
  const double vdet = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
                      V[2] * (V[3] * V[7] - V[4] * V[6]);
  if (vdet < 0.0)
    for (int r = 0; r < 3; ++r) V[3 * r + 2] = -V[3 * r + 2];
  double q[4];
  rot_to_quat(V, q);
  const int64_t m = a.m, p = a.new_index[s];
  if (p < 0 || p >= m) return;  // an output smaller than the plan's new set
  for (int d = 0; d < 3; ++d) {
    a.o_means[d * m + p] = (float)mu[d];
    a.o_log_scales[d * m + p] = (float)(0.5 * log(fmax(A[4 * d], 1e-300)));
  }
  for (int d = 0; d < 4; ++d) a.o_quats[d * m + p] = (float)q[d];
  a.o_logits[p] = (float)log(op / (1.0 - op));
  for (int e = 0; e < a.nsh; ++e) {
    double v = 0.0;
    for (int c = 0; c < nm; ++c) v += w[c] * (double)a.sh[(int64_t)e * n + mem[c]];
    a.o_sh[(int64_t)e * m + p] = (float)(v / W);
  }
  if (a.merged) a.merged[p] = 1;
}

// planes[p][i] = value where mask[i] != 0 (plane p = blockIdx.y)
__global__ void k_masked_fill(float *planes, int64_t n, const int32_t *mask, float value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && mask[i]) planes[(int64_t)blockIdx.y * n + i] = value;
}

template <class T>
__global__ void k_fill_t(T *p, int64_t count, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

inline unsigned grid_of(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

struct PlanLayout {
  uint32_t *seed_flag, *cand_flag, *pos, *seeds, *cands, *keys, *vals, *keep, *scalars;
  unsigned long long *claim;
  float *box;
  void *scan_ws, *sort_ws;
  size_t bytes;
};

PlanLayout plan_layout(void *ws, int64_t n) {
  Carve cv(ws);
  PlanLayout L;
  const size_t N = (size_t)std::max<int64_t>(n, 1);
  L.seed_flag = cv.take<uint32_t>(N);
  L.cand_flag = cv.take<uint32_t>(N);
  L.pos = cv.take<uint32_t>(N);
  L.seeds = cv.take<uint32_t>(N);
  L.cands = cv.take<uint32_t>(N);
  L.keys = cv.take<uint32_t>(N);
  L.vals = cv.take<uint32_t>(N);
  L.keep = cv.take<uint32_t>(N);
  L.scalars = cv.take<uint32_t>(4);
  L.claim = cv.take<unsigned long long>(N);
  L.box = cv.take<float>(6 * kBoxBlocks);
  L.scan_ws = cv.take<char>(scan_workspace((int64_t)N));
  L.sort_ws = cv.take<char>(sort_pairs_workspace((int64_t)N));
  L.bytes = cv.off;
  return L;
}

}  // namespace
}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_anchor_merge_workspace(int64_t n, size_t *bytes) {
  GS_REQUIRE(bytes && n >= 0 && n < (1ll << 31), "gs_anchor_merge_workspace: bad argument");
  *bytes = plan_layout(nullptr, n).bytes;
  return GS_OK;
}

gs_status gs_anchor_merge_plan(const gs_gaussians *g, const int32_t *fine, int32_t k, uint64_t seed, int32_t *cls,
                               int32_t *nbr, int32_t *owner, int32_t *new_index, int32_t *keep_index,
                               int64_t *n_keep, void *ws, size_t ws_bytes, void *stream) {
  GS_REQUIRE(g && n_keep, "gs_anchor_merge_plan: NULL argument");
  GS_REQUIRE(k >= 1 && k <= kMaxK, "gs_anchor_merge_plan: k must be in [1, %d]", kMaxK);
  const int64_t n = g->n;
  GS_REQUIRE(n >= 0 && n < (1ll << 31), "gs_anchor_merge_plan: n out of range");
  *n_keep = n;
  if (n == 0) return GS_OK;
  GS_REQUIRE(g->means && fine && cls && nbr && owner && new_index && keep_index,
             "gs_anchor_merge_plan: NULL array");
  const PlanLayout L = plan_layout(ws, n);
  if (!ws || ws_bytes < L.bytes) {
    set_error("gs_anchor_merge_plan: workspace %zu bytes < %zu", ws_bytes, L.bytes);
    return GS_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  gs_status st;
  const uint32_t thr = (uint32_t)((1u << 24) / (uint32_t)(k + 1));
  GS_LAUNCH("merge_classes", k_merge_classes, grid_of(n), 256, 0, s, fine, n, thr, seed, cls, L.seed_flag,
            L.cand_flag);
  // the selected and the candidate indices, ascending
  if ((st = scan_exclusive(L.seed_flag, L.pos, n, L.scalars, L.scan_ws, s)) != GS_OK) return st;
  GS_LAUNCH("merge_classes", k_flag_index, grid_of(n), 256, 0, s, L.seed_flag, L.pos, n, L.seeds);
  if ((st = scan_exclusive(L.cand_flag, L.pos, n, L.scalars + 1, L.scan_ws, s)) != GS_OK) return st;
  GS_LAUNCH("merge_classes", k_flag_index, grid_of(n), 256, 0, s, L.cand_flag, L.pos, n, L.cands);
  uint32_t counts[2];
  GS_CHECK_HIP(hipMemcpyAsync(counts, L.scalars, sizeof(counts), hipMemcpyDeviceToHost, s), "merge counts");
  GS_CHECK_HIP(hipStreamSynchronize(s), "merge counts");
  const int64_t ns = counts[0], nc = counts[1];
  GS_LAUNCH("merge_fill", k_fill_t<int32_t>, grid_of(n * k), 256, 0, s, nbr, n * k, (int32_t)-1);
  GS_LAUNCH("merge_fill", k_fill_t<unsigned long long>, grid_of(n), 256, 0, s, L.claim, n, ~0ull);
  if (ns > 0 && nc > 0) {
    // the grid: the candidates' bounding box, about 8 per cell in a uniform
    // cloud, at most kCells per axis
    const unsigned bb = (unsigned)std::min<int64_t>(grid_of(nc), kBoxBlocks);
    GS_LAUNCH("merge_grid", k_cand_box, bb, 256, 0, s, L.cands, nc, g->means, n, L.box);
    std::vector<float> box(6 * bb);
    GS_CHECK_HIP(hipMemcpyAsync(box.data(), L.box, sizeof(float) * box.size(), hipMemcpyDeviceToHost, s), "box");
    GS_CHECK_HIP(hipStreamSynchronize(s), "box");
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (unsigned b = 0; b < bb; ++b)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], (double)box[6 * b + a]);
        hi[a] = std::max(hi[a], (double)box[6 * b + 3 + a]);
      }
    GS_REQUIRE(std::isfinite(lo[0] + lo[1] + lo[2] + hi[0] + hi[1] + hi[2]),
               "gs_anchor_merge_plan: a candidate mean is not finite");
    double ext = std::max(std::max(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
    if (!(ext > 0.0)) ext = 1.0;
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) vol *= std::max(hi[a] - lo[a], 1e-3 * ext);
    double h = std::cbrt(8.0 * vol / (double)nc);
    h = std::max(h, ext / (double)(kCells - 1) * (1.0 + 1e-6));
    const Grid gr{lo[0], lo[1], lo[2], 1.0 / h, h};
    GS_LAUNCH("merge_grid", k_cell_keys, grid_of(nc), 256, 0, s, L.cands, nc, g->means, n, gr, L.keys, L.vals);
    if ((st = sort_pairs_u32(L.keys, L.vals, nc, 3 * kCellBits, L.sort_ws, s)) != GS_OK) return st;
#define GS_KNN(K)                                                                                           \
  case K:                                                                                                   \
    GS_LAUNCH("merge_knn", k_knn<K>, grid_of(ns), 256, 0, s, L.seeds, ns, L.keys, L.vals, nc, g->means, n, gr, \
              nbr, L.claim);                                                                                \
    break;
    switch (k) { GS_KNN(1) GS_KNN(2) GS_KNN(3) GS_KNN(4) GS_KNN(5) GS_KNN(6) GS_KNN(7) GS_KNN(8) }
#undef GS_KNN
  }
  GS_LAUNCH("merge_owners", k_owners, grid_of(n), 256, 0, s, L.claim, n, owner, L.keep);
  if ((st = scan_exclusive(L.keep, L.pos, n, L.scalars + 2, L.scan_ws, s)) != GS_OK) return st;
  GS_LAUNCH("merge_owners", k_new_index, grid_of(n), 256, 0, s, L.keep, L.pos, n, new_index, keep_index);
  uint32_t kept = 0;
  GS_CHECK_HIP(hipMemcpyAsync(&kept, L.scalars + 2, sizeof(kept), hipMemcpyDeviceToHost, s), "merge keep count");
  GS_CHECK_HIP(hipStreamSynchronize(s), "merge keep count");
  *n_keep = kept;
  return GS_OK;
}

gs_status gs_masked_fill(float *planes, int64_t n, int32_t n_planes, const int32_t *mask, float value,
                         void *stream) {
  GS_REQUIRE(n >= 0 && n_planes >= 0, "gs_masked_fill: bad sizes");
  if (n == 0 || n_planes == 0) return GS_OK;
  GS_REQUIRE(planes && mask, "gs_masked_fill: NULL argument");
  GS_LAUNCH("masked_fill", k_masked_fill, dim3(grid_of(n), (unsigned)n_planes), 256, 0, (hipStream_t)stream, planes,
            n, mask, value);
  return GS_OK;
}

gs_status gs_anchor_offload(int32_t n_planes, const void *const *src, const size_t *bytes, void *host, void *stream) {
  GS_REQUIRE(n_planes >= 0 && (n_planes == 0 || (src && bytes && host)), "gs_anchor_offload: bad argument");
  size_t off = 0;
  for (int32_t p = 0; p < n_planes; ++p) {
    if (bytes[p]) {
      GS_REQUIRE(src[p], "gs_anchor_offload: plane %d is NULL", p);
      GS_CHECK_HIP(hipMemcpyAsync((char *)host + off, src[p], bytes[p], hipMemcpyDeviceToHost, (hipStream_t)stream),
                   "gs_anchor_offload copy");
    }
    off += align_up(bytes[p]);
  }
  return GS_OK;
}

gs_status gs_anchor_reload(int32_t n_planes, void *const *dst, const size_t *bytes, const void *host, void *stream) {
  GS_REQUIRE(n_planes >= 0 && (n_planes == 0 || (dst && bytes && host)), "gs_anchor_reload: bad argument");
  size_t off = 0;
  for (int32_t p = 0; p < n_planes; ++p) {
    if (bytes[p]) {
      GS_REQUIRE(dst[p], "gs_anchor_reload: plane %d is NULL", p);
      GS_CHECK_HIP(hipMemcpyAsync(dst[p], (const char *)host + off, bytes[p], hipMemcpyHostToDevice, (hipStream_t)stream),
                   "gs_anchor_reload copy");
    }
    off += align_up(bytes[p]);
  }
  return GS_OK;
}

size_t gs_anchor_host_bytes(int32_t n_planes, const size_t *bytes) {
  size_t off = 0;
  for (int32_t p = 0; bytes && p < n_planes; ++p) off += align_up(bytes[p]);
  return off;
}

gs_status gs_anchor_merge_apply(const gs_gaussians *g, const int32_t *cls, const int32_t *nbr, const int32_t *owner,
                                const int32_t *new_index, const int32_t *keep_index, int32_t k, gs_gaussians *out,
                                int32_t *merged, void *stream) {
  GS_REQUIRE(g && out, "gs_anchor_merge_apply: NULL argument");
  GS_REQUIRE(k >= 1 && k <= kMaxK, "gs_anchor_merge_apply: k must be in [1, %d]", kMaxK);
  GS_REQUIRE(out->sh_degree == g->sh_degree && out->n >= 0 && out->n <= g->n,
             "gs_anchor_merge_apply: output shape differs from the input's");
  const int64_t n = g->n, m = out->n;
  if (n == 0 || m == 0) return GS_OK;
  GS_REQUIRE(g->means && g->log_scales && g->quats && g->opacity_logits && g->sh && out->means &&
                 out->log_scales && out->quats && out->opacity_logits && out->sh && cls && nbr && owner &&
                 new_index && keep_index,
             "gs_anchor_merge_apply: NULL array");
  hipStream_t s = (hipStream_t)stream;
  gs_status st;
  const int nsh = 3 * (g->sh_degree + 1) * (g->sh_degree + 1);
  const float *src[5] = {g->means, g->log_scales, g->quats, g->opacity_logits, g->sh};
  float *dst[5] = {out->means, out->log_scales, out->quats, out->opacity_logits, out->sh};
  const int planes[5] = {3, 3, 4, 1, nsh};
  for (int p = 0; p < 5; ++p)
    if ((st = gs_gather_planes(src[p], n, planes[p], keep_index, m, dst[p], stream)) != GS_OK) return st;
  if (merged) GS_LAUNCH("merge_fill", k_fill_t<int32_t>, grid_of(m), 256, 0, s, merged, m, 0);
  MergeArgs a{g->means, g->log_scales, g->quats, g->opacity_logits, g->sh, n, nsh, cls, nbr, owner, new_index,
              (int)k, out->means, out->log_scales, out->quats, out->opacity_logits, out->sh, m, merged};
  GS_LAUNCH("merge_apply", k_merge_apply, grid_of(n, 128), 128, 0, s, a);
  return GS_OK;
}

}  // extern "C"
