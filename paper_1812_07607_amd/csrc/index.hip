// index.hip -- kernels of the index-pruned eps-join.
//
// Paper: section "Query Processing" builds an index on the fly inside a join
// query (one relation is indexed, the other probes it), and section "Derived
// Data" answers Euclidean threshold queries with a Ball-tree over the feature
// vectors.  Here the index is one level of balls over 256-row blocks, built
// on the GPU for the matrix-core tiles:
//   1. every row is assigned to its nearest pivot (a strided sample of S) by
//      a pass of the matrix-core kernel whose epilogue keeps each row's best
//      column, and the rows of each relation are ordered by pivot, so
//      consecutive rows are close and a 256-row block is a tight cluster;
//   2. every block gets a ball: its float32 centroid c and a radius r that
//      bounds |x - c| from above for each of its rows;
//   3. a bound pass on the matrix cores tests every row a of R against every
//      block ball (c, r) of S: a block can hold a partner of a only if
//      |a - c| <= eps + r (triangle inequality), i.e. d2(a, c) <= (eps + r)^2,
//      which the candidate filter evaluates with its usual rigorous margin
//      (so the test errs only towards keeping a block); a hit marks the pair
//      (tile of a, block) in a bitmap;
//   4. a (row tile, column tile) pair is computed only if both directions are
//      marked (rows of the R tile near the S block's ball, rows of the S
//      tile near the R tile's ball); the survivors form a tile list, in the
//      full grid's walk order, that the candidate pass walks instead of the
//      full grid.
// Pruning is exact: a pair with d2 <= eps^2 always lies in a surviving tile,
// and the candidates of surviving tiles get the usual exact recheck.
#include "core.hpp"

namespace dl {

// Rows 0, stride, 2 stride, ... (m of them) of X into out (m x d, dense).
__global__ void gather_rows_kernel(const float* __restrict__ X, int64_t ld, int64_t stride, int64_t m, int d,
                                   float* __restrict__ out) {
  const int64_t total = m * (int64_t)d;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / d, k = t - r * d;
    out[t] = X[r * stride * ld + k];
  }
}

// Sort keys (pivot << bj | row) of a relation's rows, for the row-bucketed
// ordering (which is then a stable counting sort by pivot).  argkey: per row
// the nearest pass's key, whose low word is the complement of the pivot.
__global__ void pivot_keys_kernel(const unsigned long long* __restrict__ argkey, int64_t n, uint32_t npiv, int bj,
                                  unsigned long long* __restrict__ keys, float* __restrict__ vals) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t c = 0xffffffffu - (uint32_t)(argkey[t] & 0xffffffffull);
    const uint32_t pv = c < npiv ? c : npiv - 1;  // a row no pivot won (NaN input) goes to the last
    keys[t] = ((unsigned long long)pv << bj) | (unsigned long long)t;
    vals[t] = 0.0f;
  }
}

// One workgroup per block of kTile consecutive ordered rows (row q of the
// order is row perm[q] of X): the block's centroid in float32 (the float64
// mean, rounded) and the threshold Tb = (eps + r)^2 for its ball, with r an
// upper bound of max |x - c| over the block's rows.  The squared distances
// are summed in float64 (relative error below d 2^-53) and r and Tb are
// rounded up by 2^-30 relative, far more than that error.
__global__ __launch_bounds__(256) void block_ball_kernel(const float* __restrict__ X, int64_t ld,
                                                         const uint32_t* __restrict__ perm, int64_t n, int d,
                                                         double eps, float* __restrict__ cent,
                                                         double* __restrict__ Tb) {
  extern __shared__ float c_lds[];  // d floats
  __shared__ double r2_wave[4];
  const int64_t b = blockIdx.x;
  const int64_t r0 = b * kTile;
  const int rows = (int)min((int64_t)kTile, n - r0);
  __shared__ int64_t roff[kTile];  // the block's row offsets in X
  for (int r = threadIdx.x; r < rows; r += blockDim.x) roff[r] = (int64_t)perm[r0 + r] * ld;
  __syncthreads();
  for (int k = threadIdx.x; k < d; k += blockDim.x) {
    // eight rows' loads in flight, added in row order
    double s = 0.0;
    int r = 0;
    for (; r + 8 <= rows; r += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = X[roff[r + u] + k];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; r < rows; ++r) s += (double)X[roff[r] + k];
    const float c = (float)(s / (double)rows);
    c_lds[k] = c;
    cent[b * (int64_t)d + k] = c;
  }
  __syncthreads();
  // one wave per row: lanes over k, a float64 sum per row, the block maximum
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double r2max = 0.0;
  for (int r = wave; r < rows; r += 4) {
    const float* x = X + roff[r];
    double s = 0.0;
    for (int k = lane; k < d; k += 64) {
      const double t = (double)x[k] - (double)c_lds[k];
      s += t * t;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    r2max = fmax(r2max, s);
  }
  if (lane == 0) r2_wave[wave] = r2max;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(r2_wave[0], r2_wave[1]), fmax(r2_wave[2], r2_wave[3]));
    const double r = sqrt(m) * (1.0 + 0x1p-30) + 0x1p-100;
    const double e = eps + r;
    Tb[b] = e * e * (1.0 + 0x1p-30);
  }
}

// One wave per row tile ti: the word w of its survivor bitmap holds the
// column tiles 32 w .. 32 w + 31 whose pair with ti is marked in both
// directions: m1[ti][tj] (a row of tile ti near the ball of block tj) and
// m2[tj][ti] (a row of tile tj near the ball of block ti).  A self-join keeps
// tj >= ti only.
__global__ __launch_bounds__(256) void survive_kernel(const uint32_t* __restrict__ m1, int64_t m1w,
                                                      const uint32_t* __restrict__ m2, int64_t m2w, int64_t nTR,
                                                      int64_t nTS, int self, uint32_t* __restrict__ surv, int64_t sw) {
  const int lane = threadIdx.x & 63;
  const int64_t ti = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (ti >= nTR) return;
  for (int64_t w = lane; w < sw; w += 64) {
    uint32_t word = m1[ti * m1w + w];
    uint32_t keep = 0;
    for (int bit = 0; bit < 32; ++bit) {
      const int64_t tj = w * 32 + bit;
      if (tj >= nTS || !((word >> bit) & 1u)) continue;
      if (self && tj < ti) continue;
      if ((m2[tj * m2w + (ti >> 5)] >> (ti & 31)) & 1u) keep |= 1u << bit;
    }
    surv[ti * sw + w] = keep;
  }
}

// The tile list is ordered like the full grid's walk: groups of gm row tiles
// (as many as keep their operand tiles in an XCD's L2), column tiles in
// order within a group, the group's row tiles in order for each column tile;
// consecutive workgroups then share row tiles while column tiles stream past.
// One thread per (group, column tile): its survivors.
__global__ void group_count_kernel(const uint32_t* __restrict__ surv, int64_t sw, int64_t nTR, int64_t nTS,
                                   int64_t gm, uint32_t* __restrict__ cnt) {
  const int64_t ng = (nTR + gm - 1) / gm;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ng * nTS;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = t / nTS, tj = t - g * nTS;
    const int64_t t1 = min(nTR, (g + 1) * gm);
    uint32_t c = 0;
    for (int64_t ti = g * gm; ti < t1; ++ti) c += (surv[ti * sw + (tj >> 5)] >> (tj & 31)) & 1u;
    cnt[t] = c;
  }
}

// Writes each (group, column tile)'s survivors at its offset; the list length
// (off[ng * nTS]) goes to *ntiles.
__global__ void group_list_kernel(const uint32_t* __restrict__ surv, int64_t sw, int64_t nTR, int64_t nTS, int64_t gm,
                                  const uint32_t* __restrict__ off, uint2* __restrict__ tiles,
                                  unsigned long long* __restrict__ ntiles) {
  const int64_t ng = (nTR + gm - 1) / gm;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= ng * nTS;
       t += (int64_t)gridDim.x * blockDim.x) {
    if (t == ng * nTS) {
      *ntiles = off[t];
      continue;
    }
    const int64_t g = t / nTS, tj = t - g * nTS;
    const int64_t t1 = min(nTR, (g + 1) * gm);
    uint32_t at = off[t];
    for (int64_t ti = g * gm; ti < t1; ++ti)
      if ((surv[ti * sw + (tj >> 5)] >> (tj & 31)) & 1u) tiles[at++] = make_uint2((uint32_t)ti, (uint32_t)tj);
  }
}

hipError_t launch_gather_rows(const float* X, int64_t ld, int64_t stride, int64_t m, int d, float* out,
                              hipStream_t st, int cu) {
  if (m == 0) return hipSuccess;
  const int64_t total = m * (int64_t)d;
  int64_t g = (total + 255) / 256;
  if (g > (int64_t)cu * 8) g = (int64_t)cu * 8;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)g), dim3(256), 0, st, X, ld, stride, m, d, out);
  return hipGetLastError();
}

hipError_t launch_pivot_keys(const unsigned long long* argkey, int64_t n, int64_t npiv, int bj,
                             unsigned long long* keys, float* vals, hipStream_t st, int cu) {
  if (n == 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > (int64_t)cu * 8) g = (int64_t)cu * 8;
  hipLaunchKernelGGL(pivot_keys_kernel, dim3((unsigned)g), dim3(256), 0, st, argkey, n, (uint32_t)npiv, bj, keys,
                     vals);
  return hipGetLastError();
}

hipError_t launch_block_balls(const float* X, int64_t ld, const uint32_t* perm, int64_t n, int d, double eps,
                              float* cent, double* Tb, hipStream_t st) {
  const int64_t nb = (n + kTile - 1) / kTile;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(block_ball_kernel, dim3((unsigned)nb), dim3(256), (size_t)d * sizeof(float), st, X, ld, perm, n,
                     d, eps, cent, Tb);
  return hipGetLastError();
}

hipError_t launch_survive(const uint32_t* m1, int64_t m1w, const uint32_t* m2, int64_t m2w, int64_t nTR, int64_t nTS,
                          int self, uint32_t* surv, int64_t sw, hipStream_t st) {
  if (nTR == 0) return hipSuccess;
  hipLaunchKernelGGL(survive_kernel, dim3((unsigned)((nTR + 3) / 4)), dim3(256), 0, st, m1, m1w, m2, m2w, nTR, nTS,
                     self, surv, sw);
  return hipGetLastError();
}

hipError_t launch_group_count(const uint32_t* surv, int64_t sw, int64_t nTR, int64_t nTS, int64_t gm, uint32_t* cnt,
                              hipStream_t st, int cu) {
  const int64_t m = (nTR + gm - 1) / gm * nTS;
  if (m == 0) return hipSuccess;
  int64_t g = (m + 255) / 256;
  if (g > (int64_t)cu * 16) g = (int64_t)cu * 16;
  hipLaunchKernelGGL(group_count_kernel, dim3((unsigned)g), dim3(256), 0, st, surv, sw, nTR, nTS, gm, cnt);
  return hipGetLastError();
}

hipError_t launch_group_list(const uint32_t* surv, int64_t sw, int64_t nTR, int64_t nTS, int64_t gm,
                             const uint32_t* off, uint2* tiles, unsigned long long* ntiles, hipStream_t st, int cu) {
  const int64_t m = (nTR + gm - 1) / gm * nTS + 1;
  int64_t g = (m + 255) / 256;
  if (g > (int64_t)cu * 16) g = (int64_t)cu * 16;
  hipLaunchKernelGGL(group_list_kernel, dim3((unsigned)g), dim3(256), 0, st, surv, sw, nTR, nTS, gm, off, tiles,
                     ntiles);
  return hipGetLastError();
}

}  // namespace dl
