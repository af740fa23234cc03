// index.hip -- kernels of the index-pruned eps-join.
//
// Paper: section "Query Processing" builds an index on the fly inside a join
// query (one relation is indexed, the other probes it), and section "Derived
// Data" answers Euclidean threshold queries with a Ball-tree over the feature
// vectors.  Here the index is one level of balls over 256-row blocks, built
// on the GPU for the matrix-core tiles:
//   1. every row is assigned to its nearest pivot (a strided sample of S),
//      and the rows of each relation are ordered by pivot, so consecutive
//      rows are close and a 256-row block is a tight cluster;
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
//      tile near the R tile's ball); the survivors form a tile list that the
//      candidate pass walks instead of the full grid.
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
// ordering (which is then a stable counting sort by pivot).
__global__ void pivot_keys_kernel(const uint32_t* __restrict__ pivot, int64_t n, uint32_t npiv, int bj,
                                  unsigned long long* __restrict__ keys, float* __restrict__ vals) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t pv = pivot[t] < npiv ? pivot[t] : npiv - 1;  // any pivot is a valid bucket
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
  for (int k = threadIdx.x; k < d; k += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += (double)X[(int64_t)perm[r0 + r] * ld + k];
    const float c = (float)(s / (double)rows);
    c_lds[k] = c;
    cent[b * (int64_t)d + k] = c;
  }
  __syncthreads();
  // one wave per row: lanes over k, a float64 sum per row, the block maximum
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double r2max = 0.0;
  for (int r = wave; r < rows; r += 4) {
    const float* x = X + (int64_t)perm[r0 + r] * ld;
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
// tj >= ti only.  cnt[ti] = survivors of the row tile.
__global__ __launch_bounds__(256) void survive_kernel(const uint32_t* __restrict__ m1, int64_t m1w,
                                                      const uint32_t* __restrict__ m2, int64_t m2w, int64_t nTR,
                                                      int64_t nTS, int self, uint32_t* __restrict__ surv, int64_t sw,
                                                      uint32_t* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t ti = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (ti >= nTR) return;
  uint32_t c = 0;
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
    c += (uint32_t)__popc(keep);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (lane == 0) cnt[ti] = c;
}

// One wave per row tile: its survivors (ti, tj), tj ascending, at off[ti]...
// in the tile list; the list length (off[nTR]) goes to *ntiles.
__global__ __launch_bounds__(256) void tile_list_kernel(const uint32_t* __restrict__ surv, int64_t sw, int64_t nTR,
                                                        const uint32_t* __restrict__ off, uint2* __restrict__ tiles,
                                                        unsigned long long* __restrict__ ntiles) {
  const int lane = threadIdx.x & 63;
  const int64_t ti = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (ti > nTR) return;
  if (ti == nTR) {
    if (lane == 0) *ntiles = off[nTR];
    return;
  }
  uint32_t base = off[ti];
  for (int64_t w0 = 0; w0 < sw; w0 += 64) {
    const int64_t w = w0 + lane;
    uint32_t word = w < sw ? surv[ti * sw + w] : 0u;
    // exclusive prefix of the popcounts across the wave
    const uint32_t pc = (uint32_t)__popc(word);
    uint32_t pre = pc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(pre, o, 64);
      if (lane >= o) pre += y;
    }
    const uint32_t total = __shfl(pre, 63, 64);
    uint32_t at = base + pre - pc;
    while (word) {
      const int bit = __ffs(word) - 1;
      word &= word - 1;
      tiles[at++] = make_uint2((uint32_t)ti, (uint32_t)(w * 32 + bit));
    }
    base += total;
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

hipError_t launch_pivot_keys(const uint32_t* pivot, int64_t n, int64_t npiv, int bj, unsigned long long* keys,
                             float* vals, hipStream_t st, int cu) {
  if (n == 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > (int64_t)cu * 8) g = (int64_t)cu * 8;
  hipLaunchKernelGGL(pivot_keys_kernel, dim3((unsigned)g), dim3(256), 0, st, pivot, n, (uint32_t)npiv, bj, keys,
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
                          int self, uint32_t* surv, int64_t sw, uint32_t* cnt, hipStream_t st) {
  if (nTR == 0) return hipSuccess;
  hipLaunchKernelGGL(survive_kernel, dim3((unsigned)((nTR + 3) / 4)), dim3(256), 0, st, m1, m1w, m2, m2w, nTR, nTS,
                     self, surv, sw, cnt);
  return hipGetLastError();
}

hipError_t launch_tile_list(const uint32_t* surv, int64_t sw, int64_t nTR, const uint32_t* off, uint2* tiles,
                            unsigned long long* ntiles, hipStream_t st) {
  hipLaunchKernelGGL(tile_list_kernel, dim3((unsigned)((nTR + 1 + 3) / 4)), dim3(256), 0, st, surv, sw, nTR, off,
                     tiles, ntiles);
  return hipGetLastError();
}

}  // namespace dl
