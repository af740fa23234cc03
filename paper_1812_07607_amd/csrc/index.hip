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

hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* sums, hipStream_t st);
int64_t scan_scratch_words(int64_t n);

// Rows 0, stride, 2 stride, ... (m of them) of X into out (m x d, dense).
__global__ void gather_rows_kernel(const float* __restrict__ X, int64_t ld, int64_t stride, int64_t m, int d,
                                   float* __restrict__ out) {
  const int64_t total = m * (int64_t)d;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / d, k = t - r * d;
    out[t] = X[r * stride * ld + k];
  }
}

// Ordering the rows by nearest pivot: a stable counting sort, one wave per
// chunk of kPivChunk rows.  The pivot of row t comes from the nearest pass's
// key, whose low word is the complement of the winning column; a row no
// pivot won (NaN input) goes to the last pivot.
constexpr int kPivChunk = 2048;

__device__ inline uint32_t pivot_of(unsigned long long key, uint32_t npiv) {
  const uint32_t c = 0xffffffffu - (uint32_t)(key & 0xffffffffull);
  return c < npiv ? c : npiv - 1;
}

// Pass 1: the rows of each pivot in chunk b, at cnt[p * nb + b] (pivot
// major, so an exclusive scan gives each (pivot, chunk) its first slot).
// LDS: npiv words.
__global__ __launch_bounds__(64) void pivot_count_kernel(const unsigned long long* __restrict__ argkey, int64_t n,
                                                         uint32_t npiv, uint32_t* __restrict__ cnt) {
  extern __shared__ uint32_t h[];
  const int64_t nb = gridDim.x, b = blockIdx.x;
  for (uint32_t p = threadIdx.x; p < npiv; p += 64) h[p] = 0;
  __syncthreads();
  const int64_t lo = b * kPivChunk, hi = min(n, lo + kPivChunk);
  uint32_t piv[kPivChunk / 64];  // all the chunk's loads in flight, then the counts
#pragma unroll
  for (int u = 0; u < kPivChunk / 64; ++u) {
    const int64_t t = lo + 64 * u + threadIdx.x;
    piv[u] = t < hi ? pivot_of(argkey[t], npiv) : npiv;
  }
#pragma unroll
  for (int u = 0; u < kPivChunk / 64; ++u)
    if (piv[u] < npiv) atomicAdd(&h[piv[u]], 1u);
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < npiv; p += 64) cnt[(int64_t)p * nb + b] = h[p];
}

// Pass 2: rows in row order, 64 at a time; the lanes holding the same pivot
// find each other with one ballot per pivot bit, take consecutive slots
// from the pivot's cursor in lane order, and the lowest of them advances
// the cursor.  perm[slot] = row, so perm lists the rows by (pivot, row).
// LDS: npiv words.
__global__ __launch_bounds__(64) void pivot_place_kernel(const unsigned long long* __restrict__ argkey, int64_t n,
                                                         uint32_t npiv, int pbits, const uint32_t* __restrict__ off,
                                                         uint32_t* __restrict__ perm) {
  extern __shared__ uint32_t cur[];
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int lane = threadIdx.x;
  for (uint32_t p = lane; p < npiv; p += 64) cur[p] = off[(int64_t)p * nb + b];
  __syncthreads();
  const int64_t lo = b * kPivChunk, hi = min(n, lo + kPivChunk);
  const uint64_t lower = (1ull << lane) - 1;  // lanes below this one
  // the chunk's pivots first (all its loads in flight), then the placement
  uint32_t piv[kPivChunk / 64];
#pragma unroll
  for (int u = 0; u < kPivChunk / 64; ++u) {
    const int64_t t = lo + 64 * u + lane;
    piv[u] = t < hi ? pivot_of(argkey[t], npiv) : 0u;
  }
#pragma unroll
  for (int u = 0; u < kPivChunk / 64; ++u) {
    const int64_t base = lo + 64 * u;
    if (base >= hi) break;
    const int64_t t = base + lane;
    const bool valid = t < hi;
    const uint32_t p = piv[u];
    uint64_t peers = __ballot(valid);
    for (int k = 0; k < pbits; ++k) {
      const bool bit = (p >> k) & 1u;
      const uint64_t on = __ballot(bit);
      peers &= bit ? on : ~on;
    }
    if (valid) {
      const uint32_t slot = cur[p] + (uint32_t)__popcll(peers & lower);
      perm[slot] = (uint32_t)t;
    }
    // every lane has read its cursor before the group's lowest lane moves it
    __builtin_amdgcn_wave_barrier();
    if (valid && (peers & lower) == 0) cur[p] += (uint32_t)__popcll(peers);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Block balls from the ordered operand copy, whose 256 rows of a block are
// contiguous (qld bytes each): the centroid c is the float64 mean of the
// operand values x~ rounded to float32, and r bounds |x - c| from above for
// each row x of the block through |x - c| <= |x~ - c| + |x - x~|, the second
// term being the prep's rounded-up rho of the row; the sums are float64
// (relative error below dpad 2^-53) and r and Tb are rounded up by 2^-30
// relative.  Reads the 2 to 8 times smaller operand
// copy sequentially instead of float32 rows scattered by the permutation.
template <int kPrec>
__device__ inline float op_elem(const uint8_t* row, int k, float scale) {
  if constexpr (kPrec == DL_FP32) return reinterpret_cast<const float*>(row)[k];
  else if constexpr (kPrec == DL_BF16) return dec_bf16(reinterpret_cast<const uint16_t*>(row)[k]);
  else if constexpr (kPrec == DL_FP16) return dec_f16(reinterpret_cast<const uint16_t*>(row)[k]);
  else return dec_e4m3(row[k]) * scale;
}

template <int kPrec>
__global__ __launch_bounds__(256) void block_ball_q_kernel(const uint8_t* __restrict__ q, int64_t qld,
                                                           const int* __restrict__ sexp,
                                                           const float* __restrict__ rho, int64_t n, int d,
                                                           double eps, const float* __restrict__ eps_row,
                                                           float* __restrict__ cent, double* __restrict__ Tb) {
  constexpr int kElem = kPrec == DL_FP32 ? 4 : kPrec == DL_FP8 ? 1 : 2;  // bytes per value
  constexpr int kPer = 16 / kElem;                                       // values per 16-byte piece
  extern __shared__ float c_lds[];  // qld / kElem floats: the centroid, zero past d
  __shared__ double r_wave[4];
  __shared__ float e_wave[4];
  __shared__ float scale_lds[kTile];
  const int64_t b = blockIdx.x;
  const int64_t r0 = b * kTile;
  const int rows = (int)min((int64_t)kTile, n - r0);
  const int dpad = (int)(qld / kElem);
  const uint8_t* base = q + r0 * qld;
  for (int r = threadIdx.x; r < rows; r += blockDim.x)
    scale_lds[r] = kPrec == DL_FP8 ? ldexpf(1.0f, sexp[r0 + r]) : 1.0f;
  __syncthreads();
  // the mean: one value column per thread, eight rows' loads in flight
  for (int k = threadIdx.x; k < dpad; k += blockDim.x) {
    double s = 0.0;
    int r = 0;
    for (; r + 8 <= rows; r += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = op_elem<kPrec>(base + (int64_t)(r + u) * qld, k, scale_lds[r + u]);
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; r < rows; ++r) s += (double)op_elem<kPrec>(base + (int64_t)r * qld, k, scale_lds[r]);
    const float c = k < d ? (float)(s / (double)rows) : 0.0f;
    if (k < d) cent[b * (int64_t)d + k] = c;
    c_lds[k] = c;
  }
  __syncthreads();
  // |x~ - c| + rho per row: a wave takes four rows at a time (four loads in
  // flight per lane), 16-byte pieces across the lanes; rows past the block
  // repeat its last row
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int pieces = (int)(qld / 16);
  constexpr int kRows = 4;
  double rmax = 0.0;
  for (int r = wave; r < rows; r += 4 * kRows) {
    int rq[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) rq[u] = min(r + 4 * u, rows - 1);
    double s[kRows] = {0.0, 0.0, 0.0, 0.0};
    for (int pc = lane; pc < pieces; pc += 64) {
      uint4 w[kRows];
#pragma unroll
      for (int u = 0; u < kRows; ++u) w[u] = *reinterpret_cast<const uint4*>(base + (int64_t)rq[u] * qld + (int64_t)pc * 16);
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        const uint8_t* wb = reinterpret_cast<const uint8_t*>(&w[u]);
        const float sc = scale_lds[rq[u]];
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
          const double t = (double)op_elem<kPrec>(wb, e, sc) - (double)c_lds[pc * kPer + e];
          s[u] += t * t;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      double t = s[u];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
      rmax = fmax(rmax, sqrt(t) + (double)rho[r0 + rq[u]]);
    }
  }
  // per-row eps (eps_row, the top-k bound of each row): the block's largest
  float emax = 0.0f;
  if (eps_row)
    for (int r = threadIdx.x; r < rows; r += blockDim.x) emax = fmaxf(emax, eps_row[r0 + r]);
  for (int o = 32; o > 0; o >>= 1) emax = fmaxf(emax, __shfl_xor(emax, o, 64));
  if (lane == 0) {
    r_wave[wave] = rmax;
    e_wave[wave] = emax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(r_wave[0], r_wave[1]), fmax(r_wave[2], r_wave[3]));
    const double rr = m * (1.0 + 0x1p-30) + 0x1p-100;
    const double eb = eps_row ? (double)fmaxf(fmaxf(e_wave[0], e_wave[1]), fmaxf(e_wave[2], e_wave[3])) : eps;
    const double e = eb + rr;
    Tb[b] = e * e * (1.0 + 0x1p-30);  // +inf when a row has no bound
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
    uint32_t word = m1 ? m1[ti * m1w + w] : 0xffffffffu;  // no m1: that direction marks every tile
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

// K-step masks of one operand copy (rows of qld bytes, zero-padded to whole
// tiles): bit s of mask[t] is set when some row of tile t has a nonzero byte
// in bytes [s * kChunkBytes, (s + 1) * kChunkBytes) of its row, i.e. in the
// candidate pass's K-step s.  A negative zero counts as nonzero, which only
// keeps a step.  One workgroup per tile; qld / kChunkBytes <= 64.
__global__ __launch_bounds__(256) void tile_kmask_kernel(const uint8_t* __restrict__ q, int64_t qld,
                                                         uint64_t* __restrict__ mask) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  __shared__ uint32_t part[2][4];
  const u32x4* base = reinterpret_cast<const u32x4*>(q + (int64_t)blockIdx.x * kTile * qld);
  const uint32_t per_row = (uint32_t)(qld / 16), pieces = (uint32_t)kTile * per_row;
  uint64_t m = 0;
  constexpr int kUnroll = 8;  // loads in flight per thread
  uint32_t t = threadIdx.x;
  for (; t + (kUnroll - 1) * 256 < pieces; t += kUnroll * 256) {
    u32x4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(base + t + u * 256);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (v[u].x | v[u].y | v[u].z | v[u].w) m |= 1ull << (((t + u * 256) % per_row) / (kChunkBytes / 16));
  }
  for (; t < pieces; t += 256) {
    const u32x4 v = __builtin_nontemporal_load(base + t);
    if (v.x | v.y | v.z | v.w) m |= 1ull << ((t % per_row) / (kChunkBytes / 16));
  }
  uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo |= __shfl_xor(lo, o, 64);
    hi |= __shfl_xor(hi, o, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][wave] = lo;
    part[1][wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    mask[blockIdx.x] = (uint64_t)(part[0][0] | part[0][1] | part[0][2] | part[0][3]) |
                       ((uint64_t)(part[1][0] | part[1][1] | part[1][2] | part[1][3]) << 32);
}

// The K-steps the candidate pass runs with the masks: the sum over the tile
// list (or over the grid, a self-join's upper triangle, when 2 * *ntiles >=
// list_all, as the candidate pass decides) of popcount(maskA[ti] &
// maskB[tj]), at least 1 per tile, added to *out.
__global__ __launch_bounds__(256) void kstep_count_kernel(const uint2* __restrict__ tiles,
                                                          const unsigned long long* __restrict__ ntiles,
                                                          int64_t list_all, int64_t nTR, int64_t nTS, int self,
                                                          const uint64_t* __restrict__ ma,
                                                          const uint64_t* __restrict__ mb,
                                                          unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[4];
  const int64_t nl = (int64_t)*ntiles;
  const bool list = 2 * nl < list_all;
  const int64_t n = list ? nl : nTR * nTS;
  unsigned long long c = 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t ti, tj;
    if (list) {
      ti = tiles[t].x;
      tj = tiles[t].y;
    } else {
      ti = t / nTS;
      tj = t - ti * nTS;
      if (self && tj < ti) continue;
    }
    const uint64_t m = ma[ti] & mb[tj];
    c += m ? __popcll(m) : 1;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

hipError_t launch_tile_kmask(const void* q, int64_t qld, int64_t ntiles, uint64_t* mask, hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(tile_kmask_kernel, dim3((unsigned)ntiles), dim3(256), 0, st, static_cast<const uint8_t*>(q), qld,
                     mask);
  return hipGetLastError();
}

// *out must be zero beforehand.
hipError_t launch_kstep_count(const uint2* tiles, const unsigned long long* ntiles, int64_t list_all, int64_t nTR,
                              int64_t nTS, int self, const uint64_t* ma, const uint64_t* mb, unsigned long long* out,
                              hipStream_t st, int cu) {
  const int64_t n = nTR * nTS;  // at least the list's length
  int64_t g = (n + 255) / 256;
  if (g > (int64_t)cu * 4) g = (int64_t)cu * 4;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(kstep_count_kernel, dim3((unsigned)g), dim3(256), 0, st, tiles, ntiles, list_all, nTR, nTS, self,
                     ma, mb, out);
  return hipGetLastError();
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

int64_t pivot_sort_words(int64_t n, int64_t npiv) {
  const int64_t m = (n + kPivChunk - 1) / kPivChunk * npiv;
  return 2 * m + scan_scratch_words(m) + 1;
}

// perm[q] = the q-th row of X in (nearest pivot, row) order.  scratch:
// pivot_sort_words(n, npiv) words; npiv <= 4096.
hipError_t launch_pivot_sort(const unsigned long long* argkey, int64_t n, int64_t npiv, uint32_t* perm,
                             uint32_t* scratch, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t nb = (n + kPivChunk - 1) / kPivChunk, m = nb * npiv;
  uint32_t* cnt = scratch;
  uint32_t* off = scratch + m;
  uint32_t* sums = scratch + 2 * m;
  int pbits = 0;
  while ((1ll << pbits) < npiv) ++pbits;
  const size_t lds = (size_t)npiv * sizeof(uint32_t);
  hipLaunchKernelGGL(pivot_count_kernel, dim3((unsigned)nb), dim3(64), lds, st, argkey, n, (uint32_t)npiv, cnt);
  hipError_t e = launch_exclusive_scan(cnt, m, off, sums, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pivot_place_kernel, dim3((unsigned)nb), dim3(64), lds, st, argkey, n, (uint32_t)npiv, pbits, off,
                     perm);
  return hipGetLastError();
}

// Balls of the blocks of an ordered operand copy P (n real rows).
hipError_t launch_block_balls_q(const Prep& P, int64_t n, int d, dl_prec prec, double eps, float* cent, double* Tb,
                                hipStream_t st, const float* eps_row) {
  const int64_t nb = (n + kTile - 1) / kTile;
  if (nb == 0) return hipSuccess;
  const int elem = prec == DL_FP32 ? 4 : prec == DL_FP8 ? 1 : 2;
  const size_t lds = (size_t)(P.qld / elem) * sizeof(float);
  const uint8_t* q = static_cast<const uint8_t*>(P.q);
  switch (prec) {
    case DL_FP32:
      hipLaunchKernelGGL(block_ball_q_kernel<DL_FP32>, dim3((unsigned)nb), dim3(256), lds, st, q, P.qld, P.sexp, P.rho,
                         n, d, eps, eps_row, cent, Tb);
      break;
    case DL_BF16:
      hipLaunchKernelGGL(block_ball_q_kernel<DL_BF16>, dim3((unsigned)nb), dim3(256), lds, st, q, P.qld, P.sexp, P.rho,
                         n, d, eps, eps_row, cent, Tb);
      break;
    case DL_FP16:
      hipLaunchKernelGGL(block_ball_q_kernel<DL_FP16>, dim3((unsigned)nb), dim3(256), lds, st, q, P.qld, P.sexp, P.rho,
                         n, d, eps, eps_row, cent, Tb);
      break;
    case DL_FP8:
      hipLaunchKernelGGL(block_ball_q_kernel<DL_FP8>, dim3((unsigned)nb), dim3(256), lds, st, q, P.qld, P.sexp, P.rho,
                         n, d, eps, eps_row, cent, Tb);
      break;
  }
  return hipGetLastError();
}

// The top-k join's per-row bound in the index's row order: bound[q] =
// dist[perm[q] * k + k - 1], the k-th distance of row perm[q] against a
// sample of S (+inf when the sample held fewer than k rows).
__global__ void take_bound_kernel(const float* __restrict__ dist, int k, const uint32_t* __restrict__ perm, int64_t n,
                                  float* __restrict__ bound) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    bound[q] = dist[(int64_t)perm[q] * k + k - 1];
}

// Rows of k results from the index's row order back to R's: row q goes to
// row perm[q].
__global__ void scatter_rows_kernel(const uint32_t* __restrict__ j_in, const float* __restrict__ d_in, int k,
                                    const uint32_t* __restrict__ perm, int64_t n, uint32_t* __restrict__ j_out,
                                    float* __restrict__ d_out) {
  const int64_t total = n * k;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = t / k, c = t - q * k;
    const int64_t o = (int64_t)perm[q] * k + c;
    j_out[o] = j_in[t];
    d_out[o] = d_in[t];
  }
}

hipError_t launch_take_bound(const float* dist, int k, const uint32_t* perm, int64_t n, float* bound, hipStream_t st,
                             int cu) {
  if (n == 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > (int64_t)cu * 8) g = (int64_t)cu * 8;
  hipLaunchKernelGGL(take_bound_kernel, dim3((unsigned)g), dim3(256), 0, st, dist, k, perm, n, bound);
  return hipGetLastError();
}

hipError_t launch_scatter_rows(const uint32_t* j_in, const float* d_in, int k, const uint32_t* perm, int64_t n,
                               uint32_t* j_out, float* d_out, hipStream_t st, int cu) {
  if (n == 0) return hipSuccess;
  int64_t g = (n * k + 255) / 256;
  if (g > (int64_t)cu * 8) g = (int64_t)cu * 8;
  hipLaunchKernelGGL(scatter_rows_kernel, dim3((unsigned)g), dim3(256), 0, st, j_in, d_in, k, perm, n, j_out, d_out);
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
