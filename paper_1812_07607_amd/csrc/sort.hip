// sort.hip -- canonical (i, j) order for the eps-join output.
//
// Stable least-significant-digit radix sort of 64-bit keys (i << bj | j) with
// a float payload, 8 bits per pass over only the bits the keys use.  Each
// pass: per-tile digit histograms, one exclusive scan over the digit-major
// histogram table, and a stable scatter that ranks equal digits inside a
// tile with wave ballots.  Deterministic: the output depends only on the
// set of keys, not on the order the candidate kernel produced them in.
#include "dl_internal.hpp"

namespace dl {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per tile
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;  // 4096

// --------------------------------------------------------------- scan
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds_w, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds_w[wave] = x;
  __syncthreads();
  const int nw = blockDim.x >> 6;
  uint32_t off = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    const uint32_t s = lds_w[w];
    if (w < wave) off += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return off + x - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t* in, int64_t n, uint32_t* sums) {
  __shared__ uint32_t lw[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t s = 0;
  for (int t = 0; t < kScanItems; ++t) {
    const int64_t idx = base + (int64_t)t * kScanThreads + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  uint32_t tot;
  block_exclusive_scan(s, lw, tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single workgroup: exclusive scan of nb chunk sums in place (nb <= 2^20)
__global__ __launch_bounds__(1024) void scan_top_kernel(uint32_t* sums, int64_t nb) {
  __shared__ uint32_t lw[16];
  uint32_t carry = 0;
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t idx = base + threadIdx.x;
    const uint32_t v = idx < nb ? sums[idx] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, lw, tot);
    if (idx < nb) sums[idx] = carry + ex;
    carry += tot;
    __syncthreads();
  }
}

// each thread owns kScanItems consecutive entries of the chunk
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const uint32_t* in, int64_t n, const uint32_t* sums,
                                                                  uint32_t* out) {
  __shared__ uint32_t lw[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    v[t] = base + t < n ? in[base + t] : 0u;
    s += v[t];
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan(s, lw, tot) + sums[blockIdx.x];
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    if (base + t < n) out[base + t] = run;
    run += v[t];
  }
}

int64_t scan_scratch_words(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* sums, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, sums);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, st, sums, nb);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, sums, out);
  return hipGetLastError();
}

// --------------------------------------------------------------- radix
// hist layout: digit-major, hist[digit * ntiles + tile]
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const unsigned long long* keys, int64_t n, int shift,
                                                                  uint32_t* hist, int64_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int t = 0; t < kSortItems; ++t) {
    const int64_t idx = base + (int64_t)t * kSortThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(const unsigned long long* kin, const float* vin,
                                                                     int64_t n, int shift, const uint32_t* offs,
                                                                     int64_t ntiles, unsigned long long* kout,
                                                                     float* vout) {
  __shared__ uint32_t run[256];           // keys of each digit already placed by this tile
  __shared__ uint32_t wcnt[kSortThreads / 64][256];
  const int wave = threadIdx.x >> 6;
  run[threadIdx.x] = 0;
  for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt = __lanemask_lt();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int t = 0; t < kSortItems; ++t) {
    // keys of this round are in index order wave-major, lane-minor
    const int64_t idx = base + (int64_t)t * kSortThreads + threadIdx.x;
    const bool valid = idx < n;
    unsigned long long key = 0;
    float val = 0.0f;
    uint32_t dig = 0;
    if (valid) {
      key = kin[idx];
      val = vin[idx];
      dig = (uint32_t)(key >> shift) & 255u;
    }
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((dig >> b) & 1u);
      peers &= ((dig >> b) & 1u) ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt);
    const bool leader = valid && rank == 0;
    if (leader) wcnt[wave][dig] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[dig] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][dig];
      const uint64_t gp = offs[(int64_t)dig * ntiles + blockIdx.x] + pos;
      kout[gp] = key;
      vout[gp] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kSortThreads / 64; ++w) {
      add += wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = 0;
    }
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

__global__ void unpack_pairs_kernel(const unsigned long long* keys, const float* vals, int64_t m, int bj, uint32_t* oi,
                                    uint32_t* oj, float* od) {
  const unsigned long long mask = (1ull << bj) - 1;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = keys[t];
    oi[t] = (uint32_t)(k >> bj);
    oj[t] = (uint32_t)(k & mask);
    od[t] = vals[t];
  }
}

int64_t radix_hist_words(int64_t n) { return 256 * ((n + kSortTile - 1) / kSortTile); }

// Sorts (k0, v0) of n entries by the low `bits` key bits.  Uses (k1, v1) as
// the other buffer; returns which buffer holds the result (0 or 1).
int radix_sort_pairs(unsigned long long* k0, float* v0, unsigned long long* k1, float* v1, int64_t n, int bits,
                     uint32_t* hist, uint32_t* scan_sums, hipStream_t st, hipError_t* err) {
  *err = hipSuccess;
  if (n <= 1) return 0;
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  int cur = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    unsigned long long* ki = cur ? k1 : k0;
    float* vi = cur ? v1 : v0;
    unsigned long long* ko = cur ? k0 : k1;
    float* vo = cur ? v0 : v1;
    hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, ki, n, shift, hist, ntiles);
    hipError_t e = launch_exclusive_scan(hist, 256 * ntiles, hist, scan_sums, st);
    if (e != hipSuccess) { *err = e; return cur; }
    hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, ki, vi, n, shift, hist,
                       ntiles, ko, vo);
    cur ^= 1;
  }
  *err = hipGetLastError();
  return cur;
}

hipError_t launch_unpack_pairs(const unsigned long long* keys, const float* vals, int64_t m, int bj, uint32_t* oi,
                               uint32_t* oj, float* od, hipStream_t st, int cu_count) {
  if (m == 0) return hipSuccess;
  int64_t blocks = (m + 255) / 256;
  if (blocks > (int64_t)cu_count * 8) blocks = (int64_t)cu_count * 8;
  hipLaunchKernelGGL(unpack_pairs_kernel, dim3((unsigned)blocks), dim3(256), 0, st, keys, vals, m, bj, oi, oj, od);
  return hipGetLastError();
}

}  // namespace dl
