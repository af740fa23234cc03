// plan.hip -- the relational operators around a join that let a query put a
// metadata filter before or after the match.
//
// Paper: section "Query Processing" (operators over patch collections, the
// query optimiser's choice of plan) and its plan-order experiment (a filter
// on a patch label before the match, or the match first and the filter on
// its output pairs).  Both plans give the same pairs for an exact filter;
// they differ in how many pairs the match compares.
//   select  rows of a relation whose label equals a value, in row order;
//   gather  those rows into a dense matrix;
//   remap   (i, j) of a join over gathered rows back to the original rows
//           (the maps are increasing, so (i, j) order is kept);
//   filter  a join's (i, j, dist) output to pairs whose two labels equal the
//           value, in order.
// Order-preserving compaction: per-block counts, an exclusive scan, then
// each block writes its kept items at its offset in thread order.
#include "dl_internal.hpp"

namespace dl {

hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* sums, hipStream_t st);
int64_t scan_scratch_words(int64_t n);

constexpr int kPlanThreads = 256;
constexpr int kPlanItems = 8;                            // items per thread
constexpr int64_t kPlanChunk = kPlanThreads * kPlanItems;  // items per block

__device__ inline uint32_t block_exclusive(uint32_t v, uint32_t* lw, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lw[wave] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int w = 0; w < kPlanThreads / 64; ++w) {
    if (w < wave) off += lw[w];
    tot += lw[w];
  }
  __syncthreads();
  total = tot;
  return off + x - v;
}

// keep(t): whether item t is kept.  Pass 1 counts per block.
template <class Keep>
__device__ inline void count_pass(int64_t n, uint32_t* cnt, Keep keep) {
  __shared__ uint32_t lw[kPlanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kPlanChunk + (int64_t)threadIdx.x * kPlanItems;
  uint32_t c = 0;
#pragma unroll
  for (int u = 0; u < kPlanItems; ++u) c += base + u < n && keep(base + u) ? 1u : 0u;
  uint32_t tot;
  block_exclusive(c, lw, tot);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

// Pass 2 writes each kept item (emit(t, position)) in order.
template <class Keep, class Emit>
__device__ inline void write_pass(int64_t n, const uint32_t* off, Keep keep, Emit emit) {
  __shared__ uint32_t lw[kPlanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kPlanChunk + (int64_t)threadIdx.x * kPlanItems;
  bool k[kPlanItems];
  uint32_t c = 0;
#pragma unroll
  for (int u = 0; u < kPlanItems; ++u) {
    k[u] = base + u < n && keep(base + u);
    c += k[u] ? 1u : 0u;
  }
  uint32_t tot;
  uint32_t at = off[blockIdx.x] + block_exclusive(c, lw, tot);
#pragma unroll
  for (int u = 0; u < kPlanItems; ++u)
    if (k[u]) emit(base + u, at++);
}

__global__ __launch_bounds__(kPlanThreads) void select_count_kernel(const int32_t* __restrict__ labels, int64_t n,
                                                                    int32_t want, uint32_t* __restrict__ cnt) {
  count_pass(n, cnt, [&](int64_t t) { return labels[t] == want; });
}
__global__ __launch_bounds__(kPlanThreads) void select_write_kernel(const int32_t* __restrict__ labels, int64_t n,
                                                                    int32_t want, const uint32_t* __restrict__ off,
                                                                    uint32_t* __restrict__ rows) {
  write_pass(n, off, [&](int64_t t) { return labels[t] == want; },
             [&](int64_t t, uint32_t at) { rows[at] = (uint32_t)t; });
}

__global__ __launch_bounds__(kPlanThreads) void pairs_count_kernel(const uint32_t* __restrict__ pi,
                                                                   const uint32_t* __restrict__ pj, int64_t m,
                                                                   const int32_t* __restrict__ lr,
                                                                   const int32_t* __restrict__ ls, int32_t want,
                                                                   uint32_t* __restrict__ cnt) {
  count_pass(m, cnt, [&](int64_t t) { return lr[pi[t]] == want && ls[pj[t]] == want; });
}
__global__ __launch_bounds__(kPlanThreads) void pairs_write_kernel(const uint32_t* __restrict__ pi,
                                                                   const uint32_t* __restrict__ pj,
                                                                   const float* __restrict__ pd, int64_t m,
                                                                   const int32_t* __restrict__ lr,
                                                                   const int32_t* __restrict__ ls, int32_t want,
                                                                   const uint32_t* __restrict__ off,
                                                                   uint32_t* __restrict__ oi, uint32_t* __restrict__ oj,
                                                                   float* __restrict__ od, int64_t cap) {
  write_pass(m, off, [&](int64_t t) { return lr[pi[t]] == want && ls[pj[t]] == want; },
             [&](int64_t t, uint32_t at) {
               if ((int64_t)at < cap) {
                 oi[at] = pi[t];
                 oj[at] = pj[t];
                 od[at] = pd[t];
               }
             });
}

// rows[r] of X into out (m x d dense); one wave per row.
__global__ __launch_bounds__(256) void gather_kernel(const float* __restrict__ X, int64_t ld, int d,
                                                     const uint32_t* __restrict__ rows, int64_t m,
                                                     float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < m;
       r += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    const float* x = X + (int64_t)rows[r] * ld;
    for (int k = lane; k < d; k += 64) out[r * d + k] = x[k];
  }
}

__global__ void remap_kernel(uint32_t* __restrict__ pi, uint32_t* __restrict__ pj, int64_t m,
                             const uint32_t* __restrict__ rr, const uint32_t* __restrict__ rs) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    pi[t] = rr[pi[t]];
    pj[t] = rs[pj[t]];
  }
}

__global__ void total_kernel(uint32_t* __restrict__ cnt, const uint32_t* __restrict__ off, int64_t nb,
                             unsigned long long* __restrict__ count, int zero) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (zero) cnt[nb] = 0;  // the scan's extra entry
    else *count = off[nb];
  }
}

int64_t plan_scratch_words(int64_t n) {
  const int64_t nb = (n + kPlanChunk - 1) / kPlanChunk;
  return 2 * (nb + 1) + scan_scratch_words(nb + 1) + 1;
}

// scratch: plan_scratch_words(n) words; *count (device) receives the number
// of rows kept.
hipError_t launch_select_rows(const int32_t* labels, int64_t n, int32_t want, uint32_t* rows, uint32_t* scratch,
                              unsigned long long* count, hipStream_t st) {
  const int64_t nb = (n + kPlanChunk - 1) / kPlanChunk;
  uint32_t* cnt = scratch;
  uint32_t* off = scratch + (nb + 1);
  uint32_t* sums = scratch + 2 * (nb + 1);
  hipLaunchKernelGGL(total_kernel, dim3(1), dim3(64), 0, st, cnt, off, nb, count, 1);
  if (nb > 0)
    hipLaunchKernelGGL(select_count_kernel, dim3((unsigned)nb), dim3(kPlanThreads), 0, st, labels, n, want, cnt);
  hipError_t e = launch_exclusive_scan(cnt, nb + 1, off, sums, st);
  if (e != hipSuccess) return e;
  if (nb > 0)
    hipLaunchKernelGGL(select_write_kernel, dim3((unsigned)nb), dim3(kPlanThreads), 0, st, labels, n, want, off,
                       rows);
  hipLaunchKernelGGL(total_kernel, dim3(1), dim3(64), 0, st, cnt, off, nb, count, 0);
  return hipGetLastError();
}

// Kept pairs past cap are counted, not written (out-of-place: the output
// arrays must not overlap the input).
hipError_t launch_filter_pairs(const uint32_t* pi, const uint32_t* pj, const float* pd, int64_t m, const int32_t* lr,
                               const int32_t* ls, int32_t want, uint32_t* oi, uint32_t* oj, float* od, int64_t cap,
                               uint32_t* scratch, unsigned long long* count, hipStream_t st) {
  const int64_t nb = (m + kPlanChunk - 1) / kPlanChunk;
  uint32_t* cnt = scratch;
  uint32_t* off = scratch + (nb + 1);
  uint32_t* sums = scratch + 2 * (nb + 1);
  hipLaunchKernelGGL(total_kernel, dim3(1), dim3(64), 0, st, cnt, off, nb, count, 1);
  if (nb > 0)
    hipLaunchKernelGGL(pairs_count_kernel, dim3((unsigned)nb), dim3(kPlanThreads), 0, st, pi, pj, m, lr, ls, want,
                       cnt);
  hipError_t e = launch_exclusive_scan(cnt, nb + 1, off, sums, st);
  if (e != hipSuccess) return e;
  if (nb > 0)
    hipLaunchKernelGGL(pairs_write_kernel, dim3((unsigned)nb), dim3(kPlanThreads), 0, st, pi, pj, pd, m, lr, ls,
                       want, off, oi, oj, od, cap);
  hipLaunchKernelGGL(total_kernel, dim3(1), dim3(64), 0, st, cnt, off, nb, count, 0);
  return hipGetLastError();
}

hipError_t launch_gather(const float* X, int64_t ld, int d, const uint32_t* rows, int64_t m, float* out,
                         hipStream_t st, int cu) {
  if (m == 0) return hipSuccess;
  int64_t g = (m + 3) / 4;
  if (g > (int64_t)cu * 16) g = (int64_t)cu * 16;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)g), dim3(256), 0, st, X, ld, d, rows, m, out);
  return hipGetLastError();
}

hipError_t launch_remap(uint32_t* pi, uint32_t* pj, int64_t m, const uint32_t* rr, const uint32_t* rs, hipStream_t st,
                        int cu) {
  if (m == 0) return hipSuccess;
  int64_t g = (m + 255) / 256;
  if (g > (int64_t)cu * 8) g = (int64_t)cu * 8;
  hipLaunchKernelGGL(remap_kernel, dim3((unsigned)g), dim3(256), 0, st, pi, pj, m, rr, rs);
  return hipGetLastError();
}

}  // namespace dl
