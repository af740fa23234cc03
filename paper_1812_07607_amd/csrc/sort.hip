// sort.hip -- canonical (i, j) order for the eps-join output.
//
// The confirmed pairs (keys i << bj | j with a float distance) are bucketed
// by row with a count, an exclusive scan and an atomic placement, then each
// row's segment is ordered by j.  Deterministic: the output depends only on
// the set of pairs, not on the order the candidate kernel produced them in.
#include "dl_internal.hpp"

namespace dl {

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

// --------------------------------------------------------------- rows
// Canonical (i, j) order by rows: count the pairs of each row, scan the
// counts into row offsets, place every pair in its row's segment (in any
// order), then order each segment by j, one wave per row.  A pair's output
// slot is the number of the row's pairs with a smaller j (the (i, j) pairs
// are distinct, so the result does not depend on the order of placement):
// rows of at most 64 pairs rank in registers, rows of at most 256 against
// their j values staged in LDS; longer rows set one bit per pair in an LDS
// bitmap over a window of j, take a prefix count of the bitmap words, and
// read each pair's rank from it, window by window (windows that hold no
// pair are skipped), so the work is linear in the row length.  Six
// launches where an 8-bit LSD radix sort of 34-bit keys takes 25.
__global__ void fill_words_kernel(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

// The confirmed pairs arrive in runs of equal i (the candidate pass emits
// them tile by tile), so the row counters take one atomic per run of equal
// rows inside a wave rather than one per pair.  For the pair of lane l:
// head = the lane that starts its run, len = the run's length.
struct RowRun {
  uint64_t i;
  int head, len;
  bool valid;
};

__device__ inline RowRun row_run(const unsigned long long* keys, int64_t t, int64_t m, int bj) {
  const int lane = threadIdx.x & 63;
  RowRun r;
  r.valid = t < m;
  r.i = r.valid ? keys[t] >> bj : ~0ull;
  const uint64_t prev = __shfl_up(r.i, 1, 64);
  const bool start = r.valid && (lane == 0 || prev != r.i);
  const uint64_t heads = __ballot(start);
  const uint64_t ends = heads | ~__ballot(r.valid);  // a run also ends at the first lane past m
  r.head = 63 - __clzll(heads & (~0ull >> (63 - lane)));
  const uint64_t after = ends & ~(~0ull >> (63 - r.head));
  r.len = (after ? __ffsll((long long)after) - 1 : 64) - r.head;
  return r;
}

__global__ void count_rows_kernel(const unsigned long long* __restrict__ keys, int64_t m, int bj,
                                  uint32_t* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); t0 < m; t0 += stride) {
    const RowRun r = row_run(keys, t0 + lane, m, bj);
    if (r.valid && r.head == lane) atomicAdd(&cnt[r.i], (uint32_t)r.len);
  }
}

// cnt holds each row's pair count on entry and zero on exit: each run takes
// len of its row's slots by one atomic decrement.
__global__ void place_rows_kernel(const unsigned long long* __restrict__ keys, const float* __restrict__ vals,
                                  int64_t m, int bj, const uint32_t* __restrict__ off, uint32_t* __restrict__ cnt,
                                  unsigned long long* __restrict__ pk, float* __restrict__ pv) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); t0 < m; t0 += stride) {
    const int64_t t = t0 + lane;
    const RowRun r = row_run(keys, t, m, bj);
    uint32_t first = 0;
    if (r.valid && r.head == lane) first = off[r.i] + atomicSub(&cnt[r.i], (uint32_t)r.len) - (uint32_t)r.len;
    first = __shfl(first, r.head, 64);
    if (r.valid) {
      const uint32_t pos = first + (uint32_t)(lane - r.head);
      pk[pos] = keys[t];
      pv[pos] = vals[t];
    }
  }
}

constexpr int kRowWaves = 4;
constexpr int kWinWords = 1024;             // bitmap words per wave
constexpr int kWinBits = 32 * kWinWords;    // j values per window
constexpr int kWordsPerLane = kWinWords / 64;
constexpr int kQuadRow = 256;               // longest row ranked pair against pair

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(64 * kRowWaves) void order_rows_kernel(const unsigned long long* __restrict__ pk,
                                                                   const float* __restrict__ pv, int64_t nR,
                                                                   const uint32_t* __restrict__ off, int64_t m,
                                                                   int bj, int64_t w, uint32_t* __restrict__ oi,
                                                                   uint32_t* __restrict__ oj, float* __restrict__ od) {
  __shared__ uint32_t bits_lds[kRowWaves][kWinWords];
  __shared__ uint32_t pre_lds[kRowWaves][kWinWords];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * kRowWaves + wave;
  if (i >= nR) return;
  const int64_t b = off[i], e = i + 1 < nR ? (int64_t)off[i + 1] : m;
  const unsigned long long mask = (1ull << bj) - 1;
  auto emit = [&](int64_t at, int64_t t, uint32_t j) {
    if (at < w) {
      oi[at] = (uint32_t)i;
      oj[at] = j;
      od[at] = pv[t];
    }
  };
  if (e - b <= 64) {
    const int64_t t = b + lane;
    const uint32_t j = t < e ? (uint32_t)(pk[t] & mask) : 0xffffffffu;
    int rank = 0;
    for (int u = 0; u < (int)(e - b); ++u) rank += __shfl(j, u, 64) < j;
    if (t < e) emit(b + rank, t, j);
    return;
  }
  uint32_t* bm = bits_lds[wave];
  if (e - b <= kQuadRow) {
    // rank against the row's j values staged in LDS (broadcast reads)
    for (int64_t t = b + lane; t < e; t += 64) bm[t - b] = (uint32_t)(pk[t] & mask);
    wave_lds_sync();
    const int len = (int)(e - b);
    uint32_t jq[kQuadRow / 64];
    int rk[kQuadRow / 64];
#pragma unroll
    for (int q = 0; q < kQuadRow / 64; ++q) {
      jq[q] = lane + 64 * q < len ? bm[lane + 64 * q] : 0u;
      rk[q] = 0;
    }
    for (int u = 0; u < len; ++u) {
      const uint32_t v = bm[u];
#pragma unroll
      for (int q = 0; q < kQuadRow / 64; ++q) rk[q] += v < jq[q];
    }
#pragma unroll
    for (int q = 0; q < kQuadRow / 64; ++q)
      if (lane + 64 * q < len) emit(b + rk[q], b + lane + 64 * q, jq[q]);
    return;
  }
  uint32_t* pre = pre_lds[wave];
  uint32_t jlo = 0xffffffffu, jhi = 0;
  for (int64_t t = b + lane; t < e; t += 64) {
    const uint32_t j = (uint32_t)(pk[t] & mask);
    jlo = j < jlo ? j : jlo;
    jhi = j > jhi ? j : jhi;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t a = __shfl_xor(jlo, o, 64), z = __shfl_xor(jhi, o, 64);
    jlo = a < jlo ? a : jlo;
    jhi = z > jhi ? z : jhi;
  }
  int64_t below = 0;  // pairs of the row in earlier windows
  uint64_t lo = jlo;
  while (lo <= jhi) {
#pragma unroll
    for (int q = 0; q < kWordsPerLane; ++q) bm[lane * kWordsPerLane + q] = 0;
    wave_lds_sync();
    for (int64_t t = b + lane; t < e; t += 64) {
      const uint64_t r = (pk[t] & mask) - lo;
      if (r < (uint64_t)kWinBits) atomicOr(&bm[r >> 5], 1u << (r & 31));
    }
    wave_lds_sync();
    uint32_t c[kWordsPerLane], run = 0;
#pragma unroll
    for (int q = 0; q < kWordsPerLane; ++q) {
      c[q] = run;
      run += __popc(bm[lane * kWordsPerLane + q]);
    }
    uint32_t x = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    const uint32_t base = x - run, total = __shfl(x, 63, 64);
#pragma unroll
    for (int q = 0; q < kWordsPerLane; ++q) pre[lane * kWordsPerLane + q] = base + c[q];
    wave_lds_sync();
    uint32_t nxt = 0xffffffffu;  // smallest j past this window: the next window starts there
    for (int64_t t = b + lane; t < e; t += 64) {
      const uint64_t j = pk[t] & mask;
      const uint64_t r = j - lo;
      if (r < (uint64_t)kWinBits) {
        const uint32_t wd = (uint32_t)(r >> 5);
        const uint32_t rank = pre[wd] + __popc(bm[wd] & ((1u << (r & 31)) - 1u));
        emit(b + below + rank, t, (uint32_t)j);
      } else if (j > lo && j < nxt) {
        nxt = (uint32_t)j;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const uint32_t a = __shfl_xor(nxt, o, 64);
      nxt = a < nxt ? a : nxt;
    }
    below += total;
    lo = nxt;
    wave_lds_sync();
  }
}

int64_t row_sort_words(int64_t nR) { return 2 * (nR + 1) + scan_scratch_words(nR + 1) + 1; }

// keys/vals: the m confirmed pairs (key i << bj | j); pk/pv: m entries of
// scratch; words: row_sort_words(nR) words of scratch.  Writes the first w
// pairs in (i, j) order to oi/oj/od.
hipError_t row_sort_pairs(const unsigned long long* keys, const float* vals, int64_t m, int64_t nR, int bj,
                          unsigned long long* pk, float* pv, uint32_t* words, int64_t w, uint32_t* oi, uint32_t* oj,
                          float* od, hipStream_t st, int cu_count) {
  if (m == 0 || nR == 0) return hipSuccess;
  uint32_t* cnt = words;
  uint32_t* off = words + (nR + 1);
  uint32_t* sums = words + 2 * (nR + 1);
  const int64_t gw = (nR + 255) / 256 < (int64_t)cu_count * 4 ? (nR + 255) / 256 : (int64_t)cu_count * 4;
  const int64_t gm = (m + 255) / 256 < (int64_t)cu_count * 8 ? (m + 255) / 256 : (int64_t)cu_count * 8;
  hipLaunchKernelGGL(fill_words_kernel, dim3((unsigned)gw), dim3(256), 0, st, cnt, nR, 0u);
  hipLaunchKernelGGL(count_rows_kernel, dim3((unsigned)gm), dim3(256), 0, st, keys, m, bj, cnt);
  hipError_t e = launch_exclusive_scan(cnt, nR, off, sums, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(place_rows_kernel, dim3((unsigned)gm), dim3(256), 0, st, keys, vals, m, bj, off, cnt, pk, pv);
  hipLaunchKernelGGL(order_rows_kernel, dim3((unsigned)((nR + kRowWaves - 1) / kRowWaves)), dim3(64 * kRowWaves), 0,
                     st, pk, pv, nR, off, m, bj, w, oi, oj, od);
  return hipGetLastError();
}

}  // namespace dl
