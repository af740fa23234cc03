// recheck.hip -- exact decisions for the candidates of the matrix-core pass.
//
// Every candidate pair gets d2_32 = sum_k (a_k - b_k)^2 in float32 (direct
// form, from the float32 rows).  Its distance to the canonical float64 value
// d2_64 is at most beta = 2 gamma_{d+2} d2_32 + (d+2) 2^-148 +
// (d+4) 2^-52 (|a| + |b|)^2, and beta = 0 when both rows lie on a binary grid
// fine enough that every operation is exact (lowest-set-bit certificate).
//   eps-join: in if d2_32 + beta <= T, out if d2_32 - beta > T, otherwise a
//             boundary tie, decided by d2_64 <= T in float64.
//   top-k:    entries whose [d2_32 - beta, d2_32 + beta] overlaps another
//             contender's interval are ordered by d2_64; the rest are ordered
//             by d2_32, which cannot disagree with d2_64 for them.
// d2_64 is the canonical definition (subtract, square, add in increasing k,
// each rounded separately), so every decision equals the float64 reference.
//
// Paper: Nested Loop Join semantics (section "Query Processing") with the
// Euclidean threshold predicate (section "Derived Data") and the closest-image
// query q1 (section "Queries").
#include "join_params.hpp"

namespace dl {

__device__ inline float wave_sumf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline int wave_sumi(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Direct-form bound and exactness certificate (see file comment).
__device__ inline bool exact32(int mlsb, double xsum) {
  // x rows on the grid 2^m: differences are multiples of 2^m below
  // 2^(m+12) <= 2^(m+24) and squares / sums multiples of 2^(2m) below
  // 2^(2m+24): all exact in float32 while 2m >= -126 (no subnormals).
  if (mlsb >= kLsbNone) return true;  // both rows zero
  return 2 * mlsb >= -126 && xsum * xsum <= ldexp(1.0, 2 * mlsb + 24);
}
__device__ inline double beta32(double d2, int d, double xsum) {
  return 2.0 * gamma_n((double)d + 2.0, 0x1p-24) * d2 + ((double)d + 2.0) * 0x1p-148 +
         ((double)d + 4.0) * 0x1p-52 * xsum * xsum;
}

// ------------------------------------------------------------ eps recheck


// A wave takes 64 candidates at a time: it computes their float32 distances
// one after the other with all lanes (coalesced row reads), lane t keeping
// candidate t's sum, then classifies the 64 lane-parallel and appends the
// confirmed ones with a single atomic.
__global__ __launch_bounds__(256) void recheck_eps_kernel(RecheckParams p) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t n = min((int64_t)*p.ccount, p.ccap);
  const uint64_t lt = __lanemask_lt();
  for (int64_t base = gw * 64; base < n; base += nw * 64) {
    const int cnt = (int)min((int64_t)64, n - base);
    const uint2 mine = lane < cnt ? p.cand[base + lane] : make_uint2(0, 0);
    float mys = 0.0f;
    for (int t = 0; t < cnt; ++t) {
      const uint32_t ci = __shfl(mine.x, t, 64), cj = __shfl(mine.y, t, 64);
      const float* a = p.R + (int64_t)ci * p.ldr;
      const float* b = p.S + (int64_t)cj * p.lds;
      float s = 0.0f;
      for (int k = lane; k < p.d; k += 64) {
        const float u = a[k] - b[k];
        s = fmaf(u, u, s);
      }
      s = wave_sumf(s);
      if (lane == t) mys = s;
    }
    bool in = false, tie = false;
    float dist = 0.0f;
    if (lane < cnt) {
      const double d2 = mys;
      const double xsum = (double)p.xnR[mine.x] + (double)p.xnS[mine.y];
      const bool ex = exact32(min(p.mlR[mine.x], p.mlS[mine.y]), xsum);
      const double bt = ex ? 0.0 : beta32(d2, p.d, xsum);
      const double hi = ex ? d2 : (d2 + bt) * (1.0 + 0x1p-50);
      const double lo = ex ? d2 : (d2 - bt) * (1.0 - 0x1p-50);
      const double T = p.Trow ? p.Trow[mine.x] : p.T;
      in = hi <= T;
      dist = sqrtf(mys);
      if (!in && !(lo > T)) {  // boundary tie: the canonical float64 value decides
        tie = true;
        const double d64 = canonical_d2(p.R + (int64_t)mine.x * p.ldr, p.S + (int64_t)mine.y * p.lds, p.d);
        in = d64 <= T;
        dist = (float)sqrt(d64);
      }
    }
    const uint64_t mi = __ballot(in), mt = __ballot(tie);
    unsigned long long pos = 0;
    if (lane == 0) {
      if (mi) pos = atomicAdd(p.ocount, (unsigned long long)__popcll(mi));
      if (mt) atomicAdd(p.nties, (unsigned long long)__popcll(mt));
    }
    pos = __shfl(pos, 0, 64) + __popcll(mi & lt);
    if (in && pos < (unsigned long long)p.ccap) {
      p.keys[pos] = ((unsigned long long)mine.x << p.bj) | mine.y;
      p.dist[pos] = dist;
    }
  }
}

hipError_t launch_recheck_eps(const RecheckParams& p, hipStream_t st, int cu_count) {
  hipLaunchKernelGGL(recheck_eps_kernel, dim3(cu_count * 8), dim3(256), 0, st, p);
  return hipGetLastError();
}

// ------------------------------------------------------------ pair d2
__global__ __launch_bounds__(256) void pair_d2_kernel(const float* R, int64_t ldr, int64_t nR, const float* S,
                                                      int64_t lds, int64_t nS, int d, const uint32_t* pi,
                                                      const uint32_t* pj, int64_t m, double* out, int* bad) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t i = pi[t], j = pj[t];
    if (i >= nR || j >= nS) {
      out[t] = __longlong_as_double(0x7ff8000000000000ll);
      *reinterpret_cast<volatile int*>(bad) = 1;
      continue;
    }
    out[t] = canonical_d2(R + (int64_t)i * ldr, S + (int64_t)j * lds, d);
  }
}

hipError_t launch_pair_d2(const float* R, int64_t ldr, int64_t nR, const float* S, int64_t lds, int64_t nS, int d,
                          const uint32_t* pi, const uint32_t* pj, int64_t m, double* out, int* bad,
                          hipStream_t st, int cu_count) {
  if (m == 0) return hipSuccess;
  int64_t blocks = (m + 255) / 256;
  if (blocks > (int64_t)cu_count * 16) blocks = (int64_t)cu_count * 16;
  hipLaunchKernelGGL(pair_d2_kernel, dim3((unsigned)blocks), dim3(256), 0, st, R, ldr, nR, S, lds, nS, d, pi, pj, m,
                     out, bad);
  return hipGetLastError();
}

// ------------------------------------------------------------ top-k select
constexpr int kSelMax = 512;  // contenders per row held in LDS
constexpr int kSelWaves = 4;



__device__ inline uint32_t ord_f(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(64 * kSelWaves) void topk_select_kernel(SelectParams p) {
  __shared__ float s_d2[kSelWaves][kSelMax];
  __shared__ uint32_t s_j[kSelWaves][kSelMax];
  __shared__ double s_key[kSelWaves][kSelMax];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * kSelWaves + wave;
  if (i >= p.nR) return;
  const float* a = p.R + i * p.ldr;
  const int k = p.k;

  // (1) k-th largest P~ over the union of the row's split buffers
  auto count_ge = [&](uint32_t cand) {
    int c = 0;
    for (int s = 0; s < p.P; ++s) {
      const uint2* e = p.band + (i * p.P + s) * (int64_t)p.cap;
      const int n = p.bcount[i * p.P + s];
      for (int t = lane; t < n; t += 64) c += ord_f(__uint_as_float(e[t].x)) >= cand;
    }
    return wave_sumi(c);
  };
  int total = 0;
  for (int s = 0; s < p.P; ++s) total += p.bcount[i * p.P + s];
  float bt = -INFINITY;
  if (total >= k) {
    uint32_t t = 0;
    for (int b = 31; b >= 0; --b)
      if (count_ge(t | (1u << b)) >= k) t |= 1u << b;
    const float pk = __uint_as_float((t & 0x80000000u) ? (t & 0x7fffffffu) : ~t);
    bt = f32_down((double)pk - (double)p.marg[i]);
  }

  // (2) float32 direct-form d2 of every band entry, written over its P~:
  // 64 entries at a time, each summed by the whole wave with coalesced row
  // reads; lane t keeps entry t's sum.
  int nb = 0;
  for (int s = 0; s < p.P; ++s) {
    uint2* e = p.band + (i * p.P + s) * (int64_t)p.cap;
    const int n = p.bcount[i * p.P + s];
    for (int base = 0; base < n; base += 64) {
      const int cnt = min(64, n - base);
      const uint2 v = lane < cnt ? e[base + lane] : make_uint2(0, 0);
      const bool inband = lane < cnt && __uint_as_float(v.x) >= bt;
      const uint64_t mb = __ballot(inband);
      float mine = INFINITY;
      uint64_t rest = mb;
      while (rest) {
        const int t = __ffsll((unsigned long long)rest) - 1;
        rest &= rest - 1;
        const uint32_t jt = __shfl(v.y, t, 64);
        const float* b = p.S + (int64_t)jt * p.lds;
        float acc = 0.0f;
        for (int q = lane; q < p.d; q += 64) {
          const float u = a[q] - b[q];
          acc = fmaf(u, u, acc);
        }
        acc = wave_sumf(acc);
        if (lane == t) mine = acc;
      }
      if (lane < cnt) e[base + lane].x = __float_as_uint(mine);
      nb += __popcll(mb);
    }
  }
  if (lane != 0) nb = 0;
  nb = wave_sumi(nb);
  if (lane == 0) atomicAdd(p.nband, (unsigned long long)nb);

  // (3) per-row bound beta(d2) = c1 d2 + c0 (monotone); D_k = k-th smallest d2
  const double xsum = (double)p.xnR[i] + (double)p.sS->xnorm_max;
  const bool ex = exact32(min(p.mlR[i], p.sS->mlsb_min), xsum);
  const double c1 = ex ? 0.0 : 2.0 * gamma_n((double)p.d + 2.0, 0x1p-24);
  const double c0 = ex ? 0.0 : ((double)p.d + 2.0) * 0x1p-148 + ((double)p.d + 4.0) * 0x1p-52 * xsum * xsum;
  auto count_lt = [&](uint64_t lim) {  // entries with d2 bits < lim
    int c = 0;
    for (int s = 0; s < p.P; ++s) {
      const uint2* e = p.band + (i * p.P + s) * (int64_t)p.cap;
      const int n = p.bcount[i * p.P + s];
      for (int t = lane; t < n; t += 64) c += (uint64_t)e[t].x < lim;
    }
    return wave_sumi(c);
  };
  uint64_t dk = 0;  // bits of the k-th smallest d2 (non-negative floats order as integers)
  for (int b = 31; b >= 0; --b)
    if (count_lt(dk + (1ull << b)) < k) dk += 1ull << b;
  const double Dk = dk >= 0x7f800000ull ? INFINITY : (double)__uint_as_float((uint32_t)dk);
  // entries with d2 - beta > D_k + beta(D_k) cannot be among the k nearest
  double cut = INFINITY;
  if (!isinf(Dk)) cut = (Dk * (1.0 + c1) + 2.0 * c0) / (1.0 - c1) * (1.0 + 0x1p-50);

  // (4) contenders into LDS
  float* cd = s_d2[wave];
  uint32_t* cj = s_j[wave];
  double* ck = s_key[wave];
  int nc = 0;
  const uint64_t lt = __lanemask_lt();
  for (int s = 0; s < p.P; ++s) {
    const uint2* e = p.band + (i * p.P + s) * (int64_t)p.cap;
    const int n = p.bcount[i * p.P + s];
    for (int base = 0; base < n; base += 64) {
      const int t = base + lane;
      uint2 v = make_uint2(0x7f800000u, 0);
      if (t < n) v = e[t];
      const float d2 = __uint_as_float(v.x);
      const bool keep = t < n && !isinf(d2) && (double)d2 <= cut;
      const uint64_t m = __ballot(keep);
      const int pos = nc + __popcll(m & lt);
      if (keep && pos < kSelMax) {
        cd[pos] = d2;
        cj[pos] = v.y;
      }
      nc += __popcll(m);
    }
  }
  if (nc > kSelMax) {
    if (lane == 0) atomicOr(p.too_many, 1);
    for (int t = lane; t < k; t += 64) {
      p.out_j[i * k + t] = 0xffffffffu;
      p.out_dist[i * k + t] = INFINITY;
    }
    return;
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();

  // (5) overlapping intervals -> float64 keys
  int nt = 0;
  for (int t = lane; t < nc; t += 64) {
    const double dx = cd[t];
    const double lox = dx - (c1 * dx + c0), hix = dx + (c1 * dx + c0);
    bool tie = false;
    for (int u = 0; u < nc && !tie; ++u) {
      if (u == t) continue;
      const double dy = cd[u];
      const double loy = dy - (c1 * dy + c0), hiy = dy + (c1 * dy + c0);
      tie = !(hix * (1.0 + 0x1p-50) < loy * (1.0 - 0x1p-50) || hiy * (1.0 + 0x1p-50) < lox * (1.0 - 0x1p-50));
    }
    double key = dx;
    if (tie && !ex) {
      key = canonical_d2(a, p.S + (int64_t)cj[t] * p.lds, p.d);
      ++nt;
    }
    ck[t] = key;
  }
  nt = wave_sumi(nt);
  if (lane == 0 && nt) atomicAdd(p.nties, (unsigned long long)nt);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();

  // (6) k rounds of (key, j) argmin
  for (int r = 0; r < k; ++r) {
    double bk = INFINITY;
    uint32_t bj = 0xffffffffu;
    int bpos = -1;
    for (int t = lane; t < nc; t += 64) {
      const double kk = ck[t];
      const uint32_t jj = cj[t];
      if (kk < bk || (kk == bk && jj < bj)) { bk = kk; bj = jj; bpos = t; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ok = __shfl_xor(bk, o, 64);
      const uint32_t oj = __shfl_xor(bj, o, 64);
      const int op = __shfl_xor(bpos, o, 64);
      if (ok < bk || (ok == bk && oj < bj)) { bk = ok; bj = oj; bpos = op; }
    }
    if (lane == 0) {
      p.out_j[i * k + r] = bpos >= 0 ? bj : 0xffffffffu;
      p.out_dist[i * k + r] = bpos >= 0 ? (bk == (double)cd[bpos] ? sqrtf(cd[bpos]) : (float)sqrt(bk)) : INFINITY;
      if (bpos >= 0) ck[bpos] = INFINITY, cj[bpos] = 0xffffffffu;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
}

hipError_t launch_topk_select(const SelectParams& p, hipStream_t st) {
  if (p.nR == 0) return hipSuccess;
  hipLaunchKernelGGL(topk_select_kernel, dim3((unsigned)((p.nR + kSelWaves - 1) / kSelWaves)), dim3(64 * kSelWaves), 0,
                     st, p);
  return hipGetLastError();
}

}  // namespace dl
