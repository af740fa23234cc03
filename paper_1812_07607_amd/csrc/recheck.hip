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

// float32 direct-form d2 of rows a and b, summed by one lane in increasing
// k (any order stays within the bound beta).  vec4: both rows 16-byte
// aligned.
__device__ inline float lane_d2(const float* a, const float* b, int d, bool vec4) {
  float acc = 0.0f;
  int q = 0;
  if (vec4) {
    // unrolled so that several row loads are in flight per lane; the sum is
    // still one chain in index order
#pragma unroll 8
    for (; q + 4 <= d; q += 4) {
      const float4 x = *reinterpret_cast<const float4*>(a + q);
      const float4 y = *reinterpret_cast<const float4*>(b + q);
      float u = x.x - y.x;
      acc = fmaf(u, u, acc);
      u = x.y - y.y;
      acc = fmaf(u, u, acc);
      u = x.z - y.z;
      acc = fmaf(u, u, acc);
      u = x.w - y.w;
      acc = fmaf(u, u, acc);
    }
  }
  for (; q < d; ++q) {
    const float u = a[q] - b[q];
    acc = fmaf(u, u, acc);
  }
  return acc;
}

// ------------------------------------------------------------ eps recheck


// A wave takes 64 candidates at a time: each lane computes its candidate's
// float32 distance from the two rows (16-byte row loads, several in flight),
// then the wave classifies the 64 lane-parallel; the confirmed
// ones of kRecheckChunks such batches are appended with a single atomic (one
// counter serves the whole grid, so its atomics are kept few).  A candidate
// whose P~ the matrix-core pass computed exactly (pexR) and whose float32
// form is exact (the lowest-set-bit certificate) needs no row reads: then
// d2 = |a|^2 - 2 P~ exactly (P~ = a.b - |b|^2/2), evaluated in float64
// without rounding.
constexpr int kRecheckChunks = 4;  // 64-candidate chunks per wave and output atomic

__global__ __launch_bounds__(256) void recheck_eps_kernel(RecheckParams p) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t n = min((int64_t)*p.ccount, p.ccap);
  const uint64_t lt = __lanemask_lt();
  // 16-byte row loads when S rows are aligned (R rows are checked per row)
  const bool vec4 = (reinterpret_cast<uintptr_t>(p.S) & 15) == 0 && (p.lds & 3) == 0 && (p.ldr & 3) == 0;
  constexpr int64_t kSpan = 64 * kRecheckChunks;
  for (int64_t base0 = gw * kSpan; base0 < n; base0 += nw * kSpan) {
    bool in[kRecheckChunks], tie[kRecheckChunks];
    float dist[kRecheckChunks];
    uint2 mine[kRecheckChunks];
#pragma unroll
    for (int c = 0; c < kRecheckChunks; ++c) {
      const int64_t base = base0 + c * 64;
      const int cnt = (int)max((int64_t)0, min((int64_t)64, n - base));
      mine[c] = lane < cnt ? p.cand[base + lane] : make_uint2(0, 0);
      float mys = 0.0f;
      bool quick = false;  // d2 from P~ (see above)
      if (lane < cnt && p.candp && p.pexR[mine[c].x]) {
        const double xs = (double)p.xnR[mine[c].x] + (double)p.xnS[mine[c].y];
        if (exact32(min(p.mlR[mine[c].x], p.mlS[mine[c].y]), xs)) {
          quick = true;
          mys = (float)(p.nrm2R[mine[c].x] - 2.0 * (double)p.candp[base + lane]);
        }
      }
      // the candidate's rows of R and S (through the permutations of an
      // index-pruned join; statistics stay indexed by the operand row)
      const uint32_t oi = lane < cnt && p.permR ? p.permR[mine[c].x] : mine[c].x;
      const uint32_t oj = lane < cnt && p.permS ? p.permS[mine[c].y] : mine[c].y;
      const float* a = p.R + (int64_t)oi * p.ldr;
      const float* b = p.S + (int64_t)oj * p.lds;
      // each lane sums its own candidate's row pair: the value depends on
      // the pair alone, not on which candidates share the wave
      if (lane < cnt && !quick)
        mys = lane_d2(a, b, p.d, vec4 && (reinterpret_cast<uintptr_t>(a) & 15) == 0);
      in[c] = false;
      tie[c] = false;
      dist[c] = 0.0f;
      if (lane < cnt) {
        const double d2 = mys;
        const double xsum = (double)p.xnR[mine[c].x] + (double)p.xnS[mine[c].y];
        const bool ex = exact32(min(p.mlR[mine[c].x], p.mlS[mine[c].y]), xsum);
        const double bt = ex ? 0.0 : beta32(d2, p.d, xsum);
        const double hi = ex ? d2 : (d2 + bt) * (1.0 + 0x1p-50);
        const double lo = ex ? d2 : (d2 - bt) * (1.0 - 0x1p-50);
        const double T = p.Trow ? p.Trow[mine[c].x] : p.T;
        in[c] = hi <= T;
        dist[c] = sqrtf(mys);
        if (!in[c] && !(lo > T)) {  // boundary tie: the canonical float64 value decides
          tie[c] = true;
          const double d64 = canonical_d2(a, b, p.d);
          in[c] = d64 <= T;
          dist[c] = (float)sqrt(d64);
        }
      }
      // the output names the pair by its rows of R and S (a self-join's
      // smaller row first)
      mine[c] = p.swap && oi > oj ? make_uint2(oj, oi) : make_uint2(oi, oj);
    }
    // one atomic for the whole span
    uint64_t mi[kRecheckChunks];
    int total = 0, nt = 0;
#pragma unroll
    for (int c = 0; c < kRecheckChunks; ++c) {
      mi[c] = __ballot(in[c]);
      total += __popcll(mi[c]);
      nt += __popcll(__ballot(tie[c]));
    }
    if (total == 0 && nt == 0) continue;
    unsigned long long pos = 0;
    if (lane == 0) {
      if (total) pos = atomicAdd(p.ocount, (unsigned long long)total);
      if (nt) atomicAdd(p.nties, (unsigned long long)nt);
    }
    pos = __shfl(pos, 0, 64);
#pragma unroll
    for (int c = 0; c < kRecheckChunks; ++c) {
      const unsigned long long at = pos + __popcll(mi[c] & lt);
      if (in[c] && at < (unsigned long long)p.ccap) {
        p.keys[at] = ((unsigned long long)mine[c].x << p.bj) | mine[c].y;
        p.dist[at] = dist[c];
      }
      pos += __popcll(mi[c]);
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
// Contenders per row held in LDS: kSelSmall for k <= 128 (smaller LDS
// buffers, more waves per CU), kSelLarge otherwise and whenever a row of
// the small launch had more (the host then runs the select again).
constexpr int kSelSmall = 256;
constexpr int kSelLarge = 512;
constexpr int kSelWaves = 4;
constexpr int kSelRegs = 8;   // band entries per lane held in registers (unions up to 512)



__device__ inline uint32_t ord_f(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}


// One wave per row.  Counting over the row's band entries uses ballots
// (scalar popcounts, no shuffle chains); distances are computed one entry
// per lane; the k nearest are emitted by rank, since the (key, j) pairs of a
// row are distinct.
// LDS per wave: the contenders' float32 d2, j and float64 key (16 bytes
// each), and, before any contender is written, the staged band entries
// (64 * kSelRegs of 8 bytes) in the same bytes.
template <int kSelMax>
__global__ __launch_bounds__(64 * kSelWaves, kSelMax == kSelSmall ? 6 : 4) void topk_select_kernel(SelectParams p) {
  constexpr int kBytes = 16 * kSelMax > 8 * 64 * kSelRegs ? 16 * kSelMax : 8 * 64 * kSelRegs;
  __shared__ __attribute__((aligned(16))) uint8_t s_buf[kSelWaves][kBytes];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = (int64_t)blockIdx.x * kSelWaves + wave;
  if (i >= p.nR) return;
  const float* a = p.R + i * p.ldr;
  const int k = p.k;
  if (p.gate && __builtin_amdgcn_readfirstlane(*p.gate)) {
    // invalid input: the candidate pass did no work and the band counts are
    // not set; the call reports the error, the rows hold padding
    for (int t = lane; t < k; t += 64) {
      p.out_j[i * k + t] = 0xffffffffu;
      p.out_dist[i * k + t] = INFINITY;
    }
    return;
  }
  const uint64_t lt = __lanemask_lt();
  int total = 0;
  for (int s = 0; s < p.P; ++s) total += p.bcount[i * p.P + s];
  const double xsum = (double)p.xnR[i] + (double)p.sS->xnorm_max;
  const bool ex = exact32(min(p.mlR[i], p.sS->mlsb_min), xsum);
  const double c1 = ex ? 0.0 : 2.0 * gamma_n((double)p.d + 2.0, 0x1p-24);
  const double c0 = ex ? 0.0 : ((double)p.d + 2.0) * 0x1p-148 + ((double)p.d + 4.0) * 0x1p-52 * xsum * xsum;
  const bool vec4 = ((reinterpret_cast<uintptr_t>(p.S) | reinterpret_cast<uintptr_t>(a)) & 15) == 0 &&
                    (p.lds & 3) == 0;
  float* cd = reinterpret_cast<float*>(s_buf[wave]);
  uint32_t* cj = reinterpret_cast<uint32_t*>(s_buf[wave] + 4 * kSelMax);
  double* ck = reinterpret_cast<double*>(s_buf[wave] + 8 * kSelMax);
  int nc = 0, nb = 0;
  // entries with d2 - beta > D_k + beta(D_k) cannot be among the k nearest
  auto cut_of = [&](uint64_t dk) {
    const double Dk = dk >= 0x7f800000ull ? INFINITY : (double)__uint_as_float((uint32_t)dk);
    return isinf(Dk) ? INFINITY : (Dk * (1.0 + c1) + 2.0 * c0) / (1.0 - c1) * (1.0 + 0x1p-50);
  };
  // Stage into LDS, compactly, the union's entries with P~ >= floor (up to
  // 64 * kSelRegs of them); returns how many there are.
  uint2* st = reinterpret_cast<uint2*>(s_buf[wave]);
  auto stage = [&](float floor) {
    int g = 0;
    for (int s = 0; s < p.P; ++s) {
      const uint2* e = p.band + (i * p.P + s) * (int64_t)p.cap;
      const int n = p.bcount[i * p.P + s];
      for (int base = 0; base < n; base += 64) {
        const int t = base + lane;
        const uint2 v = t < n ? e[t] : make_uint2(0, 0);
        const bool in = t < n && __uint_as_float(v.x) >= floor;
        const uint64_t m = __ballot(in);
        const int pos = g + __popcll(m & lt);
        if (in && pos < 64 * kSelRegs) st[pos] = v;
        g += __popcll(m);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    return g;
  };
  // k-th largest P~ of the staged entries, minus the margin (the band
  // threshold they imply), by ballot counts over registers
  auto band_of = [&](const uint32_t (&key)[kSelRegs], int cnt) {
    if (cnt < k) return -INFINITY;
    const int nr = (cnt + 63) / 64;
    uint32_t t = 0;
    for (int b = 31; b >= 0; --b) {
      const uint32_t cand = t | (1u << b);
      int c = 0;
#pragma unroll
      for (int r = 0; r < kSelRegs; ++r)
        if (r < nr) c += __popcll(mask_ge(key[r], cand));
      if (c >= k) t = cand;
    }
    const float pk = __uint_as_float((t & 0x80000000u) ? (t & 0x7fffffffu) : ~t);
    return f32_down((double)pk - (double)p.marg[i]);
  };
  auto load_keys = [&](uint32_t (&key)[kSelRegs], uint32_t (&jv)[kSelRegs], int cnt) {
#pragma unroll
    for (int r = 0; r < kSelRegs; ++r) {
      const int gi = r * 64 + lane;
      const uint2 v = gi < cnt ? st[gi] : make_uint2(0xff800000u, 0xffffffffu);
      key[r] = gi < cnt ? ord_f(__uint_as_float(v.x)) : 0u;
      jv[r] = v.y;
    }
  };
  uint32_t key[kSelRegs], jv[kSelRegs];
  // A row whose buffers an earlier selection over memory rewrote holds d2
  // (not P~) in its entries: it goes to the memory path with the band known.
  const bool in_d2 = p.rstate && __builtin_amdgcn_readfirstlane(p.rstate[i]);
  // A union too large for the registers is first filtered with the band of
  // its first entries: any lower bound of its k-th largest P~ keeps the
  // whole exact band, so the entries above it carry the same answer.
  int kept = in_d2 ? 64 * kSelRegs + 1 : stage(-INFINITY);
  if (!in_d2 && kept > 64 * kSelRegs) {
    load_keys(key, jv, 64 * kSelRegs);
    kept = stage(band_of(key, 64 * kSelRegs));
  }
  if (kept <= 64 * kSelRegs) {
    // the (filtered) union in registers: both order statistics are ballot
    // counts over registers
    const int total = kept;
    load_keys(key, jv, total);
#pragma unroll
    for (int r = 0; r < kSelRegs; ++r) {
      const int gi = r * 64 + lane;
      const uint2 v = gi < total ? st[gi] : make_uint2(0xff800000u, 0xffffffffu);
      key[r] = gi < total ? ord_f(__uint_as_float(v.x)) : 0u;
      jv[r] = v.y;
    }
    const int nr = (total + 63) / 64;  // register slots in use (block-uniform)
    // (1) k-th largest P~ over the union
    const float bt = band_of(key, total);
    // (2) float32 direct-form d2 of the entries in the band (+inf for the
    // others; all-ones bits, which no count below includes, for the slots
    // past the union)
    const uint32_t kbt = ord_f(bt);
    uint32_t d2b[kSelRegs];
#pragma unroll
    for (int r = 0; r < kSelRegs; ++r) {
      d2b[r] = r * 64 + lane < total ? 0x7f800000u : 0xffffffffu;
      if (r < nr) {
        const bool inband = r * 64 + lane < total && key[r] >= kbt;
        if (inband) d2b[r] = __float_as_uint(lane_d2(a, p.S + (int64_t)jv[r] * p.lds, p.d, vec4));
        nb += __popcll(__ballot(inband));
      }
    }
    // (3) D_k = k-th smallest d2 (non-negative floats order as integers)
    uint64_t dk = 0;
    for (int b = 31; b >= 0; --b) {
      const uint64_t lim = dk + (1ull << b);
      int c = 0;
#pragma unroll
      for (int r = 0; r < kSelRegs; ++r)
        if (r < nr) c += __popcll(mask_lt((uint64_t)d2b[r], lim));
      if (c < k) dk = lim;
    }
    const double cut = cut_of(dk);
    // (4) contenders into LDS
#pragma unroll
    for (int r = 0; r < kSelRegs; ++r) {
      if (r < nr) {
        const float d2 = __uint_as_float(d2b[r]);
        const bool keep = !isinf(d2) && (double)d2 <= cut;
        const uint64_t m = __ballot(keep);
        const int pos = nc + __popcll(m & lt);
        if (keep && pos < kSelMax) {
          cd[pos] = d2;
          cj[pos] = jv[r];
        }
        nc += __popcll(m);
      }
    }
  } else {
    // a large union: the same steps over the split buffers in memory
    auto count = [&](auto pred) {
      int c = 0;
      for (int s = 0; s < p.P; ++s) {
        const uint2* e = p.band + (i * p.P + s) * (int64_t)p.cap;
        const int n = p.bcount[i * p.P + s];
        for (int base = 0; base < n; base += 64) {
          const int t = base + lane;
          c += __popcll(__ballot(t < n && pred(e[t].x)));
        }
      }
      return c;
    };
    if (!in_d2) {
      float bt = -INFINITY;
      if (total >= k) {
        uint32_t t = 0;
        for (int b = 31; b >= 0; --b) {
          const uint32_t cand = t | (1u << b);
          if (count([&](uint32_t w) { return ord_f(__uint_as_float(w)) >= cand; }) >= k) t = cand;
        }
        const float pk = __uint_as_float((t & 0x80000000u) ? (t & 0x7fffffffu) : ~t);
        bt = f32_down((double)pk - (double)p.marg[i]);
      }
      // each entry's P~ is replaced by its float32 d2 (+inf outside the
      // band): the steps below, and any later selection of the row, read that
      for (int s = 0; s < p.P; ++s) {
        uint2* e = p.band + (i * p.P + s) * (int64_t)p.cap;
        const int n = p.bcount[i * p.P + s];
        for (int base = 0; base < n; base += 64) {
          const int t = base + lane;
          const uint2 v = t < n ? e[t] : make_uint2(0, 0);
          const bool inband = t < n && __uint_as_float(v.x) >= bt;
          float d2 = INFINITY;
          if (inband) d2 = lane_d2(a, p.S + (int64_t)v.y * p.lds, p.d, vec4);
          if (t < n) e[t].x = __float_as_uint(d2);
          nb += __popcll(__ballot(inband));
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      if (p.rstate && lane == 0) p.rstate[i] = 1;
    } else {
      nb = count([](uint32_t w) { return w < 0x7f800000u; });
    }
    uint64_t dk = 0;
    for (int b = 31; b >= 0; --b) {
      const uint64_t lim = dk + (1ull << b);
      if (count([&](uint32_t w) { return (uint64_t)w < lim; }) < k) dk = lim;
    }
    const double cut = cut_of(dk);
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
  }
  if (lane == 0) atomicAdd(p.nband, (unsigned long long)nb);
  if (nc > kSelMax) {
    if (lane == 0) {
      atomicOr(p.too_many, 1);
      if (p.wide) p.wide[i] = 1;
    }
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

  // (6) each contender's rank in (key, j) order is its output slot
  for (int t = lane; t < nc; t += 64) {
    const double kt = ck[t];
    const uint32_t jt = cj[t];
    int rank = 0;
    for (int u = 0; u < nc; ++u) {
      const double ku = ck[u];
      rank += ku < kt || (ku == kt && cj[u] < jt);
    }
    if (rank < k) {
      p.out_j[i * k + rank] = jt;
      p.out_dist[i * k + rank] = kt == (double)cd[t] ? sqrtf(cd[t]) : (float)sqrt(kt);
    }
  }
  for (int r = nc + lane; r < k; r += 64) {
    p.out_j[i * k + r] = 0xffffffffu;
    p.out_dist[i * k + r] = INFINITY;
  }
}

// Rows with more near-tie contenders than the selection's LDS holds (p.wide
// set): one wave per such row works on the row's band buffers in memory.
// Every contender (float32 d2 within the cut) gets its float64 canonical key,
// recomputed wherever it is needed instead of stored; the k-th smallest
// (key, j) is found bit by bit over the 96-bit pair (64 key bits, then 32
// index bits), counting the contenders below each trial value, and the k
// contenders at or below it are ranked in LDS.  Slow (96 counting passes,
// each d float64 operations per contender) but bounded by the row's band,
// so a row of many exact duplicates still gets its exact answer.
__global__ __launch_bounds__(64 * kSelWaves) void topk_select_wide_kernel(SelectParams p) {
  __shared__ double s_key[kSelWaves][256];
  __shared__ uint32_t s_j[kSelWaves][256];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = (int64_t)blockIdx.x * kSelWaves + wave;
  if (i >= p.nR || !__builtin_amdgcn_readfirstlane(p.wide[i])) return;
  const float* a = p.R + i * p.ldr;
  const int k = p.k;
  const uint64_t lt = __lanemask_lt();
  const bool vec4 = ((reinterpret_cast<uintptr_t>(p.S) | reinterpret_cast<uintptr_t>(a)) & 15) == 0 &&
                    (p.lds & 3) == 0;
  int total = 0;
  for (int s = 0; s < p.P; ++s) total += p.bcount[i * p.P + s];
  auto count = [&](auto pred) {
    int c = 0;
    for (int s = 0; s < p.P; ++s) {
      const uint2* e = p.band + (i * p.P + s) * (int64_t)p.cap;
      const int n = p.bcount[i * p.P + s];
      for (int base = 0; base < n; base += 64) {
        const int t = base + lane;
        c += __popcll(__ballot(t < n && pred(e[t])));
      }
    }
    return c;
  };
  // (1) the row's entries as float32 d2 (+inf outside the band)
  if (!__builtin_amdgcn_readfirstlane(p.rstate[i])) {
    float bt = -INFINITY;
    if (total >= k) {
      uint32_t t = 0;
      for (int b = 31; b >= 0; --b) {
        const uint32_t cand = t | (1u << b);
        if (count([&](uint2 v) { return ord_f(__uint_as_float(v.x)) >= cand; }) >= k) t = cand;
      }
      const float pk = __uint_as_float((t & 0x80000000u) ? (t & 0x7fffffffu) : ~t);
      bt = f32_down((double)pk - (double)p.marg[i]);
    }
    for (int s = 0; s < p.P; ++s) {
      uint2* e = p.band + (i * p.P + s) * (int64_t)p.cap;
      const int n = p.bcount[i * p.P + s];
      for (int base = 0; base < n; base += 64) {
        const int t = base + lane;
        const uint2 v = t < n ? e[t] : make_uint2(0, 0);
        float d2 = INFINITY;
        if (t < n && __uint_as_float(v.x) >= bt) d2 = lane_d2(a, p.S + (int64_t)v.y * p.lds, p.d, vec4);
        if (t < n) e[t].x = __float_as_uint(d2);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    if (lane == 0) p.rstate[i] = 1;
  }
  // (2) D_k and the cut, as in the selection
  const double xsum = (double)p.xnR[i] + (double)p.sS->xnorm_max;
  const bool ex = exact32(min(p.mlR[i], p.sS->mlsb_min), xsum);
  const double c1 = ex ? 0.0 : 2.0 * gamma_n((double)p.d + 2.0, 0x1p-24);
  const double c0 = ex ? 0.0 : ((double)p.d + 2.0) * 0x1p-148 + ((double)p.d + 4.0) * 0x1p-52 * xsum * xsum;
  uint64_t dk = 0;
  for (int b = 31; b >= 0; --b) {
    const uint64_t lim = dk + (1ull << b);
    if (count([&](uint2 v) { return (uint64_t)v.x < lim; }) < k) dk = lim;
  }
  const double Dk = dk >= 0x7f800000ull ? INFINITY : (double)__uint_as_float((uint32_t)dk);
  const double cut = isinf(Dk) ? INFINITY : (Dk * (1.0 + c1) + 2.0 * c0) / (1.0 - c1) * (1.0 + 0x1p-50);
  auto contender = [&](uint2 v) {
    const float d2 = __uint_as_float(v.x);
    return !isinf(d2) && (double)d2 <= cut;
  };
  auto key_of = [&](uint2 v) { return canonical_d2(a, p.S + (int64_t)v.y * p.lds, p.d); };
  const int nc = count(contender);
  const int want = nc < k ? nc : k;
  // (3) the want-th smallest (key, j): largest (K, J) with fewer than want
  // contenders below it
  uint64_t K = 0;
  uint32_t J = 0;
  if (want > 0) {
    for (int b = 63; b >= 0; --b) {
      const uint64_t cand = K | (1ull << b);
      const int c = count([&](uint2 v) {
        return contender(v) && (uint64_t)__double_as_longlong(key_of(v)) < cand;
      });
      if (c < want) K = cand;
    }
    for (int b = 31; b >= 0; --b) {
      const uint32_t cand = J | (1u << b);
      const int c = count([&](uint2 v) {
        if (!contender(v)) return false;
        const uint64_t kv = (uint64_t)__double_as_longlong(key_of(v));
        return kv < K || (kv == K && v.y < cand);
      });
      if (c < want) J = cand;
    }
  }
  // (4) the want contenders at or below (K, J) into LDS, then ranked
  int g = 0;
  for (int s = 0; s < p.P; ++s) {
    const uint2* e = p.band + (i * p.P + s) * (int64_t)p.cap;
    const int n = p.bcount[i * p.P + s];
    for (int base = 0; base < n; base += 64) {
      const int t = base + lane;
      const uint2 v = t < n ? e[t] : make_uint2(0x7f800000u, 0);
      double kd = 0.0;
      bool in = false;
      if (t < n && contender(v)) {
        kd = key_of(v);
        const uint64_t kv = (uint64_t)__double_as_longlong(kd);
        in = kv < K || (kv == K && v.y <= J);
      }
      const uint64_t m = __ballot(in);
      const int pos = g + __popcll(m & lt);
      if (in && pos < want) {
        s_key[wave][pos] = kd;
        s_j[wave][pos] = v.y;
      }
      g += __popcll(m);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  for (int t = lane; t < want; t += 64) {
    const double kt = s_key[wave][t];
    const uint32_t jt = s_j[wave][t];
    int rank = 0;
    for (int u = 0; u < want; ++u) {
      const double ku = s_key[wave][u];
      rank += ku < kt || (ku == kt && s_j[wave][u] < jt);
    }
    p.out_j[i * k + rank] = jt;
    p.out_dist[i * k + rank] = (float)sqrt(kt);
  }
  for (int r = want + lane; r < k; r += 64) {
    p.out_j[i * k + r] = 0xffffffffu;
    p.out_dist[i * k + r] = INFINITY;
  }
  const int nt = want;
  if (lane == 0) {
    atomicAdd(p.nties, (unsigned long long)nt);
    p.wide[i] = 0;
  }
}

hipError_t launch_topk_select_wide(const SelectParams& p, hipStream_t st) {
  if (p.nR == 0 || !p.wide || !p.rstate) return hipSuccess;
  const dim3 grid((unsigned)((p.nR + kSelWaves - 1) / kSelWaves)), block(64 * kSelWaves);
  hipLaunchKernelGGL(topk_select_wide_kernel, grid, block, 0, st, p);
  return hipGetLastError();
}

hipError_t launch_topk_select(const SelectParams& p, bool small, hipStream_t st) {
  if (p.nR == 0) return hipSuccess;
  const dim3 grid((unsigned)((p.nR + kSelWaves - 1) / kSelWaves)), block(64 * kSelWaves);
  if (small) hipLaunchKernelGGL(topk_select_kernel<kSelSmall>, grid, block, 0, st, p);
  else hipLaunchKernelGGL(topk_select_kernel<kSelLarge>, grid, block, 0, st, p);
  return hipGetLastError();
}
bool topk_select_small(int k) { return k <= 128; }

}  // namespace dl
