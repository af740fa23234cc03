// prep.hip -- operand copies and per-row error bounds for the candidate pass.
//
// For every row x of a relation the prep kernel writes the matrix-core
// operand q (fp32, bf16, fp16 or E4M3 with a power-of-two row scale, zero
// padded to whole K-chunks) and the quantities the margin of the candidate
// filter is built from: |x|^2, the accumulator initial value h = fl32(|x|^2)/2,
// upper bounds on |q~|, |x - q~|, |x| and | |x|^2/2 - h |, and the exponent
// of the lowest set bit of q~, h and x (an exactness certificate: sums of
// products on a common binary grid are exact in fp32 while they stay below
// 2^24 grid steps).  The reduction kernel folds these into maxima over the
// relation, and the threshold kernel turns them into one float per row of R,
// so the candidate epilogue needs a single compare per pair.
//
// Paper: the Euclidean threshold predicate of image matching (section
// "Derived Data") evaluated as |a|^2 + |b|^2 - 2 a.b on matrix cores; the
// margin and the recheck that restore exactness are this library's design.
#include "prep_row.hpp"

namespace dl {

// One wave per row; rows in [n, npad) get zero operands and zero statistics.
// perm (nullable): operand row r holds row perm[r] of X.
template <int kPrec>
__global__ __launch_bounds__(256) void prep_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                   int64_t ld, int64_t dpad, Prep P,
                                                   RelStats* __restrict__ rs, const uint32_t* __restrict__ perm) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= P.npad) return;
  const bool real = row < n;
  const float* x = X + (real ? (perm ? (int64_t)perm[row] : row) * ld : 0);
  int sexp = 0;
  if (kPrec == DL_FP8 && real) {
    float amax = 0.0f;
    for (int k = lane; k < d; k += 64) amax = fmaxf(amax, fabsf(x[k]));
    sexp = e4m3_row_scale(wave_max(amax));
  }
  RowPrep<kPrec> rp(P, row, sexp);
  constexpr bool k16 = kPrec == DL_BF16 || kPrec == DL_FP16;
  const bool vec = k16 && real && d == dpad && (d & 511) == 0 && (ld & 3) == 0 &&
                   (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  if (vec) {
    // 16-bit copies of rows whose length is a multiple of 512: each lane
    // takes eight consecutive elements per 512 (two 16-byte loads, one
    // 16-byte store); the float64 sums are exact squares added in another
    // order, within the same error bound
    for (int64_t k0 = 0; k0 < d; k0 += 512) {
      const int64_t k = k0 + 8 * lane;
      const float4 u0 = *reinterpret_cast<const float4*>(x + k);
      const float4 u1 = *reinterpret_cast<const float4*>(x + k + 4);
      float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
      uint32_t w[4];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        float t = v[u];
        if (!isfinite(t)) { rp.bad++; t = 0.0f; }
        const uint16_t c = kPrec == DL_BF16 ? enc_bf16(t) : enc_f16(t);
        const float qv = kPrec == DL_BF16 ? dec_bf16(c) : dec_f16(c);
        if (u & 1) w[u >> 1] |= (uint32_t)c << 16;
        else w[u >> 1] = c;
        rp.stats(t, qv);
      }
      *reinterpret_cast<uint4*>(rp.qrow + 2 * k) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  } else if (real) {
    // eight of the row's loads in flight per lane (clamped into the row,
    // zero past d), then the elements in order
    const int64_t dm1 = d - 1;
    int64_t k = lane;
    for (; k + 64 * 7 < dpad; k += 64 * 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t kk = k + 64 * u;
        const float t = x[kk < d ? kk : dm1];
        v[u] = kk < d ? t : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) rp.element(v[u], k + 64 * u);
    }
    for (; k < dpad; k += 64) rp.element(k < d ? x[k] : 0.0f, k);
  } else {
    for (int64_t k = lane; k < dpad; k += 64) rp.element(0.0f, k);
  }
  rp.finish(P, row, dpad, real, rs, lane);
}

__global__ void stats_init_kernel(RelStats* rs) {
  if (threadIdx.x == 0) {
    rs->h_max = rs->qnorm_max = rs->rho_max = rs->dh_max = rs->xnorm_max = 0.0f;
    rs->qlsb_min = rs->hlsb_min = rs->mlsb_min = kLsbNone;
    rs->nonfinite = 0;
  }
}

// Maxima / minima over the real rows: a grid-stride pass, a wave and then a
// workgroup reduction through LDS, and one atomic per field per workgroup.
// Non-negative floats order like their bit patterns, so integer atomics
// suffice.
__global__ __launch_bounds__(256) void stats_reduce_kernel(Prep P, int64_t n, RelStats* rs) {
  __shared__ float lf[5][4];
  __shared__ int li[3][4];
  float hm = 0, qm = 0, rm = 0, dm = 0, xm = 0;
  int ql = kLsbNone, hl = kLsbNone, ml = kLsbNone;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    hm = fmaxf(hm, P.h[r]);
    qm = fmaxf(qm, P.qnorm[r]);
    rm = fmaxf(rm, P.rho[r]);
    dm = fmaxf(dm, P.dh[r]);
    xm = fmaxf(xm, P.xnorm[r]);
    ql = min(ql, P.qlsb[r]);
    hl = min(hl, P.hlsb[r]);
    ml = min(ml, P.mlsb[r]);
  }
  hm = wave_max(hm); qm = wave_max(qm); rm = wave_max(rm); dm = wave_max(dm); xm = wave_max(xm);
  ql = wave_min(ql); hl = wave_min(hl); ml = wave_min(ml);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    lf[0][w] = hm; lf[1][w] = qm; lf[2][w] = rm; lf[3][w] = dm; lf[4][w] = xm;
    li[0][w] = ql; li[1][w] = hl; li[2][w] = ml;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int f = threadIdx.x;
    const float v = fmaxf(fmaxf(lf[f][0], lf[f][1]), fmaxf(lf[f][2], lf[f][3]));
    float* dst = f == 0 ? &rs->h_max : f == 1 ? &rs->qnorm_max : f == 2 ? &rs->rho_max : f == 3 ? &rs->dh_max
                                                                                                : &rs->xnorm_max;
    atomicMax(reinterpret_cast<unsigned*>(dst), __float_as_uint(v));
  } else if (threadIdx.x < 8) {
    const int f = threadIdx.x - 5;
    const int v = min(min(li[f][0], li[f][1]), min(li[f][2], li[f][3]));
    atomicMin(f == 0 ? &rs->qlsb_min : f == 1 ? &rs->hlsb_min : &rs->mlsb_min, v);
  }
}

// Bound E_i on |d~2 - d2_64| over every row j of S, where d~2 = |a|^2 - 2 P~
// and P~ is the matrix-core value of a.b - h_j (see the derivation in the
// design notes):
//   accumulation  2 gamma_{d+2}(h_max + |q~_i| max|q~_j|) + (d+1) 2^-126,
//                 or 0 when every partial sum is exact on a common grid;
//   operands      |q~_i| max rho_j + rho_i max|q~_j| + rho_i max rho_j;
//   init          max | |b|^2/2 - h_j |;
//   float64       (d+4) 2^-52 ((|a| + max|b|)^2 + |a|^2).
// pass_exact (optional): set when the candidate pass computes P~ for row i
// exactly, i.e. P~ = a.b - |b|^2/2 for every b of S: operand copies equal to
// the rows (rho = 0), h exact and an exact accumulation.
__device__ inline double row_margin(const Prep& R, const RelStats& s, int64_t i, int d, bool* pass_exact = nullptr) {
  const double qa = R.qnorm[i], ra = R.rho[i];
  const int ql = R.qlsb[i];
  const int prod = (ql >= kLsbNone || s.qlsb_min >= kLsbNone) ? kLsbNone : ql + s.qlsb_min;
  const int m = min(prod, s.hlsb_min);
  const bool exact = m >= -126 && (qa * (double)s.qnorm_max + (double)s.h_max) <= ldexp(1.0, min(m + 24, 1000));
  const double acc = exact ? 0.0
                           : 2.0 * gamma_n((double)d + 2.0, 0x1p-24) * ((double)s.h_max + qa * s.qnorm_max) +
                                 ((double)d + 1.0) * 0x1p-126;
  const double opnd = qa * s.rho_max + ra * s.qnorm_max + ra * s.rho_max;
  if (pass_exact) {
    // h_j = |b_j|^2 / 2 exactly for every b of S: S on the grid 2^m with
    // |b|^2 <= 2^(2m+24) (its squares and sums are exact in float32 and
    // float64 alike); dh itself always carries the float64 sum's bound
    const bool h_exact = s.mlsb_min >= kLsbNone ||
                         (2 * s.mlsb_min >= -126 &&
                          (double)s.xnorm_max * (double)s.xnorm_max <= ldexp(1.0, 2 * s.mlsb_min + 24));
    *pass_exact = exact && ra == 0.0 && s.rho_max == 0.0f && h_exact;
  }
  const double xa = R.xnorm[i], xs = s.xnorm_max;
  const double canon = ((double)d + 4.0) * 0x1p-52 * ((xa + xs) * (xa + xs) + R.nrm2[i]);
  return (2.0 * (acc + opnd + (double)s.dh_max) + canon) * (1.0 + 0x1p-40);
}

// eps mode: thr_i such that P~ >= thr_i for every pair with d2_64 <= T.
// band mode: marg_i = E_i rounded up (the top-k band is P~ >= P~_(k) - E_i).
__global__ __launch_bounds__(256) void threshold_kernel(Prep R, int64_t nR, const RelStats* __restrict__ S,
                                                        int d, double Tall, const double* __restrict__ Trow,
                                                        float* __restrict__ thr, float* __restrict__ marg,
                                                        int* __restrict__ pex, uint32_t* __restrict__ gkey) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R.npad) return;
  if (gkey) gkey[i] = order_key(-INFINITY);  // no bound yet
  if (i >= nR) {
    if (thr) thr[i] = INFINITY;
    if (marg) marg[i] = 0.0f;
    if (pex) pex[i] = 0;
    return;
  }
  const RelStats s = *S;
  bool px = false;
  const double E = row_margin(R, s, i, d, &px);
  if (pex) pex[i] = px ? 1 : 0;
  if (marg) marg[i] = f32_up(E);
  if (thr) {
    const double T = Trow ? Trow[i] : Tall;
    const double a2 = R.nrm2[i];
    if (isinf(T)) thr[i] = -INFINITY;
    else thr[i] = f32_down(0.5 * (a2 - T - E) - 0x1p-50 * (fabs(a2) + fabs(T) + E));
  }
}

// Seeds each row's top-k band from an exact top-k of the row against a
// sample of S (dist: the sample's k smallest distances, ascending, +inf
// padded).  P = x.y - |y|^2/2 = (|x|^2 - d^2)/2, so the sample's k-th
// smallest d^2 gives a lower bound of the k-th largest P over the sample,
// hence over S; the band threshold is that bound minus E_i.  The bound is
// loosened generously (the reported distance is a float rounding of the
// exact one): any smaller threshold keeps the band a superset.
__global__ __launch_bounds__(256) void band_seed_kernel(Prep R, int64_t nR, const float* __restrict__ dist, int k,
                                                        const float* __restrict__ marg, uint32_t* __restrict__ gkey) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nR) return;
  const float dk = dist[i * k + (k - 1)];
  if (!(dk < INFINITY)) return;  // fewer than k sample rows: no bound
  const double d2 = (double)dk * (double)dk * (1.0 + 0x1p-10) + 0x1p-30;
  const double x2 = R.nrm2[i] * (1.0 - 0x1p-40);
  const float t = f32_down(0.5 * (x2 - d2) - (double)marg[i] - 0x1p-30);
  gkey[i] = max(gkey[i], order_key(t));
}

hipError_t launch_band_seed(const Prep& R, int64_t nR, const float* dist, int k, const float* marg, uint32_t* gkey,
                            hipStream_t st) {
  if (nR == 0) return hipSuccess;
  hipLaunchKernelGGL(band_seed_kernel, dim3((unsigned)((nR + 255) / 256)), dim3(256), 0, st, R, nR, dist, k, marg,
                     gkey);
  return hipGetLastError();
}

hipError_t launch_prep(const float* X, int64_t n, int32_t d, int64_t ld, dl_prec prec, const Prep& P,
                       RelStats* rs, hipStream_t st, int cu_count, const uint32_t* perm) {
  hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(64), 0, st, rs);
  const int64_t dpad = dpad_of(d, prec);
  const dim3 grid((unsigned)((P.npad + 3) / 4)), block(256);
  switch (prec) {
    case DL_FP32: hipLaunchKernelGGL(prep_kernel<DL_FP32>, grid, block, 0, st, X, n, d, ld, dpad, P, rs, perm); break;
    case DL_BF16: hipLaunchKernelGGL(prep_kernel<DL_BF16>, grid, block, 0, st, X, n, d, ld, dpad, P, rs, perm); break;
    case DL_FP16: hipLaunchKernelGGL(prep_kernel<DL_FP16>, grid, block, 0, st, X, n, d, ld, dpad, P, rs, perm); break;
    case DL_FP8: hipLaunchKernelGGL(prep_kernel<DL_FP8>, grid, block, 0, st, X, n, d, ld, dpad, P, rs, perm); break;
  }
  if (n > 0) {
    int64_t blocks = (n + 1023) / 1024;
    if (blocks > (int64_t)cu_count) blocks = (int64_t)cu_count;
    hipLaunchKernelGGL(stats_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, P, n, rs);
  }
  return hipGetLastError();
}

hipError_t launch_stats_init(RelStats* rs, hipStream_t st) {
  hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(64), 0, st, rs);
  return hipGetLastError();
}

// The relation maxima of rows [0, n) of P (after launch_stats_init).
hipError_t launch_stats_reduce(const Prep& P, int64_t n, RelStats* rs, hipStream_t st, int cu_count) {
  if (n > 0) {
    int64_t blocks = (n + 1023) / 1024;
    if (blocks > (int64_t)cu_count) blocks = (int64_t)cu_count;
    hipLaunchKernelGGL(stats_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, P, n, rs);
  }
  return hipGetLastError();
}

hipError_t launch_threshold(const Prep& R, int64_t nR, const RelStats* S, int d, double T, const double* Trow,
                            float* thr, float* marg, int* pex, uint32_t* gkey, hipStream_t st) {
  const dim3 grid((unsigned)((R.npad + 255) / 256));
  hipLaunchKernelGGL(threshold_kernel, grid, dim3(256), 0, st, R, nR, S, d, T, Trow, thr, marg, pex, gkey);
  return hipGetLastError();
}

}  // namespace dl
