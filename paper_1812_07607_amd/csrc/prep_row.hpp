// prep_row.hpp -- the per-row work of the operand prep (see prep.hip), shared
// by the prep kernel and the fused featurise-and-prep kernel, which feeds it
// histogram bins straight from LDS instead of reading float32 rows back.
#pragma once

#include "dl_internal.hpp"

namespace dl {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// E4M3 row scale: the smallest s with amax <= 448 * 2^s, clamped to the E8M0
// range (0 for an all-zero or non-finite row).
__device__ inline int e4m3_row_scale(float amax) {
  if (!(amax > 0.0f && amax <= 3.4e38f)) return 0;
  int s = ilogbf(amax) - 8;
  while (amax > ldexpf(448.0f, s)) ++s;
  while (s > -127 && amax <= ldexpf(448.0f, s - 1)) --s;
  return s < -127 ? -127 : (s > 127 ? 127 : s);
}

// One wave's state for one row: element(v, k) writes the operand copy of
// element k and adds it to the lane's sums; finish() reduces over the wave
// and stores the row's statistics (see the Prep fields).
template <int kPrec>
struct RowPrep {
  float inv_scale, scale;
  int sexp;
  double nrm2 = 0.0, qn2 = 0.0, r2 = 0.0;
  int qlsb = kLsbNone, mlsb = kLsbNone, bad = 0;
  uint8_t* qrow;

  __device__ RowPrep(const Prep& P, int64_t row, int s)
      : inv_scale(ldexpf(1.0f, -s)), scale(ldexpf(1.0f, s)), sexp(s),
        qrow(reinterpret_cast<uint8_t*>(P.q) + row * P.qld) {}

  // the float64 statistics of one element v and its operand value qv
  __device__ void stats(float v, float qv) {
    const double dv = v, dq = qv, dr = dv - dq;  // exact in float64
    nrm2 += dv * dv;
    qn2 += dq * dq;
    r2 += dr * dr;
    qlsb = min(qlsb, lsb_exp(qv));
    mlsb = min(mlsb, lsb_exp(v));
  }

  __device__ void element(float v, int64_t k) {
    if (!isfinite(v)) { bad++; v = 0.0f; }
    float qv;
    if (kPrec == DL_FP32) {
      qv = v;
      reinterpret_cast<float*>(qrow)[k] = v;
    } else if (kPrec == DL_BF16) {
      uint16_t c = enc_bf16(v);
      qv = dec_bf16(c);
      reinterpret_cast<uint16_t*>(qrow)[k] = c;
    } else if (kPrec == DL_FP16) {
      uint16_t c = enc_f16(v);
      qv = dec_f16(c);
      reinterpret_cast<uint16_t*>(qrow)[k] = c;
    } else {
      uint8_t c = enc_e4m3(v * inv_scale);
      qv = dec_e4m3(c) * scale;  // exact: power-of-two scale of a normal value
      qrow[k] = c;
    }
    stats(v, qv);
  }

  // Wave reductions and the row's statistics (lane 0 stores); bad elements
  // of a real row are counted into rs.
  __device__ void finish(const Prep& P, int64_t row, int64_t dpad, bool real, RelStats* rs, int lane) {
    nrm2 = wave_sum(nrm2);
    qn2 = wave_sum(qn2);
    r2 = wave_sum(r2);
    qlsb = wave_min(qlsb);
    mlsb = wave_min(mlsb);
    bad = (int)wave_sum((double)bad);
    if (lane == 0) {
      // float64 sums of at most dpad exact squares: relative error <= gamma_dpad
      const double g = gamma_n((double)dpad + 2.0, 0x1p-53);
      const float h = ((float)nrm2) * 0.5f;
      P.nrm2[row] = nrm2;
      P.h[row] = h;
      P.qnorm[row] = f32_up(sqrt(qn2 * (1.0 + g)) * (1.0 + 0x1p-50));
      P.rho[row] = f32_up(sqrt(r2 * (1.0 + g)) * (1.0 + 0x1p-50));
      P.xnorm[row] = f32_up(sqrt(nrm2 * (1.0 + g)) * (1.0 + 0x1p-50));
      P.dh[row] = f32_up((fabs(nrm2 * 0.5 - (double)h) + g * nrm2) * (1.0 + 0x1p-50));
      P.qlsb[row] = qlsb;
      P.hlsb[row] = lsb_exp(h);
      P.mlsb[row] = mlsb;
      P.sexp[row] = sexp;
      if (bad && real) atomicAdd(&rs->nonfinite, bad);
    }
  }
};

}  // namespace dl
