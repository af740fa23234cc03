// dl_internal.hpp -- shared declarations of the dlmi HIP sources (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dlmi.h"

namespace dl {

// ------------------------------------------------------------------ limits
constexpr int kMaxDim = 4096;
constexpr int kTile = 256;          // rows of R and of S per contraction tile
constexpr int kChunkBytes = 128;    // bytes of one row per K-chunk in LDS
constexpr int kLsbNone = 100000;    // "no nonzero element" lsb sentinel
// Most candidate pairs one eps-join call holds: the canonical ordering keeps
// per-row offsets and counts in 32 bits.
constexpr int64_t kMaxPairs = (1ll << 32) - (1ll << 24);

// ------------------------------------------------------- per-row statistics
// Derived data of one relation, built by the prep kernel in the workspace.
// Every bound is rounded so that it over-estimates the quantity it bounds.
struct Prep {
  void* q = nullptr;        // operand copy, npad rows of qld bytes (zero padded)
  int64_t qld = 0;          // bytes per operand row (dpad * element size)
  int64_t npad = 0;         // rows rounded up to kTile
  double* nrm2 = nullptr;   // |x|^2 in float64 (summation error <= gamma_d)
  float* h = nullptr;       // fl32(|x|^2) / 2: accumulator initial value
  float* qnorm = nullptr;   // |q~| rounded up (q~ = value the operand encodes)
  float* rho = nullptr;     // |x - q~| rounded up
  float* dh = nullptr;      // | |x|^2/2 - h | rounded up
  float* xnorm = nullptr;   // |x| rounded up
  int* qlsb = nullptr;      // min exponent of the lowest set bit over q~
  int* hlsb = nullptr;      // exponent of the lowest set bit of h
  int* mlsb = nullptr;      // min exponent of the lowest set bit over x
  int* sexp = nullptr;      // FP8 row scale: q~ = E4M3(code) * 2^sexp
};

// Reductions of Prep over all rows of a relation.
struct RelStats {
  float h_max, qnorm_max, rho_max, dh_max, xnorm_max;
  int qlsb_min, hlsb_min, mlsb_min;
  int nonfinite;  // number of non-finite input values
  int pad[7];
};

// ---------------------------------------------------------------- helpers
__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

inline int elem_bytes(dl_prec p) {
  return p == DL_FP32 ? 4 : (p == DL_FP8 ? 1 : 2);
}
inline int64_t dpad_of(int d, dl_prec p) {
  return round_up(d, kChunkBytes / elem_bytes(p));
}

// Counting-accurate gamma_n = n u / (1 - n u) (Higham, Accuracy and Stability
// of Numerical Algorithms, Lemma 3.1).
__host__ __device__ inline double gamma_n(double n, double u) { return n * u / (1.0 - n * u); }

// Order-preserving 32-bit keys of floats (unsigned order = float order;
// -inf maps to 0x007fffff, NaNs to the ends), and back.
__host__ __device__ inline uint32_t order_key(float f) {
  const uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float key_float(uint32_t k) {
  return __builtin_bit_cast(float, (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Wave-wide comparison masks straight from the vector compare (lane l's bit
// is set when its comparison holds; inactive lanes read 0).  Written with
// the compare builtins rather than a ballot of a bool, which the compiler
// lowers through a per-lane 0/1 value and a second compare.
constexpr int kCmpUGE = 35;  // unsigned >=
constexpr int kCmpOGE = 3;   // ordered >= (false for NaN)
constexpr int kCmpULT = 36;  // unsigned <
constexpr int kCmpUGE_F = 11;  // unordered or >=
__device__ inline uint64_t mask_ge(uint32_t a, uint32_t b) { return __builtin_amdgcn_uicmp(a, b, kCmpUGE); }
__device__ inline uint64_t mask_ge(float a, float b) { return __builtin_amdgcn_fcmpf(a, b, kCmpOGE); }
__device__ inline uint64_t mask_lt(uint64_t a, uint64_t b) { return __builtin_amdgcn_uicmpl(a, b, kCmpULT); }
// a >= b or either is NaN: a pre-test that passes whatever a NaN hides
__device__ inline uint64_t mask_uge(float a, float b) { return __builtin_amdgcn_fcmpf(a, b, kCmpUGE_F); }
// Largest of four floats, NaN if any is NaN (two three-input maximum
// instructions; the NaN-ignoring fmaxf costs two more per call here, to
// quiet signalling NaNs the matrix cores never produce)
__device__ inline float max4_nan(float a, float b, float c, float d) {
  return __builtin_elementwise_maximum(__builtin_elementwise_maximum(a, b), __builtin_elementwise_maximum(c, d));
}
// lanes below n (n uniform)
__device__ inline uint64_t lanes_below(int n) {
  return n >= 64 ? ~0ull : n <= 0 ? 0ull : (1ull << n) - 1ull;
}

// float nearest to x from above / below (x finite or +-inf).
__device__ inline float f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}
__device__ inline float f32_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}

// Exponent of the lowest set bit of a finite float (kLsbNone for zero):
// v is an integer multiple of 2^lsb_exp(v).
__device__ inline int lsb_exp(float v) {
  uint32_t b = __float_as_uint(v) & 0x7fffffffu;
  if (b == 0) return kLsbNone;
  uint32_t e = b >> 23, m = b & 0x7fffffu;
  if (e == 0) return -149 + __builtin_ctz(m);
  m |= 0x800000u;
  return (int)e - 150 + __builtin_ctz(m);
}

// ------------------------------------------------- operand encodings (RNE)
// bfloat16: round to nearest even; results that would be subnormal flush to
// zero and results that would overflow saturate at the largest finite value.
// The encoded value is what the matrix core multiplies; the residual |x - q~|
// accounts for every difference.
__device__ inline uint16_t enc_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  uint16_t h = (uint16_t)(r >> 16);
  uint16_t mag = h & 0x7fffu;
  if (mag >= 0x7f80u) h = (uint16_t)((h & 0x8000u) | 0x7f7fu);  // saturate
  if ((mag >> 7) == 0) h = (uint16_t)(h & 0x8000u);              // flush subnormal
  return h;
}
__device__ inline float dec_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// IEEE half: round to nearest even, saturating at 65504, subnormals flushed.
__device__ inline uint16_t enc_f16(float x) {
  float a = fabsf(x);
  _Float16 hv;
  if (a >= 65504.0f) hv = (_Float16)copysignf(65504.0f, x);
  else hv = (_Float16)x;
  uint16_t bits = __builtin_bit_cast(uint16_t, hv);
  if (((bits >> 10) & 0x1fu) == 0) bits &= 0x8000u;  // flush subnormal
  return bits;
}
__device__ inline float dec_f16(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// OCP FP8 E4M3 (bias 7, no infinities, 448 largest finite).  Normal values
// only: magnitudes that would round below 2^-6 flush to zero, larger ones
// saturate at 448.  Input must already be scaled into range.
__device__ inline uint8_t enc_e4m3(float y) {
  uint32_t s = (__float_as_uint(y) >> 24) & 0x80u;
  float a = fabsf(y);
  if (!(a >= 0.015625f)) return (uint8_t)s;  // below 2^-6 (or NaN): zero
  int e;
  float f = frexpf(a, &e);            // a = f 2^e, f in [0.5, 1)
  float m = f * 16.0f - 8.0f;         // 3 fraction bits: (2f - 1) * 8
  float q = rintf(m);                 // nearest, ties to even
  int E = e - 1;                      // a = (1 + m/8) 2^E
  if (q >= 8.0f) { q = 0.0f; E += 1; }
  int field = E + 7;
  if (field > 15 || (field == 15 && q > 6.0f)) { field = 15; q = 6.0f; }  // 448
  return (uint8_t)(s | ((uint32_t)field << 3) | (uint32_t)q);
}
__device__ inline float dec_e4m3(uint8_t c) {
  int field = (c >> 3) & 0xf, q = c & 7;
  float v = field == 0 ? ldexpf((float)q, -9) : ldexpf(1.0f + q * 0.125f, field - 7);
  return (c & 0x80) ? -v : v;
}

// Canonical float64 squared distance: separately rounded subtract, multiply
// and add in increasing k (no contraction into fused multiply-add).
__device__ inline double canonical_d2(const float* __restrict__ a, const float* __restrict__ b, int d) {
#pragma clang fp contract(off)
  double s = 0.0;
  for (int k = 0; k < d; ++k) {
    double t = (double)a[k] - (double)b[k];
    s = s + t * t;
  }
  return s;
}

// Carves 256-byte aligned pieces off a buffer; with a null base it only
// counts the bytes (for workspace-size queries).
struct Bump {
  uint8_t* base;
  size_t off = 0;
  explicit Bump(void* b) : base(static_cast<uint8_t*>(b)) {}
  template <class T>
  T* take(int64_t count) {
    off = (size_t)round_up((int64_t)off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (size_t)count * sizeof(T);
    return p;
  }
};

// ------------------------------------------------------- error reporting
struct Error {
  dl_status code;
  std::string msg;
};

}  // namespace dl

// Context: small host-side state, no device memory.
struct dl_ctx {
  int device = 0;
  std::string err;
  size_t required_ws = 0;
  int64_t* pinned = nullptr;  // small pinned host buffer for counts
  bool timing = false;
  // per stage: pending (start, stop) event pairs and accumulated results
  struct Rec { hipEvent_t a, b; int stage; };
  std::vector<Rec>* pending = nullptr;
  double stage_ms[DL_NUM_STAGES] = {0};
  int64_t stage_calls[DL_NUM_STAGES] = {0};
  int cu_count = 256;
  void* scratch = nullptr;  // this device's fixed scratch (dl_join_eps_noalloc)
  hipError_t scratch_err = hipSuccess;
};
