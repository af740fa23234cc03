// join_params.hpp -- launch parameters shared by the join kernels and the
// C ABI layer.
#pragma once

#include "dl_internal.hpp"

namespace dl {

// Candidate pass on the matrix cores (join_mfma.hip).
struct CandParams {
  const uint8_t* qa;   // R operand rows (qld bytes each, npad rows)
  const uint8_t* qb;   // S operand rows
  int64_t qld;         // bytes per operand row (multiple of kChunkBytes)
  int nchunks;         // qld / kChunkBytes
  const float* hb;     // S accumulator init h_j (npadS)
  const int* sexa;     // FP8 row scales of R / S
  const int* sexb;
  int64_t nR, nS;      // real rows
  int64_t nTR, nTS;    // tiles
  int self_join;       // eps: keep j > i only; band: exclude j == i when excl
  int exclude_self;
  // tile order (eps mode)
  int GM;              // row tiles per group
  int64_t ngroups;
  int64_t nlogical;    // logical tiles incl. skipped ones
  // 32-bit division by the tile-order divisors (valid when small32): the
  // group size GM * nTS, GM, and the last group's height
  int small32;
  uint32_t dv_grp_m, dv_grp_s1, dv_grp_s2;
  uint32_t dv_gm_m, dv_gm_s1, dv_gm_s2;
  uint32_t dv_gl_m, dv_gl_s1, dv_gl_s2;
  // eps mode
  const float* thr;    // per R row (npadR)
  unsigned long long* ccount;  // candidate counter
  uint2* cand;         // (i, j) records
  float* candp;        // P~ of each record (null: not kept)
  int64_t ccap;
  // band mode
  int P;               // S splits
  int64_t tps;         // S tiles per split
  int k;
  int cap;             // band entries per (row, split)
  int retight;         // entries appended to a row between tightenings
  int limit;           // highest trigger; a count reaching it forces a round
  int batch;           // queued rows that start a tightening round
  uint32_t* gkey;      // per row: largest band threshold of any split (order key)
  int flood;           // 1: every threshold starts at -inf (else from gkey)
  const float* marg;   // E_i per R row
  uint2* band;         // (P~ bits, j): [(row * P + split) * cap + slot]
  int* bcount;         // [row * P + split]
  int* overflow;       // set when a band exceeds cap - 256
  // band mode over the tiles of an index (nullable): bit tj of row tile
  // ti's words surv[ti * sw ..] set when (ti, tj) may hold a row's top-k
  // neighbour (other tiles are skipped); jmap[j] = the index in S that band
  // entries carry for column j of the ordered S
  const uint32_t* surv;
  int64_t sw;
  const uint32_t* jmap;
  const int* gate;     // nonzero: invalid input, the kernel does nothing
  // eps mode over a tile list (index-pruned join): (ti, tj) entries and the
  // device-side count; null = every tile
  const uint2* tiles;
  const unsigned long long* ntiles;
  int64_t list_all;    // nonzero: walk the list only if 2 * *ntiles < list_all, else the full grid
  // mark mode: bit (tile tj, row i) at mark[tj * mark_words + i / 32]
  uint32_t* mark;
  int64_t mark_words;
  // nearest mode: per row, the maximum of (order key of P~ << 32 | ~column)
  unsigned long long* argkey;
  // eps mode (nullable, at most 64 K-steps): per tile of each operand, bit s
  // set when some row of the tile has a nonzero byte in K-step s.  A step
  // that is zero in every row of either tile adds only zero products and is
  // skipped.
  const uint64_t* kmaskA;
  const uint64_t* kmaskB;
};

// eps-join recheck (recheck.hip).
struct RecheckParams {
  const float* R; int64_t ldr;
  const float* S; int64_t lds;
  int d;
  const uint2* cand; const unsigned long long* ccount; int64_t ccap;
  const float* candp;   // P~ of each candidate, or null
  const int* pexR;      // per R row: the candidate pass computed P~ exactly
  const double* nrm2R;  // |a|^2 per R row (float64)
  const float* xnR; const int* mlR;
  const float* xnS; const int* mlS;
  double T;
  const double* Trow;  // per-row thresholds (device) or null for T
  int bj;  // bits of j in the output key
  unsigned long long* keys; float* dist; unsigned long long* ocount;
  unsigned long long* nties;
  // index-pruned join: candidates are rows of the permuted operand copies;
  // permR / permS give each one's row in R / S (null: no permutation), and
  // swap orders a self-join's pair as (min, max)
  const uint32_t* permR; const uint32_t* permS;
  int swap;
};

// top-k exact selection (recheck.hip).
struct SelectParams {
  const float* R; int64_t ldr;
  const float* S; int64_t lds;
  int d; int64_t nR;
  uint2* band; const int* bcount; int P; int cap; int k;
  const float* marg;
  const float* xnR; const int* mlR;
  const RelStats* sS;  // S maxima: xnorm_max, mlsb_min
  uint32_t* out_j; float* out_dist;
  unsigned long long* nband; unsigned long long* nties; int* too_many;
  const int* gate;  // nonzero: invalid input, every row is written as padding
  // per row (nullable): rstate 1 once a selection over memory has replaced
  // the row's band P~ by float32 d2; wide 1 when the row had more near-tie
  // contenders than the selection holds (the wide selection takes it)
  int* rstate;
  int* wide;
};

}  // namespace dl
