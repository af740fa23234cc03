// core.hpp -- join cores shared by the C ABI calls, the store calls and the
// server (api.hip implements them).
#pragma once

#include "dl_internal.hpp"

// A resident relation: the caller's float32 rows plus their operand copy and
// statistics, built once in caller-provided device memory.
struct dl_store {
  int device = 0;
  dl_mat base{};
  dl_prec prec = DL_BF16;
  dl::Prep prep;
  dl::RelStats* stats = nullptr;
};

namespace dl {

// eps-join job: S prepared in the workspace unless ps_ext (a store) is given;
// T is the squared-distance threshold, or Trow (device, one per row of R).
struct EpsJob {
  dl_mat R, S;
  bool self;
  dl_prec prec;
  const Prep* ps_ext;
  RelStats* ss_ext;
  double T;
  const double* Trow;
  // R's operand copy and statistics from a store (a store's self-join): no
  // prep of R
  const Prep* pr_ext;
  RelStats* sr_ext;
};

struct TopkJob {
  dl_mat R, S;
  bool self, excl;
  dl_prec prec;
  const Prep* ps_ext;
  RelStats* ss_ext;
  int k;
  int band_cap;
  // the index-pruned top-k join (all nullable): R's operand copy and
  // statistics built by the caller; the band pass skips the tiles whose bit
  // in surv (sw words per row tile) is clear and stores jmap[j] for column
  // j of the ordered S (the selection then reads S, the relation in its
  // own order); seed: one distance bound per R row that seeds its band
  const Prep* pr_ext;
  RelStats* sr_ext;
  const uint32_t* surv;
  int64_t sw;
  const uint32_t* jmap;
  const float* seed;
  // K-step masks of R's and S's operand tiles (nullable; both or neither)
  const uint64_t* kmA;
  const uint64_t* kmB;
};

size_t eps_workspace(int64_t nR, int64_t nS, int d, dl_prec prec, bool self, bool s_ext, int64_t cap,
                     bool r_ext = false);
size_t topk_workspace(int64_t nR, int64_t nS, int d, dl_prec prec, bool self, bool s_ext, int k, int band_cap,
                      int cu);
size_t store_bytes(int64_t n, int d, dl_prec prec);
dl_status eps_core(dl_ctx* c, const EpsJob& J, void* ws, size_t ws_bytes, dl_pairs* out, hipStream_t st);
dl_status topk_core(dl_ctx* c, const TopkJob& J, void* ws, size_t ws_bytes, uint32_t* out_j, float* out_dist,
                    dl_topk_info* info, hipStream_t st);
double eps_threshold(double eps);

}  // namespace dl
