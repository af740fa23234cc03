// api.hip -- the C ABI of libdlmi.so: validation, workspace layout, launch
// sequencing and status codes.  Kernels live in the other sources.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>
#include <new>

#include "core.hpp"

namespace dl {
// featurize.hip
hipError_t launch_hist_rgb8(const uint8_t*, int64_t, int32_t, int32_t, int32_t, float*, hipStream_t, int);
hipError_t launch_hist_crops(const uint8_t*, int64_t, int32_t, int32_t, const dl_box*, int64_t, int32_t, float*, int*,
                             hipStream_t, int);
hipError_t launch_hist_prep(const uint8_t*, int64_t, int32_t, int32_t, const dl_box*, int64_t, int32_t, float*, int*,
                            dl_prec, const Prep&, RelStats*, hipStream_t, int);
// prep.hip
hipError_t launch_stats_init(RelStats*, hipStream_t);
hipError_t launch_stats_reduce(const Prep&, int64_t, RelStats*, hipStream_t, int);
hipError_t launch_prep(const float*, int64_t, int32_t, int64_t, dl_prec, const Prep&, RelStats*, hipStream_t, int,
                       const uint32_t* perm = nullptr);
hipError_t launch_threshold(const Prep&, int64_t, const RelStats*, int, double, const double*, float*, float*, int*,
                            uint32_t*, hipStream_t);
hipError_t launch_band_seed(const Prep&, int64_t, const float*, int, const float*, uint32_t*, hipStream_t);
}  // namespace dl

#include "join_params.hpp"

namespace dl {
hipError_t launch_cand_eps(dl_prec, CandParams, hipStream_t, int);
hipError_t launch_cand_list(dl_prec, CandParams, hipStream_t, int);
hipError_t launch_cand_mark(dl_prec, CandParams, hipStream_t, int);
hipError_t launch_cand_nearest(dl_prec, CandParams, hipStream_t, int);
// index.hip
hipError_t launch_gather_rows(const float*, int64_t, int64_t, int64_t, int, float*, hipStream_t, int);
int64_t pivot_sort_words(int64_t n, int64_t npiv);
hipError_t launch_pivot_sort(const unsigned long long*, int64_t, int64_t, uint32_t*, uint32_t*, hipStream_t);
hipError_t launch_block_balls_q(const Prep&, int64_t, int, dl_prec, double, float*, double*, hipStream_t,
                                const float* eps_row = nullptr);
hipError_t launch_take_bound(const float*, int, const uint32_t*, int64_t, float*, hipStream_t, int);
hipError_t launch_scatter_rows(const uint32_t*, const float*, int, const uint32_t*, int64_t, uint32_t*, float*,
                               hipStream_t, int);
hipError_t launch_survive(const uint32_t*, int64_t, const uint32_t*, int64_t, int64_t, int64_t, int, uint32_t*,
                          int64_t, hipStream_t);
hipError_t launch_group_count(const uint32_t*, int64_t, int64_t, int64_t, int64_t, uint32_t*, hipStream_t, int);
hipError_t launch_group_list(const uint32_t*, int64_t, int64_t, int64_t, int64_t, const uint32_t*, uint2*,
                             unsigned long long*, hipStream_t, int);
int cand_group_rows(int64_t qld, int64_t nTR);
hipError_t launch_tile_kmask(const void*, int64_t, int64_t, uint64_t*, hipStream_t);
hipError_t launch_kstep_count(const uint2*, const unsigned long long*, int64_t, int64_t, int64_t, int,
                              const uint64_t*, const uint64_t*, unsigned long long*, hipStream_t, int);
// plan.hip
int64_t plan_scratch_words(int64_t);
hipError_t launch_select_rows(const int32_t*, int64_t, int32_t, uint32_t*, uint32_t*, unsigned long long*, hipStream_t);
hipError_t launch_filter_pairs(const uint32_t*, const uint32_t*, const float*, int64_t, const int32_t*,
                               const int32_t*, int32_t, uint32_t*, uint32_t*, float*, int64_t, uint32_t*,
                               unsigned long long*, hipStream_t);
hipError_t launch_gather(const float*, int64_t, int, const uint32_t*, int64_t, float*, hipStream_t, int);
hipError_t launch_remap(uint32_t*, uint32_t*, int64_t, const uint32_t*, const uint32_t*, hipStream_t, int);
// sort.hip
hipError_t launch_exclusive_scan(const uint32_t*, int64_t, uint32_t*, uint32_t*, hipStream_t);
int64_t scan_scratch_words(int64_t);
hipError_t launch_cand_band(dl_prec, CandParams, hipStream_t);
hipError_t launch_recheck_eps(const RecheckParams&, hipStream_t, int);
hipError_t launch_pair_d2(const float*, int64_t, int64_t, const float*, int64_t, int64_t, int, const uint32_t*,
                          const uint32_t*, int64_t, double*, int*, hipStream_t, int);
hipError_t launch_topk_select(const SelectParams&, bool, hipStream_t);
hipError_t launch_topk_select_wide(const SelectParams&, hipStream_t);
bool topk_select_small(int);
int64_t row_sort_words(int64_t);
hipError_t row_sort_pairs(const unsigned long long*, const float*, int64_t, int64_t, int, unsigned long long*, float*,
                          uint32_t*, int64_t, uint32_t*, uint32_t*, float*, hipStream_t, int);

// ------------------------------------------------------------ small kernels
__global__ void zero_words_kernel(uint32_t* p, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) p[t] = 0;
}

// Device-side counters of one call (zeroed by a kernel, so the sequence can
// be captured in a graph).
struct Counters {
  unsigned long long cand;   // candidates appended
  unsigned long long out;    // pairs confirmed
  unsigned long long ties;   // float64 decisions
  unsigned long long band;   // top-k band entries
  int bad_index;
  int overflow;
  int too_many;
  int invalid;  // an input relation has a non-finite value or a row norm >= 2^62
  int pad[12];
};
static_assert(sizeof(Counters) == 96, "counter block size");
static_assert(offsetof(Counters, band) == offsetof(Counters, ties) + 8, "ties and band are cleared together");

// Sets *invalid when either relation holds a non-finite value or a row whose
// norm reaches 2^62 (squared distances would overflow float32).  The
// candidate and selection kernels read the flag first and do no work when it
// is set, so bad input costs prep, not a whole join, before the call reports
// DL_ERR_INVALID.
__global__ void input_gate_kernel(const RelStats* r, const RelStats* s, int* invalid) {
  if (threadIdx.x == 0)
    *invalid = (r->nonfinite || s->nonfinite || !(r->xnorm_max < 0x1p62f) || !(s->xnorm_max < 0x1p62f)) ? 1 : 0;
}

// ------------------------------------------------------------ workspace
static Prep carve_prep(Bump& b, int64_t n, int d, dl_prec prec) {
  Prep P;
  P.npad = round_up(n < 1 ? 1 : n, kTile);
  P.qld = dpad_of(d, prec) * elem_bytes(prec);
  P.q = b.take<uint8_t>(P.npad * P.qld);
  P.nrm2 = b.take<double>(P.npad);
  P.h = b.take<float>(P.npad);
  P.qnorm = b.take<float>(P.npad);
  P.rho = b.take<float>(P.npad);
  P.dh = b.take<float>(P.npad);
  P.xnorm = b.take<float>(P.npad);
  P.qlsb = b.take<int>(P.npad);
  P.hlsb = b.take<int>(P.npad);
  P.mlsb = b.take<int>(P.npad);
  P.sexp = b.take<int>(P.npad);
  return P;
}

struct EpsLayout {
  Prep pr, ps;
  RelStats *sr, *ss;
  Counters* cnt;
  float* thr;
  int* pex;
  uint2* cand;
  float* candp;
  unsigned long long *k0, *k1;
  float *v0, *v1;
  uint32_t* rows;  // row-sort scratch
  size_t bytes;
};

// s_ext: the S side (operand copy and statistics) comes from a store and is
// not carved from the workspace.
static EpsLayout layout_eps(void* ws, int64_t nR, int64_t nS, int d, dl_prec prec, bool self, int64_t cap,
                            bool s_ext = false, bool r_ext = false) {
  EpsLayout L;
  Bump b(ws);
  L.cnt = b.take<Counters>(1);
  L.sr = b.take<RelStats>(1);
  L.ss = (self || s_ext) ? L.sr : b.take<RelStats>(1);
  if (r_ext) {  // R's operand copy comes from a store: only its row count matters below
    L.pr = Prep{};
    L.pr.npad = round_up(nR < 1 ? 1 : nR, kTile);
  } else {
    L.pr = carve_prep(b, nR, d, prec);
  }
  L.ps = (self || s_ext) ? L.pr : carve_prep(b, nS, d, prec);
  L.thr = b.take<float>(L.pr.npad);
  L.pex = b.take<int>(L.pr.npad);
  const int64_t c = cap < 1 ? 1 : cap;
  L.cand = b.take<uint2>(c);
  L.candp = b.take<float>(c);
  L.k0 = b.take<unsigned long long>(c);
  L.k1 = b.take<unsigned long long>(c);
  L.v0 = b.take<float>(c);
  L.v1 = b.take<float>(c);
  L.rows = b.take<uint32_t>(row_sort_words(nR < 1 ? 1 : nR));
  L.bytes = round_up((int64_t)b.off, 256);
  return L;
}

struct TopkLayout {
  Prep pr, ps;
  RelStats *sr, *ss;
  Counters* cnt;
  float* marg;
  uint32_t* gkey;  // per row: best band threshold of any split so far (order key)
  uint2* band;
  int* bcount;
  int* rstate;  // per row: the band buffers hold float32 d2 (selection state)
  int* wide;    // per row: more near-tie contenders than the selection holds
  size_t bytes;
};

// S splits for the top-k pass: enough workgroups for every CU, and a count
// that fills the last round of workgroups well.
static int topk_splits(int64_t nR, int64_t nS, int cu_count, int64_t* tps_out) {
  const int64_t nTR = (nR + kTile - 1) / kTile, nTS = (nS + kTile - 1) / kTile;
  const int64_t rows = nTR < 1 ? 1 : nTR;
  int64_t pmin = (int64_t)(cu_count + rows - 1) / rows;
  if (pmin < 1) pmin = 1;
  int64_t best = pmin, best_tps = 1;
  double best_cost = 1e300;
  for (int64_t P0 = pmin; P0 <= 4 * pmin; ++P0) {
    int64_t P = P0 > nTS ? (nTS < 1 ? 1 : nTS) : P0;
    int64_t tps = (nTS + P - 1) / P;
    if (tps < 1) tps = 1;
    P = (nTS + tps - 1) / tps;
    if (P < 1) P = 1;
    // time ~ rounds of workgroups x tiles per workgroup
    const int64_t items = rows * P;
    const double cost = (double)((items + cu_count - 1) / cu_count) * (double)tps;
    if (cost < best_cost - 1e-9) {
      best_cost = cost;
      best = P;
      best_tps = tps;
    }
  }
  if (tps_out) *tps_out = best_tps;
  return (int)best;
}

static TopkLayout layout_topk(void* ws, int64_t nR, int64_t nS, int d, dl_prec prec, bool self, int P, int cap,
                              bool s_ext = false) {
  TopkLayout L;
  Bump b(ws);
  L.cnt = b.take<Counters>(1);
  L.sr = b.take<RelStats>(1);
  L.ss = (self || s_ext) ? L.sr : b.take<RelStats>(1);
  L.pr = carve_prep(b, nR, d, prec);
  L.ps = (self || s_ext) ? L.pr : carve_prep(b, nS, d, prec);
  L.marg = b.take<float>(L.pr.npad);
  L.gkey = b.take<uint32_t>(L.pr.npad);
  L.band = b.take<uint2>((nR < 1 ? 1 : nR) * (int64_t)P * cap);
  L.bcount = b.take<int>((nR < 1 ? 1 : nR) * (int64_t)P);
  L.rstate = b.take<int>(nR < 1 ? 1 : nR);
  L.wide = b.take<int>(nR < 1 ? 1 : nR);
  L.bytes = round_up((int64_t)b.off, 256);
  return L;
}

static int bits_for(int64_t n) {  // bits to hold values 0..n-1 (at least 1)
  int b = 1;
  while (b < 62 && (1ll << b) < n) ++b;
  return b;
}

// Largest double T with sqrt(T) <= eps (sqrt is monotone and correctly
// rounded, so d2 <= T exactly when sqrt(d2) <= eps).
static double threshold_from_eps(double eps);
double eps_threshold(double eps) { return threshold_from_eps(eps); }

static double threshold_from_eps(double eps) {
  if (std::isinf(eps)) return INFINITY;
  double x = eps * eps;
  while (x > 0 && std::sqrt(x) > eps) x = std::nextafter(x, 0.0);
  for (;;) {
    const double y = std::nextafter(x, INFINITY);
    if (std::isinf(y) || std::sqrt(y) > eps) break;
    x = y;
  }
  return x;
}

}  // namespace dl

using namespace dl;

// ---------------------------------------------------------------- helpers
static dl_status fail(dl_ctx* c, dl_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
static dl_status fail(dl_ctx* c, dl_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define DL_HIP(c, call)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail((c), DL_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

namespace {
struct StageTimer {
  dl_ctx* c;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageTimer(dl_ctx* c_, int s, hipStream_t st_) : c(c_), stage(s), st(st_) {
    if (c->timing && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, st);
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) == hipSuccess) {
      (void)hipEventRecord(b, st);
      c->pending->push_back({a, b, stage});
    } else {
      (void)hipEventDestroy(a);
    }
  }
};

dl_status check_mat(dl_ctx* c, const dl_mat& m, const char* name) {
  if (m.n < 0 || m.n >= (1ll << 31)) return fail(c, DL_ERR_INVALID, "%s.n = %lld out of range", name, (long long)m.n);
  if (m.d < 1 || m.d > kMaxDim) return fail(c, DL_ERR_INVALID, "%s.d = %d out of range [1, %d]", name, m.d, kMaxDim);
  if (m.ld < m.d) return fail(c, DL_ERR_INVALID, "%s.ld = %lld < d", name, (long long)m.ld);
  if (m.n > 0 && !m.data) return fail(c, DL_ERR_INVALID, "%s.data is null", name);
  return DL_OK;
}

bool prec_ok(int p) { return p == DL_FP32 || p == DL_BF16 || p == DL_FP16 || p == DL_FP8; }

// Counters and both relations' statistics into the pinned block, then wait:
// the one host synchronisation of a join.
hipError_t readback(dl_ctx* c, const Counters* cnt, const RelStats* sr, const RelStats* ss, hipStream_t st) {
  hipError_t e;
  if ((e = hipMemcpyAsync(c->pinned, cnt, sizeof(Counters), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(c->pinned + 12, sr, sizeof(RelStats), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(c->pinned + 20, ss, sizeof(RelStats), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

// Rows must be finite, and |x| < 2^62 so that every squared distance
// (at most (|a| + |b|)^2 < 2^126) and norm is finite in float32.
dl_status check_inputs(dl_ctx* c) {
  const RelStats* r = reinterpret_cast<const RelStats*>(c->pinned + 12);
  const RelStats* s = reinterpret_cast<const RelStats*>(c->pinned + 20);
  if (r->nonfinite || s->nonfinite)
    return fail(c, DL_ERR_INVALID, "non-finite values in R (%d) or S (%d)", r->nonfinite, s->nonfinite);
  if (!(r->xnorm_max < 0x1p62f) || !(s->xnorm_max < 0x1p62f))
    return fail(c, DL_ERR_INVALID, "row norms up to %g exceed the float32 range of squared distances (2^62)",
                (double)fmaxf(r->xnorm_max, s->xnorm_max));
  return DL_OK;
}
}  // namespace

// ------------------------------------------------------------ fixed scratch
// The workspace of dl_join_eps_noalloc: a file-scope device array, so that
// the call needs no allocation.  Each device holds its own copy at its own
// address, looked up once per device (with that device current) when the
// first context on it is created.  In host code `scratch` names a host-side
// stand-in, never the device memory: only the looked-up address is used.
static __device__ __align__(256) uint8_t scratch[DL_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// The device's scratch address (call with `device` current).  A failed
// lookup is kept and reported by the no-allocation call, not by dl_create.
void* scratch_of(int device, hipError_t* err) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  if (!g_scratch_ptr[device] && g_scratch_err[device] == hipSuccess) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p) g_scratch_ptr[device] = p;
    else g_scratch_err[device] = e == hipSuccess ? hipErrorInvalidSymbol : e;
  }
  *err = g_scratch_err[device];
  return g_scratch_ptr[device];
}
}  // namespace

extern "C" {

const char* dl_version(void) { return "dlmi 0.1 (gfx950)"; }

dl_status dl_create(int device, dl_ctx** out) {
  if (!out) return DL_ERR_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DL_ERR_DEVICE;
  dl_ctx* c = new (std::nothrow) dl_ctx();
  if (!c) return DL_ERR_OOM;
  c->device = device;
  c->pending = new (std::nothrow) std::vector<dl_ctx::Rec>();
  if (hipSetDevice(device) != hipSuccess || !c->pending ||
      hipHostMalloc(reinterpret_cast<void**>(&c->pinned), 256, hipHostMallocDefault) != hipSuccess) {
    delete c->pending;
    delete c;
    return DL_ERR_DEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->cu_count = prop.multiProcessorCount;
  c->scratch = scratch_of(device, &c->scratch_err);
  *out = c;
  return DL_OK;
}

void dl_destroy(dl_ctx* c) {
  if (!c) return;
  if (c->pending) {
    for (auto& r : *c->pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    delete c->pending;
  }
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

const char* dl_last_error(const dl_ctx* c) { return c ? c->err.c_str() : "null context"; }

size_t dl_required_workspace(const dl_ctx* c) { return c ? c->required_ws : 0; }

dl_status dl_set_timing(dl_ctx* c, int enable) {
  if (!c) return DL_ERR_INVALID;
  c->timing = enable != 0;
  return DL_OK;
}

dl_status dl_get_timing(dl_ctx* c, double* ms, int64_t* calls, int reset) {
  if (!c) return DL_ERR_INVALID;
  (void)hipSetDevice(c->device);
  for (auto& r : *c->pending) {
    float t = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      c->stage_ms[r.stage] += t;
      c->stage_calls[r.stage] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c->pending->clear();
  for (int s = 0; s < DL_NUM_STAGES; ++s) {
    if (ms) ms[s] = c->stage_ms[s];
    if (calls) calls[s] = c->stage_calls[s];
    if (reset) {
      c->stage_ms[s] = 0;
      c->stage_calls[s] = 0;
    }
  }
  return DL_OK;
}

dl_status dl_featurize_rgb8(dl_ctx* c, const uint8_t* patches, int64_t n, int32_t h, int32_t w, int32_t bins,
                            float* out_hist, void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  if (n < 0) return fail(c, DL_ERR_INVALID, "n = %lld < 0", (long long)n);
  if (h < 1 || w < 1 || (int64_t)h * w >= (1 << 24)) return fail(c, DL_ERR_INVALID, "bad patch size %dx%d", h, w);
  if (bins < 1 || bins > 256 || 256 % bins != 0 || bins * bins * bins > 4096)
    return fail(c, DL_ERR_INVALID, "bins = %d must divide 256 with bins^3 <= 4096", bins);
  if (n > 0 && (!patches || !out_hist)) return fail(c, DL_ERR_INVALID, "null pointer");
  DL_HIP(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  StageTimer t(c, 0, st);
  DL_HIP(c, launch_hist_rgb8(patches, n, h, w, bins, out_hist, st, c->cu_count));
  return DL_OK;
}

static dl_status check_bins(dl_ctx* c, int32_t bins) {
  if (bins < 1 || bins > 256 || 256 % bins != 0 || bins * bins * bins > 4096)
    return fail(c, DL_ERR_INVALID, "bins = %d must divide 256 with bins^3 <= 4096", bins);
  return DL_OK;
}

dl_status dl_featurize_crops_rgb8(dl_ctx* c, const uint8_t* frames, int64_t nframes, int32_t height, int32_t width,
                                  const dl_box* boxes, int64_t nboxes, int32_t bins, float* out_hist, void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  if (nframes < 0 || nboxes < 0) return fail(c, DL_ERR_INVALID, "negative count");
  if (height < 1 || width < 1 || (int64_t)height * width >= (1 << 24))
    return fail(c, DL_ERR_INVALID, "bad frame size %dx%d", height, width);
  if (dl_status s = check_bins(c, bins)) return s;
  if (nboxes > 0 && (!frames || !boxes || !out_hist)) return fail(c, DL_ERR_INVALID, "null pointer");
  if (nboxes == 0) return DL_OK;
  DL_HIP(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  // bad-box flag: a plain store into the context's pinned host block
  volatile int* bad = reinterpret_cast<volatile int*>(c->pinned + 30);
  *bad = 0;
  {
    StageTimer t(c, 0, st);
    DL_HIP(c, launch_hist_crops(frames, nframes, height, width, boxes, nboxes, bins, out_hist, (int*)bad, st,
                                c->cu_count));
  }
  DL_HIP(c, hipStreamSynchronize(st));
  if (*bad) return fail(c, DL_ERR_INVALID, "a box lies outside its frame (its histogram is all zero)");
  return DL_OK;
}

dl_status dl_pair_d2(dl_ctx* c, dl_mat R, dl_mat S, const uint32_t* pi, const uint32_t* pj, int64_t m, double* out,
                     void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  dl_status s;
  if ((s = check_mat(c, R, "R")) != DL_OK || (s = check_mat(c, S, "S")) != DL_OK) return s;
  if (R.d != S.d) return fail(c, DL_ERR_INVALID, "R.d %d != S.d %d", R.d, S.d);
  if (m < 0) return fail(c, DL_ERR_INVALID, "m < 0");
  if (m > 0 && (!pi || !pj || !out)) return fail(c, DL_ERR_INVALID, "null pointer");
  DL_HIP(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  // out-of-range flag: a plain store into the context's pinned host block
  volatile int* bad = reinterpret_cast<volatile int*>(c->pinned + 31);
  *bad = 0;
  DL_HIP(c, launch_pair_d2(R.data, R.ld, R.n, S.data, S.ld, S.n, R.d, pi, pj, m, out, (int*)bad, st, c->cu_count));
  DL_HIP(c, hipStreamSynchronize(st));
  if (*bad) return fail(c, DL_ERR_INVALID, "pair index out of range");
  return DL_OK;
}

}  // extern "C"

// ------------------------------------------------------------ join cores
// Shared by the plain calls, the store calls and the server.
namespace dl {

// Band entries per (row, split).  A workgroup that runs through more than
// two S tiles defers tightening (rows are tightened in batches, one per
// wave), which needs room for two more tiles above the trigger ceiling, so
// its default buffer is twice as large.
static bool band_defers(int band_cap, int k, int64_t tps) { return tps > 2 && band_cap >= 2 * k + 2 * kTile; }

static int band_cap_of(int32_t band_cap, int k, int64_t tps) {
  if (band_cap <= 0) band_cap = tps > 2 ? 1024 : 512;
  band_cap = (int32_t)round_up(band_cap, 64);
  if (band_cap < 2 * k + kTile) band_cap = (int32_t)round_up(2 * k + kTile, 64);
  return band_cap;
}

// Highest count a row's trigger may be armed at: one tile (two when
// tightening is deferred) below the buffer's end.
static int band_limit_of(int band_cap, int k, int64_t tps) {
  return band_cap - (band_defers(band_cap, k, tps) ? 2 : 1) * kTile;
}

// Entries a row's band buffer grows by before it is tightened again: often
// enough that the running threshold follows the k-th best seen so far
// (fewer hits per tile), rarely enough that selection does not dominate.
static int retight_of(int k, int limit) {
  int x = 4 * k < 64 ? 64 : 4 * k;
  return x > limit ? limit : x;
}

size_t eps_workspace(int64_t nR, int64_t nS, int d, dl_prec prec, bool self, bool s_ext, int64_t cap, bool r_ext) {
  return layout_eps(nullptr, nR, nS, d, prec, self, cap, s_ext, r_ext).bytes;
}

// E4M3 top-k pilot.  The E4M3 margin E_i (about 0.1 on unit vectors) is
// wide next to the spread of unrelated rows' P, so a band seeded at -inf
// keeps most of them until the row has met k close neighbours, and can
// overflow any buffer.  An exact bf16 top-k of R against every
// kPilotStride-th row of S first gives each row a lower bound of its k-th
// largest P (the sample is a subset of S), and the E4M3 pass starts from
// that bound minus E_i.
constexpr int kPilotStride = 16;
static bool pilot_of(dl_prec prec, bool self, int64_t nS, int k) {
  return prec == DL_FP8 && !self && nS >= (int64_t)kPilotStride * kTile && nS / kPilotStride >= 4 * (int64_t)k;
}
static int64_t pilot_rows(int64_t nS) { return (nS + kPilotStride - 1) / kPilotStride; }
static size_t pilot_out_bytes(int64_t nR, int k) { return (size_t)round_up(nR * (int64_t)k * 4, 256); }

size_t topk_workspace(int64_t nR, int64_t nS, int d, dl_prec prec, bool self, bool s_ext, int k, int band_cap,
                      int cu) {
  int64_t tps = 1;
  const int P = topk_splits(nR, nS, cu, &tps);
  size_t b = layout_topk(nullptr, nR, nS, d, prec, self, P, band_cap_of(band_cap, k, tps), s_ext).bytes;
  if (pilot_of(prec, self, nS, k))  // the pilot's outputs and workspace follow
    b += 2 * pilot_out_bytes(nR, k) + topk_workspace(nR, pilot_rows(nS), d, DL_BF16, false, false, k, 0, cu);
  return b;
}

dl_status eps_core(dl_ctx* c, const EpsJob& J, void* ws, size_t ws_bytes, dl_pairs* out, hipStream_t st) {
  const dl_mat &R = J.R, &S = J.S;
  const bool self = J.self, sx = J.ps_ext != nullptr, rx = J.pr_ext != nullptr;
  const dl_prec prec = J.prec;
  out->count = out->candidates = out->ties = 0;
  // candidate capacity from the workspace size
  const size_t fixed = layout_eps(nullptr, R.n, S.n, R.d, prec, self, 1, sx, rx).bytes;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(c, DL_ERR_INVALID, "workspace is not 256-byte aligned");
  if (!ws || ws_bytes < fixed) {
    c->required_ws = layout_eps(nullptr, R.n, S.n, R.d, prec, self, 1 << 20, sx, rx).bytes;
    return fail(c, DL_ERR_WORKSPACE, "workspace of %zu bytes below the minimum %zu", ws_bytes, fixed);
  }
  const size_t per = layout_eps(nullptr, R.n, S.n, R.d, prec, self, 1 << 16, sx, rx).bytes - fixed;
  int64_t cap = (int64_t)((double)(ws_bytes - fixed) / ((double)per / (1 << 16))) - 1024;
  while (cap > 1 && layout_eps(nullptr, R.n, S.n, R.d, prec, self, cap, sx, rx).bytes > ws_bytes) cap = cap * 63 / 64;
  if (cap < 1) cap = 1;
  // the canonical ordering keeps per-row offsets in 32 bits
  if (cap > kMaxPairs) cap = kMaxPairs;
  if (R.n == 0 || S.n == 0) return DL_OK;

  EpsLayout L = layout_eps(ws, R.n, S.n, R.d, prec, self, cap, sx, rx);
  if (rx) {
    L.pr = *J.pr_ext;
    L.sr = J.sr_ext;
    if (self) {
      L.ps = L.pr;
      L.ss = L.sr;
    }
  }
  if (sx) {
    L.ps = *J.ps_ext;
    L.ss = J.ss_ext;
  }
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(L.cnt),
                     (int64_t)(sizeof(Counters) / 4));
  {
    StageTimer t(c, 1, st);
    if (!rx) DL_HIP(c, launch_prep(R.data, R.n, R.d, R.ld, prec, L.pr, L.sr, st, c->cu_count));
    if (!self && !sx) DL_HIP(c, launch_prep(S.data, S.n, S.d, S.ld, prec, L.ps, L.ss, st, c->cu_count));
    hipLaunchKernelGGL(input_gate_kernel, dim3(1), dim3(64), 0, st, L.sr, L.ss, &L.cnt->invalid);
    DL_HIP(c, launch_threshold(L.pr, R.n, L.ss, R.d, J.T, J.Trow, L.thr, nullptr, L.pex, nullptr, st));
  }
  {
    StageTimer t(c, 2, st);
    CandParams p{};
    p.qa = static_cast<const uint8_t*>(L.pr.q);
    p.qb = static_cast<const uint8_t*>(L.ps.q);
    p.qld = L.pr.qld;
    p.nchunks = (int)(L.pr.qld / kChunkBytes);
    p.hb = L.ps.h;
    p.sexa = L.pr.sexp;
    p.sexb = L.ps.sexp;
    p.nR = R.n;
    p.nS = S.n;
    p.self_join = self;
    p.thr = L.thr;
    p.ccount = &L.cnt->cand;
    p.cand = L.cand;
    p.candp = prec == DL_FP8 ? nullptr : L.candp;  // E4M3 stages no P~ (LDS budget)
    p.ccap = cap;
    p.gate = &L.cnt->invalid;
    DL_HIP(c, launch_cand_eps(prec, p, st, c->cu_count));
  }
  const int bj = bits_for(S.n);  // the recheck's keys are i << bj | j
  {
    StageTimer t(c, 3, st);
    RecheckParams q{};
    q.R = R.data; q.ldr = R.ld;
    q.S = S.data; q.lds = S.ld;
    q.d = R.d;
    q.cand = L.cand; q.ccount = &L.cnt->cand; q.ccap = cap;
    q.candp = prec == DL_FP8 ? nullptr : L.candp;
    q.pexR = L.pex;
    q.nrm2R = L.pr.nrm2;
    q.xnR = L.pr.xnorm; q.mlR = L.pr.mlsb;
    q.xnS = L.ps.xnorm; q.mlS = L.ps.mlsb;
    q.T = J.T;
    q.Trow = J.Trow;
    q.bj = bj;
    q.keys = L.k0; q.dist = L.v0; q.ocount = &L.cnt->out; q.nties = &L.cnt->ties;
    DL_HIP(c, launch_recheck_eps(q, st, c->cu_count));
  }
  DL_HIP(c, readback(c, L.cnt, L.sr, L.ss, st));
  const Counters hc = *reinterpret_cast<const Counters*>(c->pinned);
  if (dl_status bad = check_inputs(c)) return bad;
  out->candidates = (int64_t)hc.cand;
  out->ties = (int64_t)hc.ties;
  if ((int64_t)hc.cand > cap && cap == kMaxPairs)
    return fail(c, DL_ERR_CAPACITY, "%llu candidates exceed the %lld one call can order; split R", hc.cand,
                (long long)kMaxPairs);
  if ((int64_t)hc.cand > cap) {
    c->required_ws =
        layout_eps(nullptr, R.n, S.n, R.d, prec, self, (int64_t)hc.cand + (int64_t)hc.cand / 8 + 1024, sx).bytes;
    return fail(c, DL_ERR_WORKSPACE, "%llu candidates exceed the workspace capacity %lld", hc.cand, (long long)cap);
  }
  const int64_t m = (int64_t)hc.out;
  out->count = m;
  {
    StageTimer t(c, 4, st);
    const int64_t w = m < out->capacity ? m : out->capacity;
    DL_HIP(c, row_sort_pairs(L.k0, L.v0, m, R.n, bj, L.k1, L.v1, L.rows, w, out->i, out->j, out->dist, st,
                             c->cu_count));
  }
  if (m > out->capacity)
    return fail(c, DL_ERR_CAPACITY, "%lld pairs exceed the output capacity %lld", (long long)m,
                (long long)out->capacity);
  return DL_OK;
}

dl_status topk_core(dl_ctx* c, const TopkJob& J, void* ws, size_t ws_bytes, uint32_t* out_j, float* out_dist,
                    dl_topk_info* info, hipStream_t st) {
  const dl_mat &R = J.R, &S = J.S;
  const bool self = J.self, sx = J.ps_ext != nullptr;
  const bool excl = self && J.excl;
  const dl_prec prec = J.prec;
  const int k = J.k;
  if (info) info->band_entries = info->ties = 0;
  int64_t tps = 1;
  const int P = topk_splits(R.n, S.n, c->cu_count, &tps);
  const int band_cap = band_cap_of(J.band_cap, k, tps);
  const size_t main_bytes = layout_topk(nullptr, R.n, S.n, R.d, prec, self, P, band_cap, sx).bytes;
  const bool pilot = !J.seed && pilot_of(prec, self, S.n, k);
  const size_t need = pilot ? main_bytes + 2 * pilot_out_bytes(R.n, k) +
                                  topk_workspace(R.n, pilot_rows(S.n), R.d, DL_BF16, false, false, k, 0, c->cu_count)
                            : main_bytes;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(c, DL_ERR_INVALID, "workspace is not 256-byte aligned");
  if (!ws || ws_bytes < need) {
    c->required_ws = need;
    return fail(c, DL_ERR_WORKSPACE, "workspace of %zu bytes below the %zu needed", ws_bytes, need);
  }
  if (R.n == 0) return DL_OK;
  // the pilot (see pilot_of) runs first, in its own part of the workspace
  const float* pilot_dist = nullptr;
  if (pilot) {
    uint8_t* pw = static_cast<uint8_t*>(ws) + main_bytes;
    uint32_t* pj = reinterpret_cast<uint32_t*>(pw);
    float* pd = reinterpret_cast<float*>(pw + pilot_out_bytes(R.n, k));
    uint8_t* pws = pw + 2 * pilot_out_bytes(R.n, k);
    dl_mat Ss = S;
    Ss.n = pilot_rows(S.n);
    Ss.ld = S.ld * kPilotStride;
    const TopkJob Jp{R, Ss, false, false, DL_BF16, nullptr, nullptr, k, 0};
    const dl_status ps = topk_core(c, Jp, pws, ws_bytes - main_bytes - 2 * pilot_out_bytes(R.n, k), pj, pd, nullptr,
                                   st);
    if (ps == DL_OK) pilot_dist = pd;  // otherwise the E4M3 pass starts unseeded
    else if (ps != DL_ERR_WORKSPACE) return ps;
  }
  TopkLayout L = layout_topk(ws, R.n, S.n, R.d, prec, self, P, band_cap, sx);
  if (sx) {
    L.ps = *J.ps_ext;
    L.ss = J.ss_ext;
  }
  const bool rx = J.pr_ext != nullptr;
  if (rx) {
    L.pr = *J.pr_ext;
    L.sr = J.sr_ext;
    if (self) {
      L.ps = L.pr;
      L.ss = L.sr;
    }
  }
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(L.cnt),
                     (int64_t)(sizeof(Counters) / 4));
  hipLaunchKernelGGL(zero_words_kernel, dim3(64), dim3(256), 0, st, reinterpret_cast<uint32_t*>(L.rstate), R.n);
  hipLaunchKernelGGL(zero_words_kernel, dim3(64), dim3(256), 0, st, reinterpret_cast<uint32_t*>(L.wide), R.n);
  if (S.n == 0 || J.surv) {
    // nothing to match (every row is padding), or work items whose tiles
    // the index rules out all (they store no count)
    hipLaunchKernelGGL(zero_words_kernel, dim3(256), dim3(256), 0, st, reinterpret_cast<uint32_t*>(L.bcount),
                       R.n * (int64_t)P);
  }
  {
    StageTimer t(c, 1, st);
    if (!rx) DL_HIP(c, launch_prep(R.data, R.n, R.d, R.ld, prec, L.pr, L.sr, st, c->cu_count));
    if (!self && !sx) DL_HIP(c, launch_prep(S.data, S.n, S.d, S.ld, prec, L.ps, L.ss, st, c->cu_count));
    hipLaunchKernelGGL(input_gate_kernel, dim3(1), dim3(64), 0, st, L.sr, L.ss, &L.cnt->invalid);
    DL_HIP(c, launch_threshold(L.pr, R.n, L.ss, R.d, 0.0, nullptr, nullptr, L.marg, nullptr, L.gkey, st));
    if (pilot_dist) DL_HIP(c, launch_band_seed(L.pr, R.n, pilot_dist, k, L.marg, L.gkey, st));
    if (J.seed) DL_HIP(c, launch_band_seed(L.pr, R.n, J.seed, 1, L.marg, L.gkey, st));
  }
  if (S.n > 0) {
    StageTimer t(c, 2, st);
    CandParams p{};
    p.qa = static_cast<const uint8_t*>(L.pr.q);
    p.qb = static_cast<const uint8_t*>(L.ps.q);
    p.qld = L.pr.qld;
    p.nchunks = (int)(L.pr.qld / kChunkBytes);
    p.hb = L.ps.h;
    p.sexa = L.pr.sexp;
    p.sexb = L.ps.sexp;
    p.nR = R.n;
    p.nS = S.n;
    p.self_join = self;
    p.exclude_self = excl;
    p.P = P;
    p.k = k;
    p.cap = band_cap;
    p.limit = band_limit_of(band_cap, k, tps);
    p.batch = band_defers(band_cap, k, tps) ? 8 : 1;  // one row per wave of the workgroup
    p.retight = retight_of(k, p.limit);
    p.marg = L.marg;
    p.gkey = L.gkey;
    p.flood = (pilot_dist || J.seed) ? 0 : 1;  // (flood_band stores unmapped j: never with jmap)
    p.surv = J.surv;
    p.sw = J.sw;
    p.jmap = J.jmap;
    p.kmaskA = J.kmA;
    p.kmaskB = J.kmB;
    p.band = L.band;
    p.bcount = L.bcount;
    p.overflow = &L.cnt->overflow;
    p.gate = &L.cnt->invalid;
    DL_HIP(c, launch_cand_band(prec, p, st));
  }
  SelectParams q{};
  const bool small_sel = topk_select_small(k);
  {
    StageTimer t(c, 5, st);
    q.R = R.data; q.ldr = R.ld;
    q.S = S.data; q.lds = S.ld;
    q.d = R.d; q.nR = R.n;
    q.band = L.band; q.bcount = L.bcount; q.P = P; q.cap = band_cap; q.k = k;
    q.marg = L.marg;
    q.xnR = L.pr.xnorm; q.mlR = L.pr.mlsb;
    q.sS = L.ss;
    q.out_j = out_j; q.out_dist = out_dist;
    q.nband = &L.cnt->band; q.nties = &L.cnt->ties; q.too_many = &L.cnt->too_many;
    q.gate = &L.cnt->invalid;
    q.rstate = L.rstate;
    q.wide = L.wide;
    DL_HIP(c, launch_topk_select(q, small_sel, st));
  }
  DL_HIP(c, readback(c, L.cnt, L.sr, L.ss, st));
  Counters hc = *reinterpret_cast<const Counters*>(c->pinned);
  if (small_sel && hc.too_many && !hc.overflow) {
    // a row had more near-tie contenders than the small selection holds:
    // select again (the bands are unchanged) with the large one
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(&L.cnt->ties),
                       (int64_t)4);  // ties and band
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(&L.cnt->too_many),
                       (int64_t)1);
    hipLaunchKernelGGL(zero_words_kernel, dim3(64), dim3(256), 0, st, reinterpret_cast<uint32_t*>(L.wide), R.n);
    {
      StageTimer t(c, 5, st);
      DL_HIP(c, launch_topk_select(q, false, st));
    }
    DL_HIP(c, readback(c, L.cnt, L.sr, L.ss, st));
    hc = *reinterpret_cast<const Counters*>(c->pinned);
  }
  if (hc.too_many && !hc.overflow) {
    // rows with more near-tie contenders than the selection holds: the wide
    // selection works on their band buffers in memory (the others are done)
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(&L.cnt->too_many),
                       (int64_t)1);
    {
      StageTimer t(c, 5, st);
      DL_HIP(c, launch_topk_select_wide(q, st));
    }
    DL_HIP(c, readback(c, L.cnt, L.sr, L.ss, st));
    hc = *reinterpret_cast<const Counters*>(c->pinned);
  }
  if (info) {
    info->band_entries = (int64_t)hc.band;
    info->ties = (int64_t)hc.ties;
  }
  if (dl_status bad = check_inputs(c)) return bad;
  if (hc.overflow || hc.too_many) {
    c->required_ws = topk_workspace(R.n, S.n, R.d, prec, self, sx, k, band_cap * 2, c->cu_count);
    return fail(c, DL_ERR_WORKSPACE, "top-k band exceeded its capacity (%s); retry with band_cap %d",
                hc.overflow ? "band buffer" : "near-tie contenders", band_cap * 2);
  }
  return DL_OK;
}

// ------------------------------------------------------------ indexed eps-join
// The index-pruned eps-join (index.hip): pivot assignment and ordering, block
// balls, a bound pass on the matrix cores, and the candidate pass over the
// surviving tiles only; the recheck and the output are the plain join's.

// Pivots: a strided sample of S, about one per 1,024 rows (16 to 4,096).
static int64_t index_pivots(int64_t nS, int32_t want) {
  int64_t p = want > 0 ? want : nS / 1024;
  if (p < 16) p = 16;
  if (p > 4096) p = 4096;
  if (p > nS) p = nS;
  return p;
}
struct IndexLayout {
  uint32_t *permR, *permS;          // operand row -> row of R / S
  float* piv;                       // pivots (P x d)
  Prep ppiv;                        // their operand copy
  RelStats* spiv;
  unsigned long long* argkey;       // nearest pivot of each row (one relation at a time)
  uint32_t* psort;                  // scratch of the ordering by pivot
  float *centS, *centR;             // block centroids
  double *TbS, *TbR;                // (eps + r)^2 per block
  Prep pcS, pcR;                    // their operand copies
  RelStats *scS, *scR;
  float *thrS, *thrR;
  uint32_t *m1, *m2, *surv, *cnt, *off, *sums;
  int64_t m1w, m2w, sw, gm;
  uint2* tiles;
  unsigned long long* ntiles;
  uint64_t *kmR, *kmS;              // K-step masks per tile of the ordered operand copies
  unsigned long long* ksteps;       // K-steps the candidate pass runs
  size_t bytes;
};

static IndexLayout layout_index(void* base, int64_t nR, int64_t nS, int d, dl_prec prec, bool self, int64_t P,
                                int cu) {
  IndexLayout X{};
  Bump b(base);
  const int64_t n = nR > nS ? nR : nS;
  const int64_t nTR = (nR + kTile - 1) / kTile, nTS = (nS + kTile - 1) / kTile;
  X.permR = b.take<uint32_t>(nR);
  X.permS = self ? X.permR : b.take<uint32_t>(nS);
  X.piv = b.take<float>(P * (int64_t)d);
  X.ppiv = carve_prep(b, P, d, prec);
  X.spiv = b.take<RelStats>(1);
  X.argkey = b.take<unsigned long long>(n);
  X.psort = b.take<uint32_t>(pivot_sort_words(n, P));
  X.centS = b.take<float>(nTS * (int64_t)d);
  X.TbS = b.take<double>(nTS);
  X.pcS = carve_prep(b, nTS, d, prec);
  X.scS = b.take<RelStats>(1);
  X.thrS = b.take<float>(X.pcS.npad);
  X.m1w = X.pcS.npad / 32;
  X.m1 = b.take<uint32_t>(nTR * X.m1w);
  if (self) {
    X.centR = X.centS;
    X.TbR = X.TbS;
    X.pcR = X.pcS;
    X.scR = X.scS;
    X.thrR = X.thrS;
    X.m2w = X.m1w;
    X.m2 = X.m1;
  } else {
    X.centR = b.take<float>(nTR * (int64_t)d);
    X.TbR = b.take<double>(nTR);
    X.pcR = carve_prep(b, nTR, d, prec);
    X.scR = b.take<RelStats>(1);
    X.thrR = b.take<float>(X.pcR.npad);
    X.m2w = X.pcR.npad / 32;
    X.m2 = b.take<uint32_t>(nTS * X.m2w);
  }
  X.sw = (nTS + 31) / 32;
  X.surv = b.take<uint32_t>(nTR * X.sw);
  X.gm = cand_group_rows(dpad_of(d, prec) * elem_bytes(prec), nTR);
  const int64_t ncnt = (nTR + X.gm - 1) / X.gm * nTS + 1;  // (group, column tile) counts and the total
  X.cnt = b.take<uint32_t>(ncnt);
  X.off = b.take<uint32_t>(ncnt);
  X.sums = b.take<uint32_t>(scan_scratch_words(ncnt) + 1);
  X.tiles = b.take<uint2>(self ? nTR * (nTR + 1) / 2 : nTR * nTS);
  X.ntiles = b.take<unsigned long long>(1);
  X.kmR = b.take<uint64_t>(nTR);
  X.kmS = self ? X.kmR : b.take<uint64_t>(nTS);
  X.ksteps = b.take<unsigned long long>(1);
  X.bytes = round_up((int64_t)b.off, 256);
  return X;
}

// The index-pruned join applies when eps is finite and each side spans at
// least two tiles (and the tile list fits 32-bit counts).
static bool index_applies(int64_t nR, int64_t nS, double eps) {
  const int64_t nTR = (nR + kTile - 1) / kTile, nTS = (nS + kTile - 1) / kTile;
  return std::isfinite(eps) && nTR >= 2 && nTS >= 2 && nTR * nTS < (1ll << 32) - 1;
}

size_t eps_indexed_workspace(int64_t nR, int64_t nS, int d, dl_prec prec, bool self, int64_t cap, int32_t pivots,
                             int cu) {
  const size_t main = layout_eps(nullptr, nR, nS, d, prec, self, cap).bytes;
  if (!index_applies(nR, nS, 1.0)) return main;
  return main + layout_index(nullptr, nR, nS, d, prec, self, index_pivots(nS, pivots), cu).bytes;
}

// Orders the rows of X (n x d) by nearest pivot: perm[q] = the q-th row in
// (pivot, row) order.  PX, sX: room for X's operand copy (in row order), used
// by the nearest pass only.
static dl_status order_by_pivot(dl_ctx* c, const dl_mat& X, const IndexLayout& I, int64_t P, dl_prec prec,
                                const Prep& PX, RelStats* sX, uint32_t* perm, hipStream_t st) {
  DL_HIP(c, launch_prep(X.data, X.n, X.d, X.ld, prec, PX, sX, st, c->cu_count));
  hipLaunchKernelGGL(zero_words_kernel, dim3(256), dim3(256), 0, st, reinterpret_cast<uint32_t*>(I.argkey),
                     2 * X.n);
  CandParams q{};
  q.qa = static_cast<const uint8_t*>(PX.q);
  q.qb = static_cast<const uint8_t*>(I.ppiv.q);
  q.qld = PX.qld;
  q.nchunks = (int)(PX.qld / kChunkBytes);
  q.hb = I.ppiv.h;
  q.sexa = PX.sexp;
  q.sexb = I.ppiv.sexp;
  q.nR = X.n;
  q.nS = P;
  q.argkey = I.argkey;
  DL_HIP(c, launch_cand_nearest(prec, q, st, c->cu_count));
  DL_HIP(c, launch_pivot_sort(I.argkey, X.n, P, perm, I.psort, st));
  return DL_OK;
}

// Bound pass: rows = the block centroids of one relation (their thresholds
// Tb), columns = the ordered operand rows of the other (prep D, statistics
// sD); marks bit (column tile, block) of m.
static dl_status bound_pass(dl_ctx* c, const float* cent, int64_t nb, const double* Tb, int d, dl_prec prec,
                            const Prep& pc, RelStats* sc, float* thr, const Prep& D, int64_t nD, const RelStats* sD,
                            uint32_t* m, int64_t mw, const int* gate, hipStream_t st) {
  const int64_t nTD = (nD + kTile - 1) / kTile;
  hipLaunchKernelGGL(zero_words_kernel, dim3(256), dim3(256), 0, st, m, nTD * mw);
  DL_HIP(c, launch_prep(cent, nb, d, d, prec, pc, sc, st, c->cu_count));
  DL_HIP(c, launch_threshold(pc, nb, sD, d, 0.0, Tb, thr, nullptr, nullptr, nullptr, st));
  CandParams q{};
  q.qa = static_cast<const uint8_t*>(pc.q);
  q.qb = static_cast<const uint8_t*>(D.q);
  q.qld = pc.qld;
  q.nchunks = (int)(pc.qld / kChunkBytes);
  q.hb = D.h;
  q.sexa = pc.sexp;
  q.sexb = D.sexp;
  q.nR = nb;
  q.nS = nD;
  q.thr = thr;
  q.mark = m;
  q.mark_words = mw;
  q.gate = gate;
  DL_HIP(c, launch_cand_mark(prec, q, st, c->cu_count));
  return DL_OK;
}

dl_status eps_indexed_core(dl_ctx* c, const EpsJob& J, double eps, int32_t pivots, void* ws, size_t ws_bytes,
                           dl_pairs* out, dl_index_info* info, hipStream_t st) {
  const dl_mat &R = J.R, &S = J.S;
  const bool self = J.self;
  const dl_prec prec = J.prec;
  const int d = R.d;
  const int64_t nTR = (R.n + kTile - 1) / kTile, nTS = (S.n + kTile - 1) / kTile;
  const int64_t all_tiles = self ? nTR * (nTR + 1) / 2 : nTR * nTS;
  if (info) {
    info->tiles_total = all_tiles;
    info->tiles_computed = all_tiles;
    info->pivots = 0;
    info->ksteps_per_tile = (int32_t)(dpad_of(d, prec) * elem_bytes(prec) / kChunkBytes);
    info->ksteps_computed = all_tiles * info->ksteps_per_tile;
  }
  if (!index_applies(R.n, S.n, eps)) return eps_core(c, J, ws, ws_bytes, out, st);
  out->count = out->candidates = out->ties = 0;
  const int64_t P = index_pivots(S.n, pivots);
  const size_t xbytes = layout_index(nullptr, R.n, S.n, d, prec, self, P, c->cu_count).bytes;
  // candidate capacity from what the workspace leaves beside the index
  const size_t fixed = layout_eps(nullptr, R.n, S.n, d, prec, self, 1).bytes + xbytes;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(c, DL_ERR_INVALID, "workspace is not 256-byte aligned");
  if (!ws || ws_bytes < fixed) {
    c->required_ws = eps_indexed_workspace(R.n, S.n, d, prec, self, 1 << 20, pivots, c->cu_count);
    return fail(c, DL_ERR_WORKSPACE, "workspace of %zu bytes below the minimum %zu", ws_bytes, fixed);
  }
  const size_t per = layout_eps(nullptr, R.n, S.n, d, prec, self, 1 << 16).bytes -
                     layout_eps(nullptr, R.n, S.n, d, prec, self, 1).bytes;
  int64_t cap = (int64_t)((double)(ws_bytes - fixed) / ((double)per / (1 << 16))) - 1024;
  while (cap > 1 && layout_eps(nullptr, R.n, S.n, d, prec, self, cap).bytes + xbytes > ws_bytes) cap = cap * 63 / 64;
  if (cap < 1) cap = 1;
  if (cap > kMaxPairs) cap = kMaxPairs;
  EpsLayout L = layout_eps(ws, R.n, S.n, d, prec, self, cap);
  IndexLayout I = layout_index(static_cast<uint8_t*>(ws) + L.bytes, R.n, S.n, d, prec, self, P, c->cu_count);
  if (info) info->pivots = (int32_t)P;

  {
    StageTimer t(c, 6, st);
    // pivots, nearest-pivot order of each relation (its operand copy in row
    // order goes where the ordered copy will be)
    DL_HIP(c, launch_gather_rows(S.data, S.ld, S.n / P, P, d, I.piv, st, c->cu_count));
    DL_HIP(c, launch_prep(I.piv, P, d, d, prec, I.ppiv, I.spiv, st, c->cu_count));
    dl_status s = order_by_pivot(c, R, I, P, prec, L.pr, L.sr, I.permR, st);
    if (s == DL_OK && !self) s = order_by_pivot(c, S, I, P, prec, L.ps, L.ss, I.permS, st);
    if (s != DL_OK) return s;
  }
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(L.cnt),
                     (int64_t)(sizeof(Counters) / 4));
  {
    StageTimer t(c, 1, st);
    DL_HIP(c, launch_prep(R.data, R.n, d, R.ld, prec, L.pr, L.sr, st, c->cu_count, I.permR));
    if (!self) DL_HIP(c, launch_prep(S.data, S.n, d, S.ld, prec, L.ps, L.ss, st, c->cu_count, I.permS));
    hipLaunchKernelGGL(input_gate_kernel, dim3(1), dim3(64), 0, st, L.sr, L.ss, &L.cnt->invalid);
    DL_HIP(c, launch_threshold(L.pr, R.n, L.ss, d, J.T, nullptr, L.thr, nullptr, L.pex, nullptr, st));
  }
  // K-step masks: rows ordered by pivot make a tile's rows alike, and bins
  // (elements) that are zero in every row of a tile drop out of its K-steps
  // (at most 64 steps per row)
  const int nsteps = (int)(L.pr.qld / kChunkBytes);
  const bool kmask = nsteps <= 64;
  {
    StageTimer t(c, 6, st);
    if (kmask) {
      DL_HIP(c, launch_tile_kmask(L.pr.q, L.pr.qld, nTR, I.kmR, st));
      if (!self) DL_HIP(c, launch_tile_kmask(L.ps.q, L.ps.qld, nTS, I.kmS, st));
    }
    // block balls and the bound passes (both directions), then the tile list
    // balls from the ordered operand copies (contiguous blocks; the prep's
    // rho bounds what the copy leaves out of each row)
    DL_HIP(c, launch_block_balls_q(L.ps, S.n, d, prec, eps, I.centS, I.TbS, st));
    dl_status s = bound_pass(c, I.centS, nTS, I.TbS, d, prec, I.pcS, I.scS, I.thrS, L.pr, R.n, L.sr, I.m1, I.m1w,
                             &L.cnt->invalid, st);
    if (s == DL_OK && !self) {
      DL_HIP(c, launch_block_balls_q(L.pr, R.n, d, prec, eps, I.centR, I.TbR, st));
      s = bound_pass(c, I.centR, nTR, I.TbR, d, prec, I.pcR, I.scR, I.thrR, L.ps, S.n, L.ss, I.m2, I.m2w,
                     &L.cnt->invalid, st);
    }
    if (s != DL_OK) return s;
    const int64_t ncnt = (nTR + I.gm - 1) / I.gm * nTS;
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, I.cnt + ncnt, (int64_t)1);
    DL_HIP(c, launch_survive(I.m1, I.m1w, I.m2, I.m2w, nTR, nTS, self ? 1 : 0, I.surv, I.sw, st));
    DL_HIP(c, launch_group_count(I.surv, I.sw, nTR, nTS, I.gm, I.cnt, st, c->cu_count));
    DL_HIP(c, launch_exclusive_scan(I.cnt, ncnt + 1, I.off, I.sums, st));
    DL_HIP(c, launch_group_list(I.surv, I.sw, nTR, nTS, I.gm, I.off, I.tiles, I.ntiles, st, c->cu_count));
    DL_HIP(c, hipMemcpyAsync(c->pinned + 28, I.ntiles, 8, hipMemcpyDeviceToHost, st));  // read after the final sync
  }
  // When most tiles survive, the full grid (its order needs no per-tile
  // list reads, which for a list of many millions of entries miss every
  // cache) beats the list; the kernel reads the list's length and picks, so
  // the host does not wait for it.  The ordered operand copies serve either.
  {
    StageTimer t(c, 2, st);
    CandParams p{};
    p.qa = static_cast<const uint8_t*>(L.pr.q);
    p.qb = static_cast<const uint8_t*>(L.ps.q);
    p.qld = L.pr.qld;
    p.nchunks = (int)(L.pr.qld / kChunkBytes);
    p.hb = L.ps.h;
    p.sexa = L.pr.sexp;
    p.sexb = L.ps.sexp;
    p.nR = R.n;
    p.nS = S.n;
    p.self_join = self;
    p.thr = L.thr;
    p.ccount = &L.cnt->cand;
    p.cand = L.cand;
    p.candp = prec == DL_FP8 ? nullptr : L.candp;
    p.ccap = cap;
    p.gate = &L.cnt->invalid;
    if (kmask) {
      p.kmaskA = I.kmR;
      p.kmaskB = I.kmS;
    }
    p.tiles = I.tiles;
    p.ntiles = I.ntiles;
    p.list_all = all_tiles;
    DL_HIP(c, launch_cand_list(prec, p, st, c->cu_count));
  }
  c->pinned[29] = -1;
  if (kmask && info) {
    // the K-steps run, read back with the counters below
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(I.ksteps),
                       (int64_t)2);
    DL_HIP(c, launch_kstep_count(I.tiles, I.ntiles, all_tiles, nTR, nTS, self ? 1 : 0, I.kmR, I.kmS, I.ksteps, st,
                                 c->cu_count));
    DL_HIP(c, hipMemcpyAsync(c->pinned + 29, I.ksteps, 8, hipMemcpyDeviceToHost, st));
  }
  const int bj = bits_for(S.n);
  {
    StageTimer t(c, 3, st);
    RecheckParams q{};
    q.R = R.data; q.ldr = R.ld;
    q.S = S.data; q.lds = S.ld;
    q.d = d;
    q.cand = L.cand; q.ccount = &L.cnt->cand; q.ccap = cap;
    q.candp = prec == DL_FP8 ? nullptr : L.candp;
    q.pexR = L.pex;
    q.nrm2R = L.pr.nrm2;
    q.xnR = L.pr.xnorm; q.mlR = L.pr.mlsb;
    q.xnS = L.ps.xnorm; q.mlS = L.ps.mlsb;
    q.T = J.T;
    q.bj = bj;
    q.keys = L.k0; q.dist = L.v0; q.ocount = &L.cnt->out; q.nties = &L.cnt->ties;
    q.permR = I.permR;
    q.permS = I.permS;
    q.swap = self ? 1 : 0;
    DL_HIP(c, launch_recheck_eps(q, st, c->cu_count));
  }
  DL_HIP(c, readback(c, L.cnt, L.sr, L.ss, st));
  const Counters hc = *reinterpret_cast<const Counters*>(c->pinned);
  if (info) {
    const int64_t survivors = c->pinned[28];
    info->tiles_computed = 2 * survivors < all_tiles ? survivors : all_tiles;
    info->ksteps_per_tile = nsteps;
    info->ksteps_computed = c->pinned[29] >= 0 ? c->pinned[29] : info->tiles_computed * nsteps;
  }
  if (dl_status bad = check_inputs(c)) return bad;
  out->candidates = (int64_t)hc.cand;
  out->ties = (int64_t)hc.ties;
  if ((int64_t)hc.cand > cap && cap == kMaxPairs)
    return fail(c, DL_ERR_CAPACITY, "%llu candidates exceed the %lld one call can order; split R", hc.cand,
                (long long)kMaxPairs);
  if ((int64_t)hc.cand > cap) {
    c->required_ws = eps_indexed_workspace(R.n, S.n, d, prec, self, (int64_t)hc.cand + (int64_t)hc.cand / 8 + 1024,
                                           pivots, c->cu_count);
    return fail(c, DL_ERR_WORKSPACE, "%llu candidates exceed the workspace capacity %lld", hc.cand, (long long)cap);
  }
  const int64_t m = (int64_t)hc.out;
  out->count = m;
  {
    StageTimer t(c, 4, st);
    const int64_t w = m < out->capacity ? m : out->capacity;
    DL_HIP(c, row_sort_pairs(L.k0, L.v0, m, R.n, bj, L.k1, L.v1, L.rows, w, out->i, out->j, out->dist, st,
                             c->cu_count));
  }
  if (m > out->capacity)
    return fail(c, DL_ERR_CAPACITY, "%lld pairs exceed the output capacity %lld", (long long)m,
                (long long)out->capacity);
  return DL_OK;
}

// ------------------------------------------------------------ indexed top-k join
// The top-k join pruned by the same index: each row's k-th distance is
// bounded by an exact top-k against every 16th row of S; a row tile's ball
// with the largest bound of its rows as radius marks, in the bound pass, the
// S tiles that may hold a neighbour of one of its rows; the band pass runs
// over the ordered operand copies and skips every other tile.  Its entries
// carry S's own row indices, so the exact selection (which reads the rows of
// S and breaks ties by index) is the plain join's; the rows of the result
// are scattered back to R's order.

struct TopkIndexLayout {
  Prep pr, ps;           // operand copies in pivot order (ps: not for a self-join)
  RelStats *sr, *ss;
  float* Rp;             // R's float32 rows in pivot order (the selection's R)
  float* sdist;          // the sample top-k: k1 distances per row of R
  uint32_t* sj;
  float* bound;          // per ordered row: its k-th distance bound
  uint32_t* oj;          // the result in pivot order
  float* od;
  size_t bytes;
};

static constexpr int kSampleStride = 16;

static TopkIndexLayout layout_topk_index(void* base, int64_t nR, int64_t nS, int d, dl_prec prec, bool self, int k,
                                         int k1) {
  TopkIndexLayout X{};
  Bump b(base);
  X.sr = b.take<RelStats>(1);
  X.pr = carve_prep(b, nR, d, prec);
  if (self) {
    X.ss = X.sr;
    X.ps = X.pr;
  } else {
    X.ss = b.take<RelStats>(1);
    X.ps = carve_prep(b, nS, d, prec);
  }
  X.Rp = b.take<float>(nR * (int64_t)d);
  X.sdist = b.take<float>(nR * (int64_t)k1);
  X.sj = b.take<uint32_t>(nR * (int64_t)k1);
  X.bound = b.take<float>(nR);
  X.oj = b.take<uint32_t>(nR * (int64_t)k);
  X.od = b.take<float>(nR * (int64_t)k);
  X.bytes = round_up((int64_t)b.off, 256);
  return X;
}

// the index's parts of the workspace: [index | top-k index | sample top-k | main top-k]
struct TopkIndexSizes {
  size_t index, tk, sample, main, total;
};
// The sampled pass runs in the join's own candidate format (never E4M3 here,
// see indexed_topk_prec): bf16's margin is wide on histogram rows, where a
// bf16 sample of an fp16 join would keep tens of near-tie contenders per row.

static TopkIndexSizes topk_index_sizes(int64_t nR, int64_t nS, int d, dl_prec prec, bool self, bool excl, int k,
                                       int band_cap, int64_t P, int cu) {
  TopkIndexSizes z{};
  const int k1 = k + (excl ? 1 : 0);
  z.index = layout_index(nullptr, nR, nS, d, prec, self, P, cu).bytes;
  z.tk = layout_topk_index(nullptr, nR, nS, d, prec, self, k, k1).bytes;
  z.sample = topk_workspace(nR, (nS + kSampleStride - 1) / kSampleStride, d, prec, false, false, k1, 0,
                            cu);
  z.main = topk_workspace(nR, nS, d, prec, self, !self, k, band_cap, cu);
  z.total = z.index + z.tk + z.sample + z.main;
  return z;
}

static bool topk_index_applies(int64_t nR, int64_t nS, int k, bool excl) {
  return index_applies(nR, nS, 1.0) && k + (excl ? 1 : 0) <= 256;
}

size_t topk_indexed_workspace(int64_t nR, int64_t nS, int d, dl_prec prec, bool self, bool excl, int k, int band_cap,
                              int32_t pivots, int cu) {
  const size_t plain = topk_workspace(nR, nS, d, prec, self, false, k, band_cap, cu);
  if (!topk_index_applies(nR, nS, k, excl)) return plain;
  const int64_t P = index_pivots(nS, pivots);
  int64_t tps = 1;
  const int bc = band_cap_of(band_cap, k, (topk_splits(nR, nS, cu, &tps), tps));
  const size_t z = topk_index_sizes(nR, nS, d, prec, self, excl, k, bc, P, cu).total;
  return z > plain ? z : plain;
}

dl_status topk_indexed_core(dl_ctx* c, const TopkJob& J, int32_t pivots, void* ws, size_t ws_bytes, uint32_t* out_j,
                            float* out_dist, dl_topk_info* info, dl_index_info* xinfo, hipStream_t st) {
  const dl_mat &R = J.R, &S = J.S;
  const bool self = J.self, excl = self && J.excl;
  const dl_prec prec = J.prec;
  const int d = R.d, k = J.k, k1 = k + (excl ? 1 : 0);
  const int64_t nTR = (R.n + kTile - 1) / kTile, nTS = (S.n + kTile - 1) / kTile;
  if (xinfo) {
    xinfo->tiles_total = nTR * nTS;
    xinfo->tiles_computed = nTR * nTS;
    xinfo->pivots = 0;
    xinfo->ksteps_per_tile = 0;
    xinfo->ksteps_computed = 0;
  }
  if (!topk_index_applies(R.n, S.n, k, excl)) return topk_core(c, J, ws, ws_bytes, out_j, out_dist, info, st);
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(c, DL_ERR_INVALID, "workspace is not 256-byte aligned");
  const int64_t P = index_pivots(S.n, pivots);
  int64_t tps = 1;
  topk_splits(R.n, S.n, c->cu_count, &tps);
  const int band_cap = band_cap_of(J.band_cap, k, tps);
  const TopkIndexSizes z = topk_index_sizes(R.n, S.n, d, prec, self, excl, k, band_cap, P, c->cu_count);
  if (!ws || ws_bytes < z.total) {
    c->required_ws = z.total;
    return fail(c, DL_ERR_WORKSPACE, "workspace of %zu bytes below the %zu needed", ws_bytes, z.total);
  }
  uint8_t* w = static_cast<uint8_t*>(ws);
  IndexLayout I = layout_index(w, R.n, S.n, d, prec, self, P, c->cu_count);
  TopkIndexLayout X = layout_topk_index(w + z.index, R.n, S.n, d, prec, self, k, k1);
  uint8_t* sws = w + z.index + z.tk;
  uint8_t* mws = sws + z.sample;
  if (xinfo) xinfo->pivots = (int32_t)P;
  const int nsteps = (int)(X.pr.qld / kChunkBytes);
  const bool kmask = nsteps <= 64;

  // each row's k-th distance bound: an exact top-k1 against every 16th row
  // of S (k1 = k + 1 when the row itself is excluded, which the sample may
  // hold); should it fail, the plain join runs instead
  {
    dl_mat Ss = S;
    Ss.n = (S.n + kSampleStride - 1) / kSampleStride;
    Ss.ld = S.ld * kSampleStride;
    const TopkJob Js{R, Ss, false, false, prec, nullptr, nullptr, k1, 0};
    const dl_status ss = topk_core(c, Js, sws, z.sample, X.sj, X.sdist, nullptr, st);
    if (ss == DL_ERR_WORKSPACE) {
      c->err.clear();
      c->required_ws = 0;
      return topk_core(c, J, ws, ws_bytes, out_j, out_dist, info, st);
    }
    if (ss != DL_OK) return ss;
  }
  {
    StageTimer t(c, 6, st);
    // pivots and the nearest-pivot order of each relation (the row-order
    // operand copy goes where the ordered one will be)
    DL_HIP(c, launch_gather_rows(S.data, S.ld, S.n / P, P, d, I.piv, st, c->cu_count));
    DL_HIP(c, launch_prep(I.piv, P, d, d, prec, I.ppiv, I.spiv, st, c->cu_count));
    dl_status s = order_by_pivot(c, R, I, P, prec, X.pr, X.sr, I.permR, st);
    if (s == DL_OK && !self) s = order_by_pivot(c, S, I, P, prec, X.ps, X.ss, I.permS, st);
    if (s != DL_OK) return s;
    DL_HIP(c, launch_prep(R.data, R.n, d, R.ld, prec, X.pr, X.sr, st, c->cu_count, I.permR));
    if (!self) DL_HIP(c, launch_prep(S.data, S.n, d, S.ld, prec, X.ps, X.ss, st, c->cu_count, I.permS));
    DL_HIP(c, launch_gather(R.data, R.ld, d, I.permR, R.n, X.Rp, st, c->cu_count));
    DL_HIP(c, launch_take_bound(X.sdist, k1, I.permR, R.n, X.bound, st, c->cu_count));
    // K-step masks of the ordered operand tiles, as in the index-pruned
    // eps-join (a tile's rows are alike, so many bins are zero in all of them)
    if (kmask) {
      DL_HIP(c, launch_tile_kmask(X.pr.q, X.pr.qld, nTR, I.kmR, st));
      if (!self) DL_HIP(c, launch_tile_kmask(X.ps.q, X.ps.qld, nTS, I.kmS, st));
    }
    // R's row-tile balls with the bound as radius, the bound pass against
    // the ordered S rows (bit (S tile, R tile) of m2), every (ti, tj) kept
    // that m2 marks
    DL_HIP(c, launch_block_balls_q(X.pr, R.n, d, prec, 0.0, I.centR, I.TbR, st, X.bound));
    s = bound_pass(c, I.centR, nTR, I.TbR, d, prec, I.pcR, I.scR, I.thrR, X.ps, S.n, X.ss, I.m2, I.m2w, nullptr, st);
    if (s != DL_OK) return s;
    DL_HIP(c, launch_survive(nullptr, 0, I.m2, I.m2w, nTR, nTS, 0, I.surv, I.sw, st));
  }
  // the band pass over the surviving tiles, the exact selection, the rows
  // back in R's order
  const dl_mat Rp{X.Rp, R.n, d, d};
  const TopkJob Jm{Rp, self ? R : S, self, excl, prec, self ? nullptr : &X.ps, self ? nullptr : X.ss, k, band_cap,
                   &X.pr, X.sr, I.surv, I.sw, self ? I.permR : I.permS, X.bound,
                   kmask ? I.kmR : nullptr, kmask ? (self ? I.kmR : I.kmS) : nullptr};
  const dl_status ms = topk_core(c, Jm, mws, z.main, X.oj, X.od, info, st);
  if (ms == DL_ERR_WORKSPACE && c->required_ws) {
    // a larger band: the whole call's workspace at the capacity asked for
    c->required_ws = z.index + z.tk + z.sample + c->required_ws;
    return ms;
  }
  if (ms != DL_OK) return ms;
  DL_HIP(c, launch_scatter_rows(X.oj, X.od, k, I.permR, R.n, out_j, out_dist, st, c->cu_count));
  if (xinfo) {
    std::vector<uint32_t> h((size_t)(nTR * I.sw));
    std::vector<uint64_t> mR(kmask ? nTR : 0), mS(kmask ? nTS : 0);
    DL_HIP(c, hipMemcpyAsync(h.data(), I.surv, h.size() * 4, hipMemcpyDeviceToHost, st));
    if (kmask) {
      DL_HIP(c, hipMemcpyAsync(mR.data(), I.kmR, nTR * 8, hipMemcpyDeviceToHost, st));
      DL_HIP(c, hipMemcpyAsync(mS.data(), self ? I.kmR : I.kmS, nTS * 8, hipMemcpyDeviceToHost, st));
    }
    DL_HIP(c, hipStreamSynchronize(st));
    int64_t n = 0, ks = 0;
    for (int64_t ti = 0; ti < nTR; ++ti)
      for (int64_t tj = 0; tj < nTS; ++tj)
        if ((h[ti * I.sw + (tj >> 5)] >> (tj & 31)) & 1u) {
          ++n;
          if (kmask) {
            const uint64_t m = mR[ti] & mS[tj];
            ks += m ? __builtin_popcountll(m) : 1;  // a tile runs one step at least
          }
        }
    xinfo->tiles_computed = n;
    if (kmask) {
      xinfo->ksteps_per_tile = nsteps;
      xinfo->ksteps_computed = ks;
    }
  } else {
    DL_HIP(c, hipStreamSynchronize(st));
  }
  return DL_OK;
}

// ------------------------------------------------------------ filtered eps-join
// A label filter before or after the match (plan.hip).
struct FilterLayout {
  uint32_t *rowsR, *rowsS, *scratch;
  unsigned long long* counts;  // rows kept of R and S, pairs kept
  float *Rg, *Sg;              // gathered rows (filter first)
  uint32_t *ti, *tj;           // unfiltered pairs (match first)
  float* td;
  uint8_t* jws;                // the join's workspace
  size_t jws_bytes, bytes;
};

static FilterLayout layout_filter(void* base, int64_t nR, int64_t nS, int d, dl_prec prec, bool self, int plan,
                                  int64_t max_cand, int64_t max_pairs) {
  FilterLayout F{};
  Bump b(base);
  const int64_t n = nR > nS ? nR : nS;
  F.counts = b.take<unsigned long long>(4);
  F.scratch = b.take<uint32_t>(plan_scratch_words(plan == 0 ? n : (max_pairs < 1 ? 1 : max_pairs)));
  if (plan == 0) {
    F.rowsR = b.take<uint32_t>(nR);
    F.rowsS = self ? F.rowsR : b.take<uint32_t>(nS);
    F.Rg = b.take<float>(nR * (int64_t)d);
    F.Sg = self ? F.Rg : b.take<float>(nS * (int64_t)d);
  } else {
    const int64_t m = max_pairs < 1 ? 1 : max_pairs;
    F.ti = b.take<uint32_t>(m);
    F.tj = b.take<uint32_t>(m);
    F.td = b.take<float>(m);
  }
  F.jws_bytes = layout_eps(nullptr, nR, nS, d, prec, self, max_cand < 1 ? 1 : max_cand).bytes;
  F.jws = b.take<uint8_t>((int64_t)F.jws_bytes);
  F.bytes = round_up((int64_t)b.off, 256);
  return F;
}

dl_status eps_filtered_core(dl_ctx* c, const EpsJob& J, const int32_t* labR, const int32_t* labS, int32_t want,
                            int plan, int64_t max_cand, int64_t max_pairs, void* ws, size_t ws_bytes, dl_pairs* out,
                            hipStream_t st) {
  const dl_mat &R = J.R, &S = J.S;
  const bool self = J.self;
  const int d = R.d;
  out->count = out->candidates = out->ties = 0;
  const FilterLayout need = layout_filter(nullptr, R.n, S.n, d, J.prec, self, plan, max_cand, max_pairs);
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(c, DL_ERR_INVALID, "workspace is not 256-byte aligned");
  if (!ws || ws_bytes < need.bytes) {
    c->required_ws = need.bytes;
    return fail(c, DL_ERR_WORKSPACE, "workspace of %zu bytes below the %zu needed", ws_bytes, need.bytes);
  }
  const FilterLayout F = layout_filter(ws, R.n, S.n, d, J.prec, self, plan, max_cand, max_pairs);
  if (plan == 0) {
    // filter first: the rows whose label matches, gathered; the join of those;
    // pairs mapped back to the original rows (increasing maps keep the order)
    DL_HIP(c, launch_select_rows(labR, R.n, want, F.rowsR, F.scratch, F.counts, st));
    if (!self) DL_HIP(c, launch_select_rows(labS, S.n, want, F.rowsS, F.scratch, F.counts + 1, st));
    DL_HIP(c, hipMemcpyAsync(c->pinned + 24, F.counts, 16, hipMemcpyDeviceToHost, st));
    DL_HIP(c, hipStreamSynchronize(st));
    const int64_t mR = c->pinned[24], mS = self ? mR : c->pinned[25];
    DL_HIP(c, launch_gather(R.data, R.ld, d, F.rowsR, mR, F.Rg, st, c->cu_count));
    if (!self) DL_HIP(c, launch_gather(S.data, S.ld, d, F.rowsS, mS, F.Sg, st, c->cu_count));
    EpsJob Jf = J;
    Jf.R = dl_mat{F.Rg, mR, d, d};
    Jf.S = self ? Jf.R : dl_mat{F.Sg, mS, d, d};
    const dl_status s = eps_core(c, Jf, F.jws, F.jws_bytes, out, st);
    if (s != DL_OK) return s;
    const int64_t w = out->count < out->capacity ? out->count : out->capacity;
    DL_HIP(c, launch_remap(out->i, out->j, w, F.rowsR, F.rowsS, st, c->cu_count));
    DL_HIP(c, hipStreamSynchronize(st));
    return DL_OK;
  }
  // match first: the whole join into the workspace, then the pairs whose two
  // rows match the label, in order, into the output
  dl_pairs all{F.ti, F.tj, F.td, max_pairs, 0, 0, 0};
  const dl_status s = eps_core(c, J, F.jws, F.jws_bytes, &all, st);
  if (s == DL_ERR_CAPACITY) {
    c->required_ws = layout_filter(nullptr, R.n, S.n, d, J.prec, self, plan, max_cand, all.count + all.count / 8).bytes;
    return fail(c, DL_ERR_WORKSPACE, "%lld unfiltered pairs exceed the workspace's %lld", (long long)all.count,
                (long long)max_pairs);
  }
  if (s != DL_OK) return s;
  out->candidates = all.candidates;
  out->ties = all.ties;
  DL_HIP(c, launch_filter_pairs(F.ti, F.tj, F.td, all.count, labR, self ? labR : labS, want, out->i, out->j,
                                out->dist, out->capacity, F.scratch, F.counts + 2, st));
  DL_HIP(c, hipMemcpyAsync(c->pinned + 26, F.counts + 2, 8, hipMemcpyDeviceToHost, st));
  DL_HIP(c, hipStreamSynchronize(st));
  const int64_t m = c->pinned[26];
  out->count = m;
  if (m > out->capacity)
    return fail(c, DL_ERR_CAPACITY, "%lld pairs exceed the output capacity %lld", (long long)m,
                (long long)out->capacity);
  return DL_OK;
}

size_t store_bytes(int64_t n, int d, dl_prec prec) {
  Bump b(nullptr);
  b.take<RelStats>(1);
  carve_prep(b, n, d, prec);
  return round_up((int64_t)b.off, 256);
}

}  // namespace dl

// ------------------------------------------------------------ ABI: joins
extern "C" {

size_t dl_join_eps_workspace(int64_t nR, int64_t nS, int32_t d, dl_prec prec, int self_join, int64_t max_cand) {
  if (nR < 0 || d < 1 || d > kMaxDim || !prec_ok(prec) || max_cand < 0) return 0;
  if (self_join) nS = nR;
  return eps_workspace(nR, nS, d, prec, self_join != 0, false, max_cand);
}

dl_status dl_join_eps(dl_ctx* c, dl_mat R, dl_mat S, int self_join, double eps, dl_prec prec, void* ws,
                      size_t ws_bytes, dl_pairs* out, void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  c->required_ws = 0;
  if (self_join) S = R;
  dl_status s;
  if ((s = check_mat(c, R, "R")) != DL_OK || (s = check_mat(c, S, "S")) != DL_OK) return s;
  if (R.d != S.d) return fail(c, DL_ERR_INVALID, "R.d %d != S.d %d", R.d, S.d);
  if (std::isnan(eps) || eps < 0) return fail(c, DL_ERR_INVALID, "eps must be >= 0 (got %g)", eps);
  if (!prec_ok(prec)) return fail(c, DL_ERR_INVALID, "unknown precision %d", (int)prec);
  if (!out || out->capacity < 0) return fail(c, DL_ERR_INVALID, "bad output struct");
  if (out->capacity > 0 && (!out->i || !out->j || !out->dist)) return fail(c, DL_ERR_INVALID, "null output array");
  DL_HIP(c, hipSetDevice(c->device));
  EpsJob J{R, S, self_join != 0, prec, nullptr, nullptr, threshold_from_eps(eps), nullptr};
  return eps_core(c, J, ws, ws_bytes, out, static_cast<hipStream_t>(stream));
}

dl_status dl_join_eps_noalloc(dl_ctx* c, dl_mat R, dl_mat S, int self_join, double eps, dl_prec prec,
                              dl_pairs* out, void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  c->required_ws = 0;
  if (self_join) S = R;
  dl_status s;
  if ((s = check_mat(c, R, "R")) != DL_OK || (s = check_mat(c, S, "S")) != DL_OK) return s;
  if (R.d != S.d) return fail(c, DL_ERR_INVALID, "R.d %d != S.d %d", R.d, S.d);
  if (std::isnan(eps) || eps < 0) return fail(c, DL_ERR_INVALID, "eps must be >= 0 (got %g)", eps);
  if (!prec_ok(prec)) return fail(c, DL_ERR_INVALID, "unknown precision %d", (int)prec);
  if (!out || out->capacity < 0) return fail(c, DL_ERR_INVALID, "bad output struct");
  if (out->capacity > 0 && (!out->i || !out->j || !out->dist)) return fail(c, DL_ERR_INVALID, "null output array");
  if (!c->scratch)
    return fail(c, DL_ERR_DEVICE, "fixed scratch unavailable on device %d: %s", c->device,
                hipGetErrorString(c->scratch_err));
  const size_t need = eps_workspace(R.n, S.n, R.d, prec, self_join != 0, false, 1);
  if (need > (size_t)DL_NOALLOC_SCRATCH_BYTES)
    return fail(c, DL_ERR_WORKSPACE,
                "a %lld x %lld d=%d join needs at least %zu bytes of scratch; the fixed scratch holds %zu "
                "(use dl_join_eps with a workspace)",
                (long long)R.n, (long long)S.n, R.d, need, (size_t)DL_NOALLOC_SCRATCH_BYTES);
  DL_HIP(c, hipSetDevice(c->device));
  EpsJob J{R, S, self_join != 0, prec, nullptr, nullptr, threshold_from_eps(eps), nullptr};
  // no per-stage events either: the call creates nothing
  const bool timing = c->timing;
  c->timing = false;
  const dl_status r = eps_core(c, J, c->scratch, (size_t)DL_NOALLOC_SCRATCH_BYTES, out, static_cast<hipStream_t>(stream));
  c->timing = timing;
  if (r == DL_ERR_WORKSPACE) c->required_ws = 0;  // a larger workspace is not an option here
  return r;
}

size_t dl_join_eps_indexed_workspace(int64_t nR, int64_t nS, int32_t d, dl_prec prec, int self_join,
                                     int64_t max_cand, int32_t pivots) {
  if (nR < 0 || nS < 0 || d < 1 || d > kMaxDim || !prec_ok(prec) || max_cand < 0) return 0;
  if (self_join) nS = nR;
  int cu = 256, dev;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) cu = prop.multiProcessorCount;
  return eps_indexed_workspace(nR, nS, d, prec, self_join != 0, max_cand < 1 ? 1 : max_cand, pivots, cu);
}

dl_status dl_join_eps_indexed(dl_ctx* c, dl_mat R, dl_mat S, int self_join, double eps, dl_prec prec,
                              int32_t pivots, void* ws, size_t ws_bytes, dl_pairs* out, dl_index_info* info,
                              void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  c->required_ws = 0;
  if (self_join) S = R;
  dl_status s;
  if ((s = check_mat(c, R, "R")) != DL_OK || (s = check_mat(c, S, "S")) != DL_OK) return s;
  if (R.d != S.d) return fail(c, DL_ERR_INVALID, "R.d %d != S.d %d", R.d, S.d);
  if (std::isnan(eps) || eps < 0) return fail(c, DL_ERR_INVALID, "eps must be >= 0 (got %g)", eps);
  if (!prec_ok(prec)) return fail(c, DL_ERR_INVALID, "unknown precision %d", (int)prec);
  if (pivots < 0) return fail(c, DL_ERR_INVALID, "pivots = %d < 0", pivots);
  if (!out || out->capacity < 0) return fail(c, DL_ERR_INVALID, "bad output struct");
  if (out->capacity > 0 && (!out->i || !out->j || !out->dist)) return fail(c, DL_ERR_INVALID, "null output array");
  DL_HIP(c, hipSetDevice(c->device));
  EpsJob J{R, S, self_join != 0, prec, nullptr, nullptr, threshold_from_eps(eps), nullptr};
  return eps_indexed_core(c, J, eps, pivots, ws, ws_bytes, out, info, static_cast<hipStream_t>(stream));
}

size_t dl_join_eps_filtered_workspace(int64_t nR, int64_t nS, int32_t d, dl_prec prec, int self_join, int32_t plan,
                                      int64_t max_candidates, int64_t max_pairs) {
  if (nR < 0 || nS < 0 || d < 1 || d > kMaxDim || !prec_ok(prec) || max_candidates < 0 || max_pairs < 0 ||
      (plan != 0 && plan != 1))
    return 0;
  if (self_join) nS = nR;
  return layout_filter(nullptr, nR, nS, d, prec, self_join != 0, plan, max_candidates, max_pairs).bytes;
}

dl_status dl_join_eps_filtered(dl_ctx* c, dl_mat R, dl_mat S, int self_join, double eps, dl_prec prec,
                               const int32_t* labels_R, const int32_t* labels_S, int32_t label, int32_t plan,
                               int64_t max_candidates, int64_t max_pairs, void* ws, size_t ws_bytes, dl_pairs* out,
                               void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  c->required_ws = 0;
  if (self_join) {
    S = R;
    labels_S = labels_R;
  }
  dl_status s;
  if ((s = check_mat(c, R, "R")) != DL_OK || (s = check_mat(c, S, "S")) != DL_OK) return s;
  if (R.d != S.d) return fail(c, DL_ERR_INVALID, "R.d %d != S.d %d", R.d, S.d);
  if (std::isnan(eps) || eps < 0) return fail(c, DL_ERR_INVALID, "eps must be >= 0 (got %g)", eps);
  if (!prec_ok(prec)) return fail(c, DL_ERR_INVALID, "unknown precision %d", (int)prec);
  if (plan != 0 && plan != 1) return fail(c, DL_ERR_INVALID, "plan = %d (0: filter first, 1: match first)", plan);
  if (max_candidates < 1 || max_pairs < 0) return fail(c, DL_ERR_INVALID, "bad capacities");
  if ((R.n > 0 && !labels_R) || (S.n > 0 && !labels_S)) return fail(c, DL_ERR_INVALID, "null labels");
  if (!out || out->capacity < 0) return fail(c, DL_ERR_INVALID, "bad output struct");
  if (out->capacity > 0 && (!out->i || !out->j || !out->dist)) return fail(c, DL_ERR_INVALID, "null output array");
  DL_HIP(c, hipSetDevice(c->device));
  EpsJob J{R, S, self_join != 0, prec, nullptr, nullptr, threshold_from_eps(eps), nullptr};
  return eps_filtered_core(c, J, labels_R, labels_S, label, plan, max_candidates, max_pairs, ws, ws_bytes, out,
                           static_cast<hipStream_t>(stream));
}

size_t dl_join_topk_workspace(int64_t nR, int64_t nS, int32_t d, dl_prec prec, int self_join, int32_t k,
                              int32_t band_cap) {
  if (nR < 0 || nS < 0 || d < 1 || d > kMaxDim || !prec_ok(prec) || k < 1) return 0;
  if (self_join) nS = nR;
  int cu = 256, dev;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) cu = prop.multiProcessorCount;
  return topk_workspace(nR, nS, d, prec, self_join != 0, false, k, band_cap, cu);
}

dl_status dl_join_topk(dl_ctx* c, dl_mat R, dl_mat S, int self_join, int32_t k, int exclude_self, dl_prec prec,
                       int32_t band_cap, void* ws, size_t ws_bytes, uint32_t* out_j, float* out_dist,
                       dl_topk_info* info, void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  c->required_ws = 0;
  if (self_join) S = R;
  dl_status s;
  if ((s = check_mat(c, R, "R")) != DL_OK || (s = check_mat(c, S, "S")) != DL_OK) return s;
  if (R.d != S.d) return fail(c, DL_ERR_INVALID, "R.d %d != S.d %d", R.d, S.d);
  if (k < 1 || k > 256) return fail(c, DL_ERR_INVALID, "k = %d outside [1, 256]", k);
  if (!prec_ok(prec)) return fail(c, DL_ERR_INVALID, "unknown precision %d", (int)prec);
  if (R.n > 0 && (!out_j || !out_dist)) return fail(c, DL_ERR_INVALID, "null output array");
  DL_HIP(c, hipSetDevice(c->device));
  TopkJob J{R, S, self_join != 0, exclude_self != 0, prec, nullptr, nullptr, k, band_cap};
  return topk_core(c, J, ws, ws_bytes, out_j, out_dist, info, static_cast<hipStream_t>(stream));
}

// The indexed top-k join runs E4M3 requests with bf16 candidates.  In pivot
// order the rows near a row fall into few of its band splits, and E4M3's
// wide margin then overflows those splits' buffers: at 200,000 x 200,000,
// d = 128, the E4M3 band needed four capacity retries (155.6 ms against the
// plain E4M3 join's 31.7 ms), while bf16 took none.  The result is exact in
// either format.
static dl_prec indexed_topk_prec(dl_prec prec) { return prec == DL_FP8 ? DL_BF16 : prec; }

size_t dl_join_topk_indexed_workspace(int64_t nR, int64_t nS, int32_t d, dl_prec prec, int self_join,
                                      int exclude_self, int32_t k, int32_t band_cap, int32_t pivots) {
  if (nR < 0 || nS < 0 || d < 1 || d > kMaxDim || !prec_ok(prec) || k < 1 || pivots < 0) return 0;
  if (self_join) nS = nR;
  int cu = 256, dev;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) cu = prop.multiProcessorCount;
  return topk_indexed_workspace(nR, nS, d, indexed_topk_prec(prec), self_join != 0, self_join && exclude_self, k,
                                band_cap, pivots, cu);
}

dl_status dl_join_topk_indexed(dl_ctx* c, dl_mat R, dl_mat S, int self_join, int32_t k, int exclude_self,
                               dl_prec prec, int32_t band_cap, int32_t pivots, void* ws, size_t ws_bytes,
                               uint32_t* out_j, float* out_dist, dl_topk_info* info, dl_index_info* xinfo,
                               void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  c->required_ws = 0;
  if (self_join) S = R;
  dl_status s;
  if ((s = check_mat(c, R, "R")) != DL_OK || (s = check_mat(c, S, "S")) != DL_OK) return s;
  if (R.d != S.d) return fail(c, DL_ERR_INVALID, "R.d %d != S.d %d", R.d, S.d);
  if (k < 1 || k > 256) return fail(c, DL_ERR_INVALID, "k = %d outside [1, 256]", k);
  if (!prec_ok(prec)) return fail(c, DL_ERR_INVALID, "unknown precision %d", (int)prec);
  if (pivots < 0) return fail(c, DL_ERR_INVALID, "pivots = %d < 0", pivots);
  if (R.n > 0 && (!out_j || !out_dist)) return fail(c, DL_ERR_INVALID, "null output array");
  DL_HIP(c, hipSetDevice(c->device));
  TopkJob J{R, S, self_join != 0, exclude_self != 0, indexed_topk_prec(prec), nullptr, nullptr, k, band_cap};
  return topk_indexed_core(c, J, pivots, ws, ws_bytes, out_j, out_dist, info, xinfo, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------ ABI: store
size_t dl_store_bytes(int64_t n, int32_t d, dl_prec prec) {
  if (n < 0 || d < 1 || d > kMaxDim || !prec_ok(prec)) return 0;
  return store_bytes(n, d, prec);
}

dl_status dl_store_create(dl_ctx* c, dl_mat base, dl_prec prec, void* mem, size_t bytes, dl_store** out,
                          void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  if (!out) return fail(c, DL_ERR_INVALID, "null output handle");
  *out = nullptr;
  dl_status s;
  if ((s = check_mat(c, base, "base")) != DL_OK) return s;
  if (!prec_ok(prec)) return fail(c, DL_ERR_INVALID, "unknown precision %d", (int)prec);
  const size_t need = store_bytes(base.n, base.d, prec);
  if (reinterpret_cast<uintptr_t>(mem) & 255) return fail(c, DL_ERR_INVALID, "store memory is not 256-byte aligned");
  if (!mem || bytes < need) {
    c->required_ws = need;
    return fail(c, DL_ERR_WORKSPACE, "store memory of %zu bytes below the %zu needed", bytes, need);
  }
  DL_HIP(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  dl_store* S = new (std::nothrow) dl_store();
  if (!S) return fail(c, DL_ERR_OOM, "host allocation failed");
  Bump b(mem);
  S->stats = b.take<RelStats>(1);
  S->prep = carve_prep(b, base.n, base.d, prec);
  S->base = base;
  S->prec = prec;
  S->device = c->device;
  {
    StageTimer t(c, 1, st);
    hipError_t e = launch_prep(base.data, base.n, base.d, base.ld, prec, S->prep, S->stats, st, c->cu_count);
    if (e != hipSuccess) {
      delete S;
      return fail(c, DL_ERR_DEVICE, "prep: %s", hipGetErrorString(e));
    }
  }
  hipError_t e = hipMemcpyAsync(c->pinned + 12, S->stats, sizeof(RelStats), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->pinned + 20, S->stats, sizeof(RelStats), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete S;
    return fail(c, DL_ERR_DEVICE, "store readback: %s", hipGetErrorString(e));
  }
  if (dl_status bad = check_inputs(c)) {
    delete S;
    return bad;
  }
  *out = S;
  return DL_OK;
}

dl_status dl_store_featurize_rgb8(dl_ctx* c, const uint8_t* pixels, int64_t n, int32_t h, int32_t w,
                                  const dl_box* boxes, int64_t nboxes, int32_t bins, dl_prec prec, float* out_hist,
                                  void* mem, size_t bytes, dl_store** out, void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  if (!out) return fail(c, DL_ERR_INVALID, "null output handle");
  *out = nullptr;
  if (n < 0 || nboxes < 0) return fail(c, DL_ERR_INVALID, "negative count");
  if (h < 1 || w < 1 || (int64_t)h * w >= (1 << 24)) return fail(c, DL_ERR_INVALID, "bad patch size %dx%d", h, w);
  if (dl_status s = check_bins(c, bins)) return s;
  if (!prec_ok(prec)) return fail(c, DL_ERR_INVALID, "unknown precision %d", (int)prec);
  const int64_t rows = boxes ? nboxes : n;
  const int d = bins * bins * bins;
  if (rows >= (1ll << 31)) return fail(c, DL_ERR_INVALID, "%lld rows out of range", (long long)rows);
  if (rows > 0 && (!pixels || !out_hist)) return fail(c, DL_ERR_INVALID, "null pointer");
  const size_t need = store_bytes(rows, d, prec);
  if (reinterpret_cast<uintptr_t>(mem) & 255) return fail(c, DL_ERR_INVALID, "store memory is not 256-byte aligned");
  if (!mem || bytes < need) {
    c->required_ws = need;
    return fail(c, DL_ERR_WORKSPACE, "store memory of %zu bytes below the %zu needed", bytes, need);
  }
  DL_HIP(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  dl_store* S = new (std::nothrow) dl_store();
  if (!S) return fail(c, DL_ERR_OOM, "host allocation failed");
  Bump b(mem);
  S->stats = b.take<RelStats>(1);
  S->prep = carve_prep(b, rows, d, prec);
  S->base = dl_mat{out_hist, rows, d, d};
  S->prec = prec;
  S->device = c->device;
  volatile int* bad = reinterpret_cast<volatile int*>(c->pinned + 30);
  *bad = 0;
  hipError_t e;
  {
    StageTimer t(c, 0, st);
    e = launch_stats_init(S->stats, st);
    if (e == hipSuccess)
      e = launch_hist_prep(pixels, n, h, w, boxes, rows, bins, out_hist, (int*)bad, prec, S->prep, S->stats, st,
                         c->cu_count);
    if (e == hipSuccess) e = launch_stats_reduce(S->prep, rows, S->stats, st, c->cu_count);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(c->pinned + 12, S->stats, sizeof(RelStats), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->pinned + 20, S->stats, sizeof(RelStats), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete S;
    return fail(c, DL_ERR_DEVICE, "featurise into store: %s", hipGetErrorString(e));
  }
  if (*bad) {
    delete S;
    return fail(c, DL_ERR_INVALID, "a box lies outside its frame");
  }
  if (dl_status badin = check_inputs(c)) {
    delete S;
    return badin;
  }
  *out = S;
  return DL_OK;
}

size_t dl_join_eps_store_self_workspace(const dl_store* s, int64_t max_cand) {
  if (!s || max_cand < 0) return 0;
  return eps_workspace(s->base.n, s->base.n, s->base.d, s->prec, true, false, max_cand, true);
}

dl_status dl_join_eps_store_self(dl_ctx* c, const dl_store* store, double eps, void* ws, size_t ws_bytes,
                                 dl_pairs* out, void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  c->required_ws = 0;
  if (!store) return fail(c, DL_ERR_INVALID, "null store");
  if (std::isnan(eps) || eps < 0) return fail(c, DL_ERR_INVALID, "eps must be >= 0 (got %g)", eps);
  if (!out || out->capacity < 0) return fail(c, DL_ERR_INVALID, "bad output struct");
  if (out->capacity > 0 && (!out->i || !out->j || !out->dist)) return fail(c, DL_ERR_INVALID, "null output array");
  DL_HIP(c, hipSetDevice(c->device));
  EpsJob J{store->base, store->base, true, store->prec, nullptr, nullptr, threshold_from_eps(eps), nullptr,
           &store->prep, store->stats};
  return eps_core(c, J, ws, ws_bytes, out, static_cast<hipStream_t>(stream));
}

void dl_store_destroy(dl_store* s) { delete s; }

int64_t dl_store_rows(const dl_store* s) { return s ? s->base.n : -1; }

size_t dl_join_eps_store_workspace(int64_t nR, const dl_store* s, int64_t max_cand) {
  if (!s || nR < 0 || max_cand < 0) return 0;
  return eps_workspace(nR, s->base.n, s->base.d, s->prec, false, true, max_cand);
}

dl_status dl_join_eps_store(dl_ctx* c, dl_mat R, const dl_store* store, double eps, void* ws, size_t ws_bytes,
                            dl_pairs* out, void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  c->required_ws = 0;
  if (!store) return fail(c, DL_ERR_INVALID, "null store");
  dl_status s;
  if ((s = check_mat(c, R, "R")) != DL_OK) return s;
  if (R.d != store->base.d) return fail(c, DL_ERR_INVALID, "R.d %d != store d %d", R.d, store->base.d);
  if (std::isnan(eps) || eps < 0) return fail(c, DL_ERR_INVALID, "eps must be >= 0 (got %g)", eps);
  if (!out || out->capacity < 0) return fail(c, DL_ERR_INVALID, "bad output struct");
  if (out->capacity > 0 && (!out->i || !out->j || !out->dist)) return fail(c, DL_ERR_INVALID, "null output array");
  DL_HIP(c, hipSetDevice(c->device));
  EpsJob J{R, store->base, false, store->prec, &store->prep, store->stats, threshold_from_eps(eps), nullptr};
  return eps_core(c, J, ws, ws_bytes, out, static_cast<hipStream_t>(stream));
}

size_t dl_join_topk_store_workspace(int64_t nR, const dl_store* s, int32_t k, int32_t band_cap) {
  if (!s || nR < 0 || k < 1) return 0;
  int cu = 256, dev;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) cu = prop.multiProcessorCount;
  return topk_workspace(nR, s->base.n, s->base.d, s->prec, false, true, k, band_cap, cu);
}

dl_status dl_join_topk_store(dl_ctx* c, dl_mat R, const dl_store* store, int32_t k, int32_t band_cap, void* ws,
                             size_t ws_bytes, uint32_t* out_j, float* out_dist, dl_topk_info* info, void* stream) {
  if (!c) return DL_ERR_INVALID;
  c->err.clear();
  c->required_ws = 0;
  if (!store) return fail(c, DL_ERR_INVALID, "null store");
  dl_status s;
  if ((s = check_mat(c, R, "R")) != DL_OK) return s;
  if (R.d != store->base.d) return fail(c, DL_ERR_INVALID, "R.d %d != store d %d", R.d, store->base.d);
  if (k < 1 || k > 256) return fail(c, DL_ERR_INVALID, "k = %d outside [1, 256]", k);
  if (R.n > 0 && (!out_j || !out_dist)) return fail(c, DL_ERR_INVALID, "null output array");
  DL_HIP(c, hipSetDevice(c->device));
  TopkJob J{R, store->base, false, false, store->prec, &store->prep, store->stats, k, band_cap};
  return topk_core(c, J, ws, ws_bytes, out_j, out_dist, info, static_cast<hipStream_t>(stream));
}

}  // extern "C"
