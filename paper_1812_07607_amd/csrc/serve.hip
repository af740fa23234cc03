// serve.hip -- the serving loop: a resident store probed by batched requests.
//
// Paper: the on-the-fly index similarity join of section "Query Processing"
// keeps one relation resident and probes it with the other; here the resident
// relation is a dl_store (operand copy and statistics built once) and the
// probes are requests of query rows, each an eps-join or a top-k join.
//
// Design.  n_streams worker threads, each with its own context and HIP
// stream.  A worker that is idle takes the request at the head of the FIFO
// queue plus every later queued request with the same mode (and k), up to
// the batch limits, reserves the batch's memory from the caller's arena, and
// runs the whole batch as one join against the store: the query rows are
// packed into one matrix (one eps threshold per row), so many small requests
// share one pass over the store.  If the arena cannot hold the batch it is
// shrunk; if not even the head fits, the worker waits for memory to be
// released (or rejects the head when nothing else holds memory).  Requests
// that arrive while batches are on the GPU are admitted by the next worker
// that frees up: continuous batching.  Per-pair arithmetic does not depend on
// which rows share a batch, so a request's result is the same alone and in a
// mix.  So is its status: a batch that outgrows its output, candidate or band
// capacity does not fail its requests; they go back to the head of the queue
// to run alone, and a request that outgrows them alone runs again with the
// capacity its own run reported.  With two or more streams, the first one is
// a lane for small requests (at most `small_rows` rows): it packs only those,
// so they do not queue behind a long batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "core.hpp"

namespace dl {

static double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over byte offsets of the arena (256-byte granules).
class ArenaAlloc {
 public:
  explicit ArenaAlloc(size_t size) : size_(size) {
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (size_t)round_up((int64_t)(bytes ? bytes : 1), 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (size_t)round_up((int64_t)(bytes ? bytes : 1), 256);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_, used_ = 0, peak_ = 0;
};

struct Batch;

struct Req {
  uint64_t ticket = 0;
  dl_request rq{};
  int state = 0;  // 0 queued, 1 running, 2 done
  dl_status status = DL_OK;
  double t_submit = 0, t_start = 0, t_done = 0;
  const uint32_t *oi = nullptr, *oj = nullptr;
  const float* od = nullptr;
  int64_t count = 0;
  int64_t row_off = 0;
  std::shared_ptr<Batch> batch;
  bool released = false;
  // after a capacity failure: run in a batch of its own, with at least these
  // capacities (0 = the defaults for its rows)
  bool solo = false;
  int retries = 0;
  int64_t pair_hint = 0, cand_hint = 0;  // eps output pairs and candidates
  int32_t band_hint = 0;                 // top-k band entries per row and split
};

struct Batch {
  int64_t id = 0;
  int mode = DL_MODE_EPS, k = 0;
  std::vector<Req*> reqs;
  int64_t rows = 0;
  size_t work_off = 0, work_bytes = 0;  // freed when the batch finishes
  size_t out_off = 0, out_bytes = 0;    // freed when every request is released
  bool work_held = false;
  int live = 0;                         // requests not yet released
  int64_t pair_cap = 0, cand_cap = 0;   // eps capacities of this batch
  int32_t band_cap = 0;                 // top-k band capacity (0 = library default)
  // what a failed run reported: pairs and candidates it found (eps), a band
  // buffer that overflowed (top-k)
  int64_t need_pairs = 0, need_cands = 0;
  bool band_full = false;
};

// Device helpers for one eps batch: start of each request's pairs in the
// (i, j)-sorted output, and batch-row -> request-row conversion of i.
__global__ void eps_demux_starts(const uint32_t* oi, int64_t m, const int64_t* row_off, int nreq,
                                 int64_t* starts) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r > nreq) return;
  const int64_t key = row_off[r];
  int64_t lo = 0, hi = m;  // first t with oi[t] >= key
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)oi[mid] < key) lo = mid + 1; else hi = mid;
  }
  starts[r] = lo;
}

__global__ void eps_demux_rows(uint32_t* oi, int64_t m, const int64_t* row_off, int nreq) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = oi[t];
    int lo = 0, hi = nreq - 1;  // last r with row_off[r] <= i
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (row_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    oi[t] = (uint32_t)(i - row_off[lo]);
  }
}

}  // namespace dl

using namespace dl;

struct dl_server {
  const dl_store* store = nullptr;
  dl_server_config cfg{};
  uint8_t* arena = nullptr;
  ArenaAlloc alloc{0};
  int device = 0;
  int cu = 256;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::map<uint64_t, Req*> reqs;
  std::vector<std::thread> workers;
  bool stopping = false;
  int busy = 0;  // batches running (holding a work block)
  uint64_t next_ticket = 1;
  int64_t next_batch = 1;

  // statistics
  int64_t submitted = 0, completed = 0, rejected = 0, cancelled = 0, batches = 0, batch_reqs = 0;
  double pairs_done = 0, t_first = -1, t_last = 0;
  double batch_ms = 0, batch_pairs = 0;  // summed over successful batch runs
  std::vector<double> lat;

  ArenaAlloc& A() { return alloc; }
};

namespace {

int64_t rows_of(const Req* r) { return r->rq.query.n; }

// Layout of one batch's two arena blocks.  The work block holds the packed
// query rows, request row offsets and output starts, per-row thresholds
// (eps) and the join's workspace; the output block holds the results.  The
// same carving sizes the blocks (null bases) and lays them out, so a batch
// never writes past its blocks.
struct BatchLayout {
  float* R = nullptr;
  int64_t* row_off = nullptr;
  int64_t* starts = nullptr;
  double* Trow = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t *oi = nullptr, *oj = nullptr;
  float* od = nullptr;
  int64_t pair_cap = 0;
  size_t work_bytes = 0, out_bytes = 0;
};

// Capacities of a batch: the defaults for its rows, raised to what its
// requests' earlier runs reported they need.
struct Caps {
  int64_t pairs = 0, cands = 0;
  int32_t band = 0;
};
Caps caps_for(const dl_server* S, int64_t rows, const std::vector<Req*>& reqs) {
  const int64_t ppr = S->cfg.pairs_per_row > 0 ? S->cfg.pairs_per_row : 64;
  Caps c;
  c.pairs = std::max<int64_t>(1 << 16, rows * ppr);
  c.cands = std::max<int64_t>(1 << 17, 2 * rows * ppr);
  c.band = S->cfg.band_cap;
  for (const Req* r : reqs) {
    c.pairs = std::max(c.pairs, r->pair_hint);
    c.cands = std::max(c.cands, r->cand_hint);
    c.band = std::max(c.band, r->band_hint);
  }
  return c;
}

BatchLayout carve_batch(dl_server* S, void* work, void* outb, int mode, int k, int64_t rows, int nreq,
                        const Caps& caps) {
  const dl_store* st = S->store;
  const int d = st->base.d;
  BatchLayout L;
  Bump b(work), o(outb);
  L.R = b.take<float>(rows * (int64_t)d);
  L.row_off = b.take<int64_t>((int64_t)nreq + 1);
  L.starts = b.take<int64_t>((int64_t)nreq + 1);
  if (mode == DL_MODE_EPS) {
    const int64_t pc = caps.pairs, cc = caps.cands;
    L.pair_cap = pc;
    L.Trow = b.take<double>(rows);
    L.ws_bytes = eps_workspace(rows, st->base.n, d, st->prec, false, true, cc);
    L.ws = b.take<uint8_t>((int64_t)L.ws_bytes);
    L.oi = o.take<uint32_t>(pc);
    L.oj = o.take<uint32_t>(pc);
    L.od = o.take<float>(pc);
  } else {
    L.ws_bytes = topk_workspace(rows, st->base.n, d, st->prec, false, true, k, caps.band, S->cu);
    L.ws = b.take<uint8_t>((int64_t)L.ws_bytes);
    L.oj = o.take<uint32_t>(rows * (int64_t)k);
    L.od = o.take<float>(rows * (int64_t)k);
  }
  L.work_bytes = (size_t)round_up((int64_t)b.off, 256);
  L.out_bytes = (size_t)round_up((int64_t)o.off, 256);
  return L;
}

void finish(dl_server* S, Req* r, dl_status st, double t) {
  r->status = st;
  r->state = 2;
  r->t_done = t;
  ++S->completed;
  if (st == DL_OK) {
    S->lat.push_back(r->t_done - r->t_submit);
    S->pairs_done += (double)rows_of(r) * (double)S->store->base.n;
  }
  S->t_last = t;
}

bool small_req(const dl_server* S, const Req* r) { return S->cfg.small_rows > 0 && rows_of(r) <= S->cfg.small_rows; }

// Under the lock: form the next batch (or return null).  Requests whose
// memory can never fit are rejected here.  small_only: the small-request
// lane, which starts from the first small request in the queue and packs
// only small ones.
std::shared_ptr<Batch> take_batch(dl_server* S, bool small_only) {
  for (;;) {
    size_t h = 0;
    if (small_only)
      while (h < S->queue.size() && !small_req(S, S->queue[h])) ++h;
    if (h >= S->queue.size()) return nullptr;
    Req* head = S->queue[h];
    const int mode = head->rq.mode, k = head->rq.k;
    std::vector<Req*> pick{head};
    int64_t rows = rows_of(head);
    for (size_t q = h + 1; q < S->queue.size() && !head->solo; ++q) {
      Req* r = S->queue[q];
      if ((int)pick.size() >= S->cfg.max_batch_requests) break;
      if (r->solo || (small_only && !small_req(S, r))) continue;
      if (r->rq.mode != mode || (mode == DL_MODE_TOPK && r->rq.k != k)) continue;
      if (rows + rows_of(r) > S->cfg.max_batch_rows) continue;
      pick.push_back(r);
      rows += rows_of(r);
    }
    // shrink until the arena has room
    for (;;) {
      const Caps caps = caps_for(S, rows, pick);
      const BatchLayout need = carve_batch(S, nullptr, nullptr, mode, k, rows, (int)pick.size(), caps);
      size_t woff = 0, ooff = 0;
      bool ok = S->alloc.alloc(need.work_bytes, &woff);
      if (ok && !S->alloc.alloc(need.out_bytes, &ooff)) {
        S->alloc.release(woff, need.work_bytes);
        ok = false;
      }
      if (ok) {
        auto b = std::make_shared<Batch>();
        b->id = S->next_batch++;
        b->mode = mode;
        b->k = k;
        b->reqs = pick;
        b->rows = rows;
        b->work_off = woff;
        b->work_bytes = need.work_bytes;
        b->out_off = ooff;
        b->out_bytes = need.out_bytes;
        b->work_held = true;
        b->live = (int)pick.size();
        b->pair_cap = caps.pairs;
        b->cand_cap = caps.cands;
        b->band_cap = caps.band;
        for (Req* r : pick) {
          S->queue.erase(std::find(S->queue.begin(), S->queue.end(), r));
          r->state = 1;
          r->batch = b;
        }
        return b;
      }
      if (pick.size() > 1) {
        rows -= rows_of(pick.back());
        pick.pop_back();
        continue;
      }
      // a request that could not fit even an empty arena is rejected; one
      // that could waits for running batches and released results
      if (round_up((int64_t)need.work_bytes, 256) + round_up((int64_t)need.out_bytes, 256) >
          (int64_t)S->alloc.size()) {
        S->queue.erase(S->queue.begin() + (std::ptrdiff_t)h);
        ++S->rejected;
        finish(S, head, DL_ERR_OOM, now_ms());
        S->cv_done.notify_all();
        break;  // try the next head
      }
      return nullptr;  // wait for memory
    }
  }
}

// Runs one batch on the worker's stream (outside the lock).
dl_status run_batch(dl_server* S, dl_ctx* ctx, hipStream_t st, Batch& b, std::string* err) {
  const dl_store* store = S->store;
  const int d = store->base.d;
  const int nreq = (int)b.reqs.size();
  Caps caps;
  caps.pairs = b.pair_cap;
  caps.cands = b.cand_cap;
  caps.band = b.band_cap;
  BatchLayout L = carve_batch(S, S->arena + b.work_off, S->arena + b.out_off, b.mode, b.k, b.rows, nreq, caps);
  if (L.work_bytes > b.work_bytes || L.out_bytes > b.out_bytes)
    return *err = "batch layout exceeds its blocks", DL_ERR_OOM;
  std::vector<int64_t> hoff(nreq + 1, 0);
  for (int q = 0; q < nreq; ++q) {
    const dl_mat& m = b.reqs[q]->rq.query;
    hoff[q + 1] = hoff[q] + m.n;
    b.reqs[q]->row_off = hoff[q];
    if (m.n > 0 && hipMemcpy2DAsync(L.R + hoff[q] * d, (size_t)d * 4, m.data, (size_t)m.ld * 4, (size_t)d * 4,
                                    (size_t)m.n, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return *err = "query copy failed", DL_ERR_DEVICE;
  }
  if (hipMemcpyAsync(L.row_off, hoff.data(), hoff.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return *err = "offset copy failed", DL_ERR_DEVICE;
  const dl_mat Rm{L.R, b.rows, d, d};
  if (b.mode == DL_MODE_TOPK) {
    const int k = b.k;
    TopkJob J{Rm, store->base, false, false, store->prec, &store->prep, store->stats, k, b.band_cap};
    dl_status s = topk_core(ctx, J, L.ws, L.ws_bytes, L.oj, L.od, nullptr, st);
    if (s != DL_OK) {
      *err = dl_last_error(ctx);
      b.band_full = s == DL_ERR_WORKSPACE && err->find("band buffer") != std::string::npos;
      return s;
    }
    for (Req* r : b.reqs) {
      r->oj = L.oj + r->row_off * k;
      r->od = L.od + r->row_off * k;
      r->count = rows_of(r) * k;
    }
    return DL_OK;
  }
  // eps: one threshold per packed row
  std::vector<double> hT((size_t)b.rows);
  for (Req* r : b.reqs) std::fill_n(hT.begin() + r->row_off, rows_of(r), eps_threshold(r->rq.eps));
  if (b.rows && hipMemcpyAsync(L.Trow, hT.data(), hT.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return *err = "threshold copy failed", DL_ERR_DEVICE;
  dl_pairs P{L.oi, L.oj, L.od, L.pair_cap, 0, 0, 0};
  EpsJob J{Rm, store->base, false, store->prec, &store->prep, store->stats, 0.0, L.Trow};
  dl_status s = eps_core(ctx, J, L.ws, L.ws_bytes, &P, st);
  if (s != DL_OK) {
    b.need_pairs = P.count;
    b.need_cands = P.candidates;
    return *err = dl_last_error(ctx), s;
  }
  hipLaunchKernelGGL(eps_demux_starts, dim3((nreq + 1 + 63) / 64), dim3(64), 0, st, L.oi, P.count, L.row_off, nreq,
                     L.starts);
  if (P.count > 0)
    hipLaunchKernelGGL(eps_demux_rows, dim3((unsigned)std::min<int64_t>((P.count + 255) / 256, 4096)), dim3(256), 0,
                       st, L.oi, P.count, L.row_off, nreq);
  std::vector<int64_t> hs(nreq + 1);
  if (hipMemcpyAsync(hs.data(), L.starts, hs.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return *err = "demux failed", DL_ERR_DEVICE;
  for (int q = 0; q < nreq; ++q) {
    Req* r = b.reqs[q];
    r->oi = L.oi + hs[q];
    r->oj = L.oj + hs[q];
    r->od = L.od + hs[q];
    r->count = hs[q + 1] - hs[q];
  }
  return DL_OK;
}

// Under the lock, after a run that failed for lack of capacity: put the
// batch's requests back at the head of the queue, each to run alone, with
// the capacity a request's own failed run reported.  Returns false (the
// failure stands) for a request that has run alone too often or whose needs
// did not grow.
bool requeue_alone(dl_server* S, Batch& b, dl_status s) {
  const bool eps = b.mode == DL_MODE_EPS;
  if (!(eps ? (s == DL_ERR_CAPACITY || s == DL_ERR_WORKSPACE) : b.band_full)) return false;
  if (b.reqs.size() == 1) {
    // alone already: again with what this run reported
    Req* r = b.reqs[0];
    const int64_t pairs = b.need_pairs + b.need_pairs / 8 + 1024, cands = b.need_cands + b.need_cands / 8 + 1024;
    const int32_t band = std::max<int32_t>(2 * std::max<int32_t>(b.band_cap, 512), 1024);
    const bool grows = eps ? (pairs > b.pair_cap || cands > b.cand_cap) : band > b.band_cap;
    if (++r->retries > 4 || !grows) return false;
    if (eps) {
      r->pair_hint = std::max(r->pair_hint, pairs);
      r->cand_hint = std::max(r->cand_hint, cands);
    } else {
      r->band_hint = band;
    }
  }
  for (auto it = b.reqs.rbegin(); it != b.reqs.rend(); ++it) {
    Req* r = *it;
    r->solo = true;
    r->state = 0;
    r->t_start = 0;
    r->batch.reset();
    S->queue.push_front(r);
  }
  return true;
}

void worker_main(dl_server* S, int idx) {
  // with two or more streams, the first is the small-request lane
  const bool small_lane = idx == 0 && S->cfg.n_streams >= 2 && S->cfg.small_rows > 0;
  if (hipSetDevice(S->device) != hipSuccess) return;
  dl_ctx* ctx = nullptr;
  if (dl_create(S->device, &ctx) != DL_OK) return;
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    dl_destroy(ctx);
    return;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    std::shared_ptr<Batch> b;
    while (!S->stopping && !(b = take_batch(S, small_lane))) S->cv_work.wait(lk);
    if (!b) break;
    ++S->busy;
    ++S->batches;
    S->batch_reqs += (int64_t)b->reqs.size();
    const double t0 = now_ms();
    for (Req* r : b->reqs) r->t_start = t0;
    lk.unlock();
    std::string err;
    dl_status s = run_batch(S, ctx, st, *b, &err);
    if (s == DL_OK && hipStreamSynchronize(st) != hipSuccess) s = DL_ERR_DEVICE;
    const double t1 = now_ms();
    lk.lock();
    if (s != DL_OK && !S->stopping && requeue_alone(S, *b, s)) {
      // nothing of this run is kept: both blocks are free again
      S->alloc.release(b->out_off, b->out_bytes);
    } else {
      for (Req* r : b->reqs) finish(S, r, s, t1);
      if (s == DL_OK) {
        S->batch_ms += t1 - t0;
        S->batch_pairs += (double)b->rows * (double)S->store->base.n;
      }
    }
    // the workspace is free as soon as the batch is done; results stay
    S->alloc.release(b->work_off, b->work_bytes);
    b->work_held = false;
    --S->busy;
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  lk.unlock();
  (void)hipStreamDestroy(st);
  dl_destroy(ctx);
}

// Under the lock: drop a batch's memory once every request is released.
void release_req(dl_server* S, Req* r) {
  r->released = true;
  std::shared_ptr<Batch> b = r->batch;
  r->batch.reset();
  if (b && --b->live == 0) {
    S->alloc.release(b->out_off, b->out_bytes);
    S->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

dl_status dl_server_create(int device, const dl_store* store, const dl_server_config* cfg, void* arena,
                           size_t arena_bytes, dl_server** out) {
  if (!out) return DL_ERR_INVALID;
  *out = nullptr;
  if (!store || !arena || arena_bytes < 4096 || (reinterpret_cast<uintptr_t>(arena) & 255)) return DL_ERR_INVALID;
  dl_server_config c{};
  if (cfg) c = *cfg;
  if (c.n_streams <= 0) c.n_streams = 2;
  if (c.n_streams > 8) c.n_streams = 8;
  if (c.max_batch_requests <= 0) c.max_batch_requests = 64;
  if (c.max_batch_rows <= 0) c.max_batch_rows = 1 << 16;
  if (c.pairs_per_row <= 0) c.pairs_per_row = 64;
  if (c.small_rows == 0) c.small_rows = 4096;
  dl_server* S = new (std::nothrow) dl_server();
  if (!S) return DL_ERR_OOM;
  S->store = store;
  S->cfg = c;
  S->arena = static_cast<uint8_t*>(arena);
  S->alloc = ArenaAlloc(arena_bytes / 256 * 256);
  S->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) S->cu = prop.multiProcessorCount;
  for (int w = 0; w < c.n_streams; ++w) S->workers.emplace_back(worker_main, S, w);
  *out = S;
  return DL_OK;
}

dl_status dl_server_submit(dl_server* S, const dl_request* rq, uint64_t* ticket) {
  if (!S || !rq || !ticket) return DL_ERR_INVALID;
  const dl_mat& q = rq->query;
  if (q.n < 0 || q.d != S->store->base.d || q.ld < q.d || (q.n > 0 && !q.data)) return DL_ERR_INVALID;
  if (rq->mode != DL_MODE_EPS && rq->mode != DL_MODE_TOPK) return DL_ERR_INVALID;
  if (rq->mode == DL_MODE_EPS && (std::isnan(rq->eps) || rq->eps < 0)) return DL_ERR_INVALID;
  if (rq->mode == DL_MODE_TOPK && (rq->k < 1 || rq->k > 256)) return DL_ERR_INVALID;
  Req* r = new (std::nothrow) Req();
  if (!r) return DL_ERR_OOM;
  r->rq = *rq;
  r->t_submit = now_ms();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stopping) {
    delete r;
    return DL_ERR_CANCELLED;
  }
  r->ticket = S->next_ticket++;
  S->reqs[r->ticket] = r;
  ++S->submitted;
  if (S->t_first < 0) S->t_first = r->t_submit;
  if (q.n == 0) {
    finish(S, r, DL_OK, r->t_submit);
  } else {
    S->queue.push_back(r);
    S->cv_work.notify_all();  // the small-request lane may not take it
  }
  *ticket = r->ticket;
  return DL_OK;
}

dl_status dl_server_wait(dl_server* S, uint64_t ticket, int32_t timeout_ms, dl_result* out) {
  if (!S || !out) return DL_ERR_INVALID;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return DL_ERR_INVALID;
  Req* r = it->second;
  auto done = [&] { return r->state == 2; };
  if (timeout_ms < 0) S->cv_done.wait(lk, done);
  else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) return DL_ERR_BUSY;
  std::memset(out, 0, sizeof *out);
  out->status = r->status;
  out->mode = r->rq.mode;
  out->rows = rows_of(r);
  out->k = r->rq.mode == DL_MODE_TOPK ? r->rq.k : 0;
  out->i = r->oi;
  out->j = r->oj;
  out->dist = r->od;
  out->count = r->count;
  out->queued_ms = r->t_start > 0 ? r->t_start - r->t_submit : 0.0;
  out->latency_ms = r->t_done - r->t_submit;
  out->batch_id = r->batch ? r->batch->id : 0;
  out->batch_requests = r->batch ? (int32_t)r->batch->reqs.size() : 0;
  return DL_OK;
}

dl_status dl_server_release(dl_server* S, uint64_t ticket) {
  if (!S) return DL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return DL_ERR_INVALID;
  Req* r = it->second;
  if (r->state != 2) return DL_ERR_BUSY;
  release_req(S, r);
  S->reqs.erase(it);
  delete r;
  return DL_OK;
}

dl_status dl_server_cancel(dl_server* S, uint64_t ticket) {
  if (!S) return DL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return DL_ERR_INVALID;
  Req* r = it->second;
  if (r->state != 0) return DL_ERR_BUSY;
  S->queue.erase(std::find(S->queue.begin(), S->queue.end(), r));
  ++S->cancelled;
  finish(S, r, DL_ERR_CANCELLED, now_ms());
  S->cv_done.notify_all();
  return DL_OK;
}

dl_status dl_server_stats(dl_server* S, dl_server_info* out) {
  if (!S || !out) return DL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(out, 0, sizeof *out);
  out->submitted = S->submitted;
  out->completed = S->completed;
  out->rejected = S->rejected;
  out->cancelled = S->cancelled;
  out->batches = S->batches;
  out->mean_batch_requests = S->batches ? (double)S->batch_reqs / (double)S->batches : 0.0;
  out->pairs_done = S->pairs_done;
  out->span_ms = S->t_first >= 0 ? S->t_last - S->t_first : 0.0;
  out->batch_ms = S->batch_ms;
  out->batch_pairs = S->batch_pairs;
  out->arena_in_use = S->alloc.used();
  out->arena_peak = S->alloc.peak();
  out->queued = (int64_t)S->queue.size();
  if (!S->lat.empty()) {
    std::vector<double> v = S->lat;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      const size_t idx = (size_t)std::min<double>((double)v.size() - 1, std::ceil(q * (double)v.size()) - 1);
      return v[idx];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->max_ms = v.back();
  }
  return DL_OK;
}

dl_status dl_server_reset_stats(dl_server* S) {
  if (!S) return DL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  S->submitted = S->completed = S->rejected = S->cancelled = S->batches = S->batch_reqs = 0;
  S->pairs_done = 0;
  S->batch_ms = S->batch_pairs = 0;
  S->t_first = -1;
  S->t_last = 0;
  S->lat.clear();
  return DL_OK;
}

void dl_server_destroy(dl_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
    // queued requests are cancelled; running batches finish
    for (Req* r : S->queue) finish(S, r, DL_ERR_CANCELLED, now_ms());
    S->queue.clear();
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
  for (auto& t : S->workers) t.join();
  for (auto& kv : S->reqs) delete kv.second;
  delete S;
}

}  // extern "C"
