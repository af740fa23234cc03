/*
 * dlmi.h -- C ABI of the MI355X (gfx950) patch-featurisation and exact
 * similarity-join library (libdlmi.so).
 *
 * The operations follow the patch/query model of Krishnan et al., "DeepLens:
 * Towards a Visual Data Management System" (CIDR 2019):
 *   - a patch carries a dense n-dimensional vector as its data (section
 *     "Iterator API for Patches"); here a relation of patches is a row-major
 *     float32 matrix, one row per patch, and a row index stands for the
 *     patch's image reference;
 *   - featurisation is the colour-histogram transformer (section "Visual
 *     ETL", Transformers);
 *   - the join compares all pairs of two patch collections and returns those
 *     that satisfy a predicate (section "Query Processing", Nested Loop Join),
 *     here the Euclidean threshold predicate of image matching (section
 *     "Derived Data") or the k closest patches (query q1, section "Queries").
 *
 * Conventions for every call:
 *   - Pointers documented as "device" point to memory on the context's GPU;
 *     the library never frees or retains them after the call's GPU work has
 *     finished.  "host" pointers are read or written before the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All GPU work of a call is enqueued on it.  A call that reports a count
 *     synchronises the stream before returning; other results are ready when
 *     the stream reaches the end of the call's work.
 *   - No call allocates device memory except where stated: scratch memory is
 *     the caller's `ws` buffer, sized by the matching *_workspace query.
 *     Workspaces, store memory and server arenas must be 256-byte aligned
 *     (DL_ERR_INVALID otherwise); every allocation of hipMalloc or of the
 *     PyTorch caching allocator is.
 *   - Errors are status codes; dl_last_error() gives a message.  No C++
 *     exception crosses this boundary.  On error, output buffers may hold
 *     partial results.
 *   - The library is thread-safe for distinct contexts; one context must not
 *     be used by two threads at once.
 */
#ifndef DLMI_H
#define DLMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dl_status {
  DL_OK = 0,
  DL_ERR_INVALID = 1,   /* null pointer, bad shape or size, non-finite input */
  DL_ERR_OOM = 2,       /* request does not fit the memory budget            */
  DL_ERR_CAPACITY = 3,  /* output buffer too small: the count says how many   */
  DL_ERR_WORKSPACE = 4, /* `ws` too small: dl_required_workspace() says how much */
  DL_ERR_DEVICE = 5,    /* HIP runtime error                                  */
  DL_ERR_BUSY = 6,      /* server queue full                                  */
  DL_ERR_CANCELLED = 7  /* request cancelled                                  */
} dl_status;

/* Operand format of the candidate pass on the matrix cores.  The emitted
 * results do not depend on it; only speed and the candidate count do. */
typedef enum dl_prec {
  DL_FP32 = 0, /* plain fp32 operands                                    */
  DL_BF16 = 1, /* bfloat16, round to nearest even                        */
  DL_FP16 = 2, /* IEEE half, round to nearest even, saturating           */
  DL_FP8 = 3   /* OCP E4M3 with a power-of-two scale per row             */
} dl_prec;

typedef struct dl_ctx dl_ctx;

/* A relation of patch vectors: n rows of d float32 values, row r at
 * data + r*ld (ld >= d, in elements).  Device memory, borrowed.
 * 0 <= n < 2^31, 1 <= d <= 4096. */
typedef struct dl_mat {
  const float* data;
  int64_t n;
  int32_t d;
  int64_t ld;
} dl_mat;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  Allocates a few bytes of pinned
 * host memory for counts.  The first context on a device also looks up that
 * device's fixed scratch of dl_join_eps_noalloc (device memory the library's
 * code object holds from when it is loaded on the device). */
dl_status dl_create(int device, dl_ctx** out);
void dl_destroy(dl_ctx* ctx);
/* Message for the last error on this context ("" if none).  Valid until the
 * next call on the context. */
const char* dl_last_error(const dl_ctx* ctx);
/* Library version string. */
const char* dl_version(void);

/* Per-stage GPU timing with HIP events, recorded on the call's stream.
 * Stages: 0 featurize, 1 prep, 2 candidate contraction (the matrix-core
 * kernel), 3 recheck (fp32 + fp64 ties), 4 canonical sort, 5 top-k select,
 * 6 index build (pivot order, block balls, bound pass, tile list).
 * dl_get_timing adds, per stage, the summed milliseconds and the number of
 * timed launches since the last reset into ms[] and calls[] (arrays of
 * DL_NUM_STAGES); it synchronises on the recorded events. */
#define DL_NUM_STAGES 7
dl_status dl_set_timing(dl_ctx* ctx, int enable);
dl_status dl_get_timing(dl_ctx* ctx, double* ms, int64_t* calls, int reset);

/* ----------------------------------------------------------- featurise */

/* Colour histogram of each patch (section "Visual ETL", Transformers).
 *   patches   device, n*h*w*3 uint8, patch-major, pixels row-major, channels
 *             R,G,B interleaved (HWC), contiguous.
 *   bins      bins per channel; must divide 256 (bin width 256/bins).
 *   out_hist  device, n * bins^3 float32, row-major: entry
 *             ((r/width)*bins + g/width)*bins + b/width counts the pixels of
 *             that colour cell, divided by h*w (correctly rounded).
 * Errors: DL_ERR_INVALID for null pointers, n < 0, h or w < 1, h*w >= 2^24,
 * bins not dividing 256 or bins^3 > 4096. */
dl_status dl_featurize_rgb8(dl_ctx* ctx, const uint8_t* patches, int64_t n,
                            int32_t h, int32_t w, int32_t bins,
                            float* out_hist, void* stream);

/* A patch given as a bounding box over a frame (section "Iterator API for
 * Patches": a patch refers to a region of an image): pixels x0 <= x < x1,
 * y0 <= y < y1 of frame `frame`. */
typedef struct dl_box {
  int32_t frame;
  int32_t x0, y0, x1, y1;
} dl_box;

/* Colour histograms of boxes cut from full frames (section "Visual ETL",
 * Transformers, over the patches a detector's boxes define).
 *   frames    device, nframes * height * width * 3 uint8, frame-major, pixels
 *             row-major, channels R,G,B interleaved (HWC), contiguous.
 *   boxes     device, nboxes boxes; each must lie inside its frame
 *             (0 <= x0 < x1 <= width, 0 <= y0 < y1 <= height, 0 <= frame <
 *             nframes).
 *   out_hist  device, nboxes * bins^3 float32: as dl_featurize_rgb8 for the
 *             box's pixels, each count divided by the box's pixel count
 *             (correctly rounded, whatever the count).
 * Errors: DL_ERR_INVALID for null pointers, bad sizes (height * width must be
 * below 2^24), bins as for dl_featurize_rgb8, or any box outside its frame
 * (checked on the GPU; such a box's row is all zero).  Synchronises
 * `stream` (to report bad boxes). */
dl_status dl_featurize_crops_rgb8(dl_ctx* ctx, const uint8_t* frames,
                                  int64_t nframes, int32_t height,
                                  int32_t width, const dl_box* boxes,
                                  int64_t nboxes, int32_t bins,
                                  float* out_hist, void* stream);

/* -------------------------------------------------------- pair distances */

/* Squared Euclidean distance in float64 for listed pairs, summed over
 * k = 0..d-1 in order with separately rounded subtract, multiply and add
 * (the canonical definition every join decision is exact against).
 *   pi, pj  device uint32[m]: row of R and row of S of each pair.
 *   out_d2  device double[m].
 * Indices must be in range (checked on the GPU: out-of-range pairs get NaN
 * and the call returns DL_ERR_INVALID). */
dl_status dl_pair_d2(dl_ctx* ctx, dl_mat R, dl_mat S, const uint32_t* pi,
                     const uint32_t* pj, int64_t m, double* out_d2,
                     void* stream);

/* ------------------------------------------------------------- eps-join */

/* Output of dl_join_eps: caller-owned device arrays of `capacity` entries. */
typedef struct dl_pairs {
  uint32_t* i;        /* device: row of R                                  */
  uint32_t* j;        /* device: row of S                                  */
  float* dist;        /* device: distance rounded to float32               */
  int64_t capacity;   /* entries available in i, j, dist                   */
  int64_t count;      /* out: number of matching pairs (may exceed capacity) */
  int64_t candidates; /* out: pairs that passed the margin-widened filter  */
  int64_t ties;       /* out: candidates decided by the float64 recheck    */
} dl_pairs;

/* Scratch bytes needed by dl_join_eps for up to `max_candidates` candidate
 * pairs after the matrix-core filter.  self_join != 0 means S is R. */
size_t dl_join_eps_workspace(int64_t nR, int64_t nS, int32_t d, dl_prec prec,
                             int self_join, int64_t max_candidates);

/* eps-range join (section "Query Processing", Nested Loop Join, with the
 * Euclidean threshold predicate of section "Derived Data").
 * Emits every pair (i, j) of R x S -- i < j when self_join != 0, S ignored
 * and R joined with itself (query q4's deduplication) -- whose float64
 * canonical distance (see dl_pair_d2) satisfies sqrt(d2) <= eps, sorted by
 * (i, j).  dist is within the documented float32 error of sqrt(d2).
 * The pair set does not depend on `prec`.
 *   eps    >= 0, may be +inf; NaN is rejected.
 *   ws     device scratch of ws_bytes (see dl_join_eps_workspace).
 *   out    host struct; its arrays are device memory.
 * Returns DL_ERR_CAPACITY if count > capacity (the first `capacity` pairs in
 * (i, j) order are written, out->count holds the total), DL_ERR_WORKSPACE if
 * the candidates exceed what ws holds (dl_required_workspace() gives the
 * bytes that would have sufficed), DL_ERR_INVALID for bad shapes or a
 * non-finite value in R or S.  Synchronises `stream`. */
dl_status dl_join_eps(dl_ctx* ctx, dl_mat R, dl_mat S, int self_join,
                      double eps, dl_prec prec, void* ws, size_t ws_bytes,
                      dl_pairs* out, void* stream);

/* Bytes of workspace the last DL_ERR_WORKSPACE failure on ctx needed. */
size_t dl_required_workspace(const dl_ctx* ctx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * eps-join as dl_join_eps, with the library's fixed scratch as its
 * workspace.  The call itself allocates nothing (no hipMalloc, hipFree or
 * event creation; no per-stage timing is recorded).
 *   The scratch is DL_NOALLOC_SCRATCH_BYTES of device memory per GPU, held
 *   from the first dl_create on that GPU until the process ends.  Every call
 *   on a GPU uses that GPU's one copy, so calls that overlap on one GPU (two
 *   threads, two streams, or a stream still running an earlier call) race
 *   and their results are undefined: serialise them.  The scratch keeps the
 *   last call's contents; the call clears what it needs cleared itself.
 * Same arguments, outputs and errors as dl_join_eps, except that a join
 * whose operand copies alone exceed the scratch, or whose candidates do not
 * fit beside them, returns DL_ERR_WORKSPACE at once (dl_last_error says how
 * much it needs; dl_required_workspace() gives 0: use dl_join_eps with a
 * workspace instead), and DL_ERR_DEVICE if the scratch could not be set up
 * on the context's device.  Synchronises `stream`. */
#define DL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dl_status dl_join_eps_noalloc(dl_ctx* ctx, dl_mat R, dl_mat S, int self_join,
                              double eps, dl_prec prec, dl_pairs* out,
                              void* stream);

/* ------------------------------------------------------ indexed eps-join */

/* What the index of dl_join_eps_indexed pruned. */
typedef struct dl_index_info {
  int64_t tiles_total;     /* 256 x 256 tiles of the join (self-join: upper triangle) */
  int64_t tiles_computed;  /* tiles the candidate pass ran on                         */
  int32_t pivots;          /* pivots of the row ordering; 0: no index was built        */
  int32_t ksteps_per_tile; /* K-steps (128 operand bytes of each row) of a full tile   */
  int64_t ksteps_computed; /* K-steps run over the computed tiles: steps where every
                              row of either tile is zero are skipped                  */
} dl_index_info;

/* Scratch bytes for dl_join_eps_indexed with room for `max_candidates`
 * candidates; pivots as for the join (0 = default). */
size_t dl_join_eps_indexed_workspace(int64_t nR, int64_t nS, int32_t d,
                                     dl_prec prec, int self_join,
                                     int64_t max_candidates, int32_t pivots);

/* The eps-join of dl_join_eps -- same pair set, order, distances, outputs
 * and errors -- with an index built on the fly inside the call (section
 * "Query Processing": an index on one relation, probed by the other, built
 * during the join; section "Derived Data": a Ball-tree answers Euclidean
 * threshold queries).  The rows of each relation are ordered by their
 * nearest pivot (`pivots` rows of S at a fixed stride; 0 = nS / 1,024,
 * clamped to 16..4,096), every block of 256 ordered rows gets a ball
 * (centroid, radius), and a 256 x 256 tile of pairs is computed only if a
 * row of each side lies within eps + radius of the other side's ball, a test
 * the triangle inequality makes exact (no result pair is ever pruned).  On
 * clustered data most tiles are skipped.  Within a computed tile, the
 * K-steps (128 bytes of each operand row: 64 bins of an fp16 histogram) in
 * which every row of the R tile or every row of the S tile is zero are
 * skipped too: their products are zero, so the result is unchanged (the
 * structure of image features that section "Conclusion and Future Work"
 * points to: the rows of one cluster share few nonzero histogram bins).
 * Without a finite eps, or with a relation under 512 rows, it runs as
 * dl_join_eps.  info (host, nullable) reports the tiles and K-steps
 * computed.  Synchronises `stream`. */
dl_status dl_join_eps_indexed(dl_ctx* ctx, dl_mat R, dl_mat S, int self_join,
                              double eps, dl_prec prec, int32_t pivots,
                              void* ws, size_t ws_bytes, dl_pairs* out,
                              dl_index_info* info, void* stream);

/* ----------------------------------------------------- filtered eps-join */

/* Scratch bytes for dl_join_eps_filtered (plan 0 or 1) with room for
 * max_candidates candidates and, for plan 1, max_pairs unfiltered pairs. */
size_t dl_join_eps_filtered_workspace(int64_t nR, int64_t nS, int32_t d,
                                      dl_prec prec, int self_join,
                                      int32_t plan, int64_t max_candidates,
                                      int64_t max_pairs);

/* The eps-join of the rows of R and S whose label equals `label` (section
 * "Query Processing": a query's filter on patch metadata and its match, in
 * either order; the paper's plan-order experiment).  The result -- pairs
 * (i, j) of the original rows with both labels equal to `label` and
 * sqrt(d2) <= eps, in (i, j) order, as dl_join_eps -- is the same for both
 * plans; the work is not:
 *   plan 0  filter first: select and gather each relation's matching rows,
 *           join those, map the pairs back to the original rows;
 *   plan 1  match first: join all rows into the workspace (at most
 *           max_pairs pairs), then keep the pairs whose two labels match.
 *   labels_R, labels_S  device int32 per row (labels_S ignored for a
 *                       self-join).
 * Errors as dl_join_eps; plan 1 returns DL_ERR_WORKSPACE when the
 * unfiltered pairs exceed max_pairs (dl_required_workspace says how much
 * would do).  Synchronises `stream`. */
dl_status dl_join_eps_filtered(dl_ctx* ctx, dl_mat R, dl_mat S, int self_join,
                               double eps, dl_prec prec,
                               const int32_t* labels_R,
                               const int32_t* labels_S, int32_t label,
                               int32_t plan, int64_t max_candidates,
                               int64_t max_pairs, void* ws, size_t ws_bytes,
                               dl_pairs* out, void* stream);

/* ---------------------------------------------------------------- top-k */

typedef struct dl_topk_info {
  int64_t band_entries; /* candidates kept by the margin-widened band filter */
  int64_t ties;         /* entries whose order was decided in float64       */
} dl_topk_info;

/* Scratch bytes for dl_join_topk with `band_cap` band entries per row and
 * S-split (0 = library default).  For DL_FP8 (not self-joins, nS at least
 * 4,096 rows) this includes an exact bf16 pilot top-k against every 16th row
 * of S, whose k-th distances seed the E4M3 band thresholds. */
size_t dl_join_topk_workspace(int64_t nR, int64_t nS, int32_t d, dl_prec prec,
                              int self_join, int32_t k, int32_t band_cap);

/* k closest rows of S for every row of R (query q1, section "Queries":
 * the closest image to a query image), by float64 canonical d2 with ties
 * broken by the smaller j, ascending.  self_join != 0: S is R, and
 * exclude_self drops j == i.
 *   out_j     device uint32[nR*k]; UINT32_MAX pads rows with fewer than k.
 *   out_dist  device float[nR*k];  +inf pads.
 *   info      host, nullable.
 * Rows with more near-tie contenders than the selection holds in LDS (512:
 * many rows of S at one distance, such as duplicates) are selected again
 * over their band buffers in memory: slower, with the same exact answer.
 * Returns DL_ERR_WORKSPACE if the workspace is too small or if a row's band
 * does not fit band_cap ("band buffer" in dl_last_error: retry with a larger
 * band_cap); DL_ERR_INVALID for bad arguments.  Synchronises `stream`. */
dl_status dl_join_topk(dl_ctx* ctx, dl_mat R, dl_mat S, int self_join,
                       int32_t k, int exclude_self, dl_prec prec,
                       int32_t band_cap, void* ws, size_t ws_bytes,
                       uint32_t* out_j, float* out_dist, dl_topk_info* info,
                       void* stream);

/* Scratch bytes for dl_join_topk_indexed (the index, a sample top-k and the
 * pruned join's own; at least dl_join_topk_workspace's). */
size_t dl_join_topk_indexed_workspace(int64_t nR, int64_t nS, int32_t d, dl_prec prec,
                                      int self_join, int exclude_self, int32_t k,
                                      int32_t band_cap, int32_t pivots);

/* The top-k join with an index built inside the call (section "Query
 * Processing": an index built on the fly inside the join; section "Derived
 * Data": ball bounds for Euclidean queries): the result of dl_join_topk,
 * exactly, while tiles of pairs that cannot hold a row's k nearest are
 * skipped.  Each row's k-th distance is bounded by an exact top-k against
 * every 16th row of S (k + 1 with exclude_self).  Rows are ordered by
 * nearest pivot as in dl_join_eps_indexed (pivots, 0 = default).  Every 256
 * ordered rows of R form a ball whose radius is the largest bound of its
 * rows.  A bound pass on the matrix cores keeps the S tiles with a row
 * within that ball's reach, and the band pass runs on the kept tiles only,
 * skipping K-steps as dl_join_eps_indexed does.  Every pass runs in prec,
 * except that DL_FP8 runs in bf16: in pivot order a row's near rows fall
 * into few band splits, where E4M3's wide margin overflows the band (the
 * result is the same).  The band and the exact selection are
 * dl_join_topk's.  Falls back to
 * dl_join_topk when either relation spans fewer than two 256-row tiles or
 * the sample top-k does not fit the workspace.
 *   out_j, out_dist, info  as dl_join_topk;
 *   xinfo     host, nullable: tiles_total = row tiles x column tiles,
 *             tiles_computed = those kept, pivots (0 when no index was
 *             built), ksteps_per_tile and ksteps_computed over the kept
 *             tiles (0 when rows span more than 64 K-steps: no masks).
 * Errors as dl_join_topk ("band buffer": retry with a larger band_cap and
 * dl_join_topk_indexed_workspace of it).  Synchronises `stream`. */
dl_status dl_join_topk_indexed(dl_ctx* ctx, dl_mat R, dl_mat S, int self_join,
                               int32_t k, int exclude_self, dl_prec prec,
                               int32_t band_cap, int32_t pivots, void* ws,
                               size_t ws_bytes, uint32_t* out_j, float* out_dist,
                               dl_topk_info* info, dl_index_info* xinfo,
                               void* stream);


/* ---------------------------------------------------------------- store */

/* A resident relation (the on-the-fly index join of section "Query
 * Processing" keeps one relation resident and probes it with the other; the
 * materialised intermediate result of section "Visual ETL").  The store
 * borrows `base` (float32 rows, device): the caller keeps it alive and
 * unchanged until dl_store_destroy.  The operand copy and statistics are
 * built once into `mem` (device, caller-owned, dl_store_bytes() bytes). */
typedef struct dl_store dl_store;

size_t dl_store_bytes(int64_t n, int32_t d, dl_prec prec);
/* Builds the store; synchronises `stream`.  DL_ERR_INVALID for bad shapes or
 * non-finite rows, DL_ERR_WORKSPACE if mem is too small. */
dl_status dl_store_create(dl_ctx* ctx, dl_mat base, dl_prec prec, void* mem, size_t bytes, dl_store** out,
                          void* stream);
void dl_store_destroy(dl_store* store);
int64_t dl_store_rows(const dl_store* store);

/* Featurise and materialise in one pass (section "Visual ETL": transformers
 * whose output is materialised for later queries): the colour histograms of
 * n patches of h x w pixels (boxes == NULL; pixels as dl_featurize_rgb8) or
 * of nboxes boxes over nframes frames of h x w pixels (pixels and boxes as
 * dl_featurize_crops_rgb8) are written to out_hist (device, rows x bins^3
 * float32) and, from the same LDS counts without reading them back, the
 * store's operand copy and statistics into `mem` (dl_store_bytes(rows,
 * bins^3, prec) bytes).  The store borrows out_hist as its float32 rows.
 * Same histograms as the featurise calls; same store as dl_store_create on
 * out_hist.  Errors as those calls.  Synchronises `stream`. */
dl_status dl_store_featurize_rgb8(dl_ctx* ctx, const uint8_t* pixels,
                                  int64_t n, int32_t h, int32_t w,
                                  const dl_box* boxes, int64_t nboxes,
                                  int32_t bins, dl_prec prec, float* out_hist,
                                  void* mem, size_t bytes, dl_store** out,
                                  void* stream);

/* The eps-join and top-k join of R against a store (S = the store's rows,
 * operand format = the store's).  Same semantics, outputs and errors as
 * dl_join_eps / dl_join_topk with self_join = 0. */
size_t dl_join_eps_store_workspace(int64_t nR, const dl_store* store, int64_t max_candidates);
dl_status dl_join_eps_store(dl_ctx* ctx, dl_mat R, const dl_store* store, double eps, void* ws,
                            size_t ws_bytes, dl_pairs* out, void* stream);
/* The eps self-join of a store's rows (i < j; query q4's deduplication),
 * using the store's operand copy for both sides (no prep pass).  Same
 * semantics, outputs and errors as dl_join_eps with self_join = 1. */
size_t dl_join_eps_store_self_workspace(const dl_store* store, int64_t max_candidates);
dl_status dl_join_eps_store_self(dl_ctx* ctx, const dl_store* store, double eps, void* ws, size_t ws_bytes,
                                 dl_pairs* out, void* stream);
size_t dl_join_topk_store_workspace(int64_t nR, const dl_store* store, int32_t k, int32_t band_cap);
dl_status dl_join_topk_store(dl_ctx* ctx, dl_mat R, const dl_store* store, int32_t k, int32_t band_cap,
                             void* ws, size_t ws_bytes, uint32_t* out_j, float* out_dist,
                             dl_topk_info* info, void* stream);

/* ---------------------------------------------------------------- server */

/* A persistent request loop over one store.  Requests (query rows + eps or
 * k) are queued; worker threads (one HIP stream each) admit the request at
 * the head of the queue and every later queued request of the same mode (and
 * k) that fits the batch limits and the free arena memory, run them as one
 * join against the store, and publish per-request results.  Requests that
 * arrive while batches run are admitted as streams and memory free up.  A
 * request's result and status do not depend on the batch it ran in: a batch
 * that outgrows its output, candidate or band capacity puts its requests
 * back at the head of the queue to run alone, and a request that outgrows
 * them alone runs again with the capacity it reported (up to four times).
 * With n_streams >= 2 the first stream is a lane for small requests. */
typedef struct dl_server dl_server;

#define DL_MODE_EPS 0
#define DL_MODE_TOPK 1

typedef struct dl_server_config {
  int32_t n_streams;          /* batches on the device at once (default 2, max 8) */
  int32_t max_batch_requests; /* requests per batch (default 64)                 */
  int64_t max_batch_rows;     /* query rows per batch (default 65536)            */
  int64_t pairs_per_row;      /* eps output room per query row (default 64)     */
  int32_t band_cap;           /* top-k band entries per row and split (0 = default) */
  int64_t small_rows;         /* with n_streams >= 2 the first stream only runs
                                 requests of at most this many rows (0 = 4,096;
                                 < 0: no small-request lane)                 */
} dl_server_config;

typedef struct dl_request {
  dl_mat query;   /* device rows, d = the store's d; borrowed until the request completes */
  int32_t mode;   /* DL_MODE_EPS or DL_MODE_TOPK */
  double eps;     /* eps-join radius (mode DL_MODE_EPS) */
  int32_t k;      /* neighbours per row, 1..256 (mode DL_MODE_TOPK) */
} dl_request;

/* Result of a completed request.  Arrays are device memory inside the
 * server's arena, valid until dl_server_release.
 *   eps:  count pairs (i = row of the request's query, j = store row, dist),
 *         sorted by (i, j).
 *   top-k: j and dist are rows x k, as dl_join_topk_store. */
typedef struct dl_result {
  dl_status status;
  int32_t mode;
  int64_t rows;
  int32_t k;
  const uint32_t* i;
  const uint32_t* j;
  const float* dist;
  int64_t count;
  double queued_ms;   /* submit -> batch start */
  double latency_ms;  /* submit -> result ready */
  int64_t batch_id;
  int32_t batch_requests;
} dl_result;

typedef struct dl_server_info {
  int64_t submitted, completed, rejected, cancelled, batches, queued;
  double mean_batch_requests;
  double pairs_done;  /* sum over completed requests of rows x store rows */
  double span_ms;     /* first submit -> last completion */
  double p50_ms, p99_ms, max_ms;
  size_t arena_in_use, arena_peak;
  double batch_ms;    /* summed wall time of successful batch runs (batch start -> results ready) */
  double batch_pairs; /* summed rows x store rows of those batches */
} dl_server_info;

/* Starts the workers on `device`.  `arena` (device, caller-owned) holds every
 * in-flight batch's packed queries, workspace and results; a batch is
 * admitted only if its footprint fits the arena's free space, and a request
 * that cannot fit an empty arena completes with DL_ERR_OOM. */
dl_status dl_server_create(int device, const dl_store* store, const dl_server_config* cfg, void* arena,
                           size_t arena_bytes, dl_server** out);
/* Queues a request; returns at once with a ticket. */
dl_status dl_server_submit(dl_server* srv, const dl_request* req, uint64_t* ticket);
/* Waits up to timeout_ms (< 0: forever) for a request; DL_ERR_BUSY on
 * timeout.  out->status is the request's own status. */
dl_status dl_server_wait(dl_server* srv, uint64_t ticket, int32_t timeout_ms, dl_result* out);
/* Frees a completed request's result memory and its ticket. */
dl_status dl_server_release(dl_server* srv, uint64_t ticket);
/* Cancels a request still in the queue (DL_ERR_BUSY once it has started). */
dl_status dl_server_cancel(dl_server* srv, uint64_t ticket);
dl_status dl_server_stats(dl_server* srv, dl_server_info* out);
dl_status dl_server_reset_stats(dl_server* srv);
/* Cancels queued requests, waits for running batches, stops the workers. */
void dl_server_destroy(dl_server* srv);

/* ------------------------------------------------------------ measurement */

/* Achievable rates of this device, measured: the denominators of roofline
 * fractions beside the published peaks.  Not a step of the method; the
 * benchmark calls it once. */
typedef struct dl_peaks {
  double mfma_fp32_tflops; /* dense matrix-core rate of each operand format on */
  double mfma_bf16_tflops; /* register operands: v_mfma_f32_16x16x4f32,         */
  double mfma_fp16_tflops; /* v_mfma_f32_16x16x32_{bf16,f16} and the E4M3       */
  double mfma_fp8_tflops;  /* v_mfma_scale_f32_16x16x128_f8f6f4, 8 chains/wave  */
  double hbm_copy_gbps;    /* a 1 GiB device copy: bytes read + written per s   */
  double mfma_bf16_2w_tflops;        /* 16x16x32 bf16 at two waves per SIMD (the  */
  double mfma_bf16_32x32_2w_tflops;  /* candidate pass's occupancy); 32x32x16 bf16 */
  double hbm_read_gbps;              /* a 1 GiB streaming read: bytes per s        */
  double mfma_bf16_lds_tflops;       /* 16x16x32 bf16 fed from LDS in the candidate */
                                     /* pass's fragment pattern, two waves per SIMD,*/
                                     /* a barrier per K-step: that loop's ceiling   */
} dl_peaks;

/* Runs the rate kernels on the context's device (default stream; it
 * allocates and frees 2 GiB of device memory and synchronises).  About
 * 0.1 s. */
dl_status dl_measure_peaks(dl_ctx* ctx, dl_peaks* out);

#ifdef __cplusplus
}
#endif

#endif /* DLMI_H */
