/*
 * dl_oracle.c -- plain CPU oracle for the DeepLens patch-matching hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) links, loads or calls this file.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
 * no code, header, table or constant with the GPU path.
 *
 * What it computes, and the passage of the paper (Krishnan et al., "DeepLens:
 * Towards a Visual Data Management System", CIDR 2019) each function follows:
 *
 *   orc_hist_rgb8   colour-histogram transformer over RGB patches
 *                   (section "Visual ETL", Transformers; Example 2 of
 *                   section "Iterator API for Patches" names colour
 *                   histograms as the matching feature).
 *   orc_hist_crops  the same histogram over the pixels of bounding boxes cut
 *                   from full frames (a patch refers to a region of an image:
 *                   section "Iterator API for Patches"; ETL crops patches
 *                   out of frames: section "Visual ETL", Patch Generators).
 *   orc_d2          Euclidean distance between two patch vectors
 *                   (section "Derived Data": Euclidean threshold queries on
 *                   image features).
 *   orc_eps_join    nested-loop join that compares all pairs of patches of
 *                   two collections and keeps those meeting the predicate
 *                   (section "Query Processing", Nested Loop Join), with the
 *                   predicate "L2 distance <= eps" (image matching, section
 *                   "Derived Data"); self-join keeps i < j (query q4,
 *                   distinct pedestrians; section "Queries").
 *   orc_topk        closest images per query image (query q1, reverse
 *                   image search; section "Queries").
 *   orc_pair_d2     the same distance for an explicit list of pairs.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - histogram: joint RGB histogram with `bins` uniform bins per channel of
 *     width 256/bins, bin index (r_bin*bins + g_bin)*bins + b_bin, channels
 *     stored R,G,B per pixel (HWC); L1 normalisation divides each count by
 *     the pixel count, computed in double and rounded once to float.
 *   - distance: d2 = sum over k in increasing order of t*t with
 *     t = (double)a[k] - (double)b[k]; sequential, no fused multiply-add
 *     (this file must be compiled with -ffp-contract=off); dist = sqrt(d2).
 *   - eps-join predicate: sqrt(d2) <= eps, inclusive; output in (i, j) order.
 *   - top-k: order by (d2, j) ascending, first min(k, |S|) entries;
 *     exclude_self drops j == i; missing entries are padded with j = -1 and
 *     d2 = +inf.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 * OpenMP only splits independent rows across threads (used for timing); the
 * per-pair arithmetic is the same sequential loop on every thread.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_NOMEM 2

static void set_threads(int32_t nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

/* ---------------------------------------------------------------------------
 * Colour histogram.  patches: n x h x w x 3 uint8, contiguous, HWC, R,G,B.
 * out: n x bins^3 floats.  counts (nullable): n x bins^3 int32 raw counts.
 * ------------------------------------------------------------------------- */
int orc_hist_rgb8(const uint8_t* patches, int64_t n, int32_t h, int32_t w,
                  int32_t bins, float* out, int32_t* counts, int32_t nthreads) {
  if (n < 0 || h <= 0 || w <= 0 || bins <= 0 || bins > 256 || 256 % bins != 0)
    return ORC_ERR_ARG;
  const int64_t nb = (int64_t)bins * bins * bins;
  const int64_t npx = (int64_t)h * w;
  const int32_t width = 256 / bins; /* uniform bin width per channel */
  set_threads(nthreads);
  int err = ORC_OK;
#pragma omp parallel
  {
    int32_t* cnt = (int32_t*)malloc((size_t)nb * sizeof(int32_t));
    if (!cnt) {
#pragma omp atomic write
      err = ORC_ERR_NOMEM;
    }
#pragma omp for schedule(dynamic, 64)
    for (int64_t p = 0; p < n; ++p) {
      if (!cnt) continue;
      memset(cnt, 0, (size_t)nb * sizeof(int32_t));
      const uint8_t* px = patches + p * npx * 3;
      for (int64_t q = 0; q < npx; ++q) {
        int32_t rb = px[3 * q + 0] / width;
        int32_t gb = px[3 * q + 1] / width;
        int32_t bb = px[3 * q + 2] / width;
        cnt[(rb * bins + gb) * bins + bb] += 1;
      }
      for (int64_t k = 0; k < nb; ++k) {
        out[p * nb + k] = (float)((double)cnt[k] / (double)npx);
        if (counts) counts[p * nb + k] = cnt[k];
      }
    }
    free(cnt);
  }
  return err;
}

/* ---------------------------------------------------------------------------
 * Colour histogram of crops.  frames: nframes x height x width x 3 uint8,
 * contiguous, HWC, R,G,B.  boxes: nboxes x 5 int32 (frame, x0, y0, x1, y1),
 * the pixels x0 <= x < x1, y0 <= y < y1 of the frame.  out: nboxes x bins^3
 * floats, each count divided by the box's pixel count (in double, rounded
 * once to float).  A box outside its frame is an argument error.
 * ------------------------------------------------------------------------- */
int orc_hist_crops(const uint8_t* frames, int64_t nframes, int32_t height,
                   int32_t width, const int32_t* boxes, int64_t nboxes,
                   int32_t bins, float* out, int32_t nthreads) {
  if (nframes < 0 || nboxes < 0 || height <= 0 || width <= 0 || bins <= 0 ||
      bins > 256 || 256 % bins != 0)
    return ORC_ERR_ARG;
  for (int64_t b = 0; b < nboxes; ++b) {
    const int32_t* bx = boxes + 5 * b;
    if (bx[0] < 0 || bx[0] >= nframes || bx[1] < 0 || bx[1] >= bx[3] ||
        bx[3] > width || bx[2] < 0 || bx[2] >= bx[4] || bx[4] > height)
      return ORC_ERR_ARG;
  }
  const int64_t nb = (int64_t)bins * bins * bins;
  const int32_t bw = 256 / bins;
  set_threads(nthreads);
  int err = ORC_OK;
#pragma omp parallel
  {
    int32_t* cnt = (int32_t*)malloc((size_t)nb * sizeof(int32_t));
    if (!cnt) {
#pragma omp atomic write
      err = ORC_ERR_NOMEM;
    }
#pragma omp for schedule(dynamic, 16)
    for (int64_t b = 0; b < nboxes; ++b) {
      if (!cnt) continue;
      const int32_t* bx = boxes + 5 * b;
      memset(cnt, 0, (size_t)nb * sizeof(int32_t));
      for (int32_t y = bx[2]; y < bx[4]; ++y) {
        for (int32_t x = bx[1]; x < bx[3]; ++x) {
          const uint8_t* px =
              frames + (((int64_t)bx[0] * height + y) * width + x) * 3;
          cnt[((px[0] / bw) * bins + px[1] / bw) * bins + px[2] / bw] += 1;
        }
      }
      const int64_t npx = (int64_t)(bx[3] - bx[1]) * (bx[4] - bx[2]);
      for (int64_t k = 0; k < nb; ++k)
        out[b * nb + k] = (float)((double)cnt[k] / (double)npx);
    }
    free(cnt);
  }
  return err;
}

/* ---------------------------------------------------------------------------
 * Canonical squared Euclidean distance in double, sequential over k.
 * ------------------------------------------------------------------------- */
double orc_d2(const float* a, const float* b, int32_t d) {
  double d2 = 0.0;
  for (int32_t k = 0; k < d; ++k) {
    double t = (double)a[k] - (double)b[k];
    d2 = d2 + t * t;
  }
  return d2;
}

void orc_pair_d2(const float* R, int64_t ldr, const float* S, int64_t lds,
                 int32_t d, const int64_t* pi, const int64_t* pj, int64_t m,
                 double* out, int32_t nthreads) {
  set_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < m; ++t)
    out[t] = orc_d2(R + pi[t] * ldr, S + pj[t] * lds, d);
}

/* ---------------------------------------------------------------------------
 * eps-join: every (i, j) in R x S (or i < j when self != 0) with
 * sqrt(d2) <= eps, in (i, j) order.  Returns the number of matches; at most
 * `cap` of them are written (the first ones in (i, j) order).  Negative return
 * is an error code.  out_dist receives (float)sqrt(d2).
 *
 * row_ids (nullable) gives, for a sample of rows, the index each row of R has
 * in the full relation: the emitted i is row_ids[i], and for a self-join the
 * rows of S paired with it are those with index > row_ids[i].  row_ids must be
 * increasing so that the output stays in (i, j) order.
 * ------------------------------------------------------------------------- */
int64_t orc_eps_join(const float* R, int64_t nR, int64_t ldr, const float* S,
                     int64_t nS, int64_t lds, int32_t d, double eps,
                     int32_t self, const int64_t* row_ids, int32_t nthreads,
                     int64_t* out_i, int64_t* out_j, double* out_d2,
                     float* out_dist, int64_t cap) {
  if (nR < 0 || nS < 0 || d <= 0) return -ORC_ERR_ARG;
  if (self && !row_ids && (R != S || nR != nS || ldr != lds)) return -ORC_ERR_ARG;
  for (int64_t i = 1; row_ids && i < nR; ++i)
    if (row_ids[i] <= row_ids[i - 1]) return -ORC_ERR_ARG;
  set_threads(nthreads);
  int64_t* rowcnt = (int64_t*)calloc((size_t)(nR + 1), sizeof(int64_t));
  if (!rowcnt) return -ORC_ERR_NOMEM;
  /* pass 1: matches per row */
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < nR; ++i) {
    int64_t c = 0;
    const int64_t gi = row_ids ? row_ids[i] : i;
    for (int64_t j = self ? gi + 1 : 0; j < nS; ++j) {
      double d2 = orc_d2(R + i * ldr, S + j * lds, d);
      if (sqrt(d2) <= eps) ++c;
    }
    rowcnt[i + 1] = c;
  }
  for (int64_t i = 0; i < nR; ++i) rowcnt[i + 1] += rowcnt[i];
  const int64_t total = rowcnt[nR];
  /* pass 2: write the matches of each row at its offset, j ascending */
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < nR; ++i) {
    int64_t pos = rowcnt[i];
    const int64_t gi = row_ids ? row_ids[i] : i;
    if (pos >= cap) continue;
    for (int64_t j = self ? gi + 1 : 0; j < nS && pos < cap; ++j) {
      double d2 = orc_d2(R + i * ldr, S + j * lds, d);
      double dist = sqrt(d2);
      if (dist <= eps) {
        if (out_i) out_i[pos] = gi;
        if (out_j) out_j[pos] = j;
        if (out_d2) out_d2[pos] = d2;
        if (out_dist) out_dist[pos] = (float)dist;
        ++pos;
      }
    }
  }
  free(rowcnt);
  return total;
}

/* ---------------------------------------------------------------------------
 * top-k: for each row i of R, the min(k, |S'|) entries of S' (S, minus j == i
 * when exclude_self) that come first in (d2, j) order, ascending.  Rows with
 * fewer than k entries are padded with j = -1, d2 = +inf, dist = +inf.
 *
 * The k best seen so far are kept as an ordered list; a new (d2, j) is
 * inserted at its ordered position when it precedes the current k-th.  This
 * yields exactly the first k of the full (d2, j) sort.
 * ------------------------------------------------------------------------- */
static int pair_less(double da, int64_t ja, double db, int64_t jb) {
  return da < db || (da == db && ja < jb);
}

int orc_topk(const float* R, int64_t nR, int64_t ldr, const float* S,
             int64_t nS, int64_t lds, int32_t d, int32_t k,
             int32_t exclude_self, const int64_t* self_ids,
             int32_t nthreads, int64_t* out_j,
             double* out_d2, float* out_dist) {
  if (nR < 0 || nS < 0 || d <= 0 || k <= 0) return ORC_ERR_ARG;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < nR; ++i) {
    int64_t* bj = out_j + i * k;
    double* bd = out_d2 + i * k;
    int32_t have = 0;
    const int64_t self_j = self_ids ? self_ids[i] : i;
    for (int64_t j = 0; j < nS; ++j) {
      if (exclude_self && j == self_j) continue;
      double d2 = orc_d2(R + i * ldr, S + j * lds, d);
      if (have == k && !pair_less(d2, j, bd[k - 1], bj[k - 1])) continue;
      int32_t pos = have < k ? have : k - 1;
      while (pos > 0 && pair_less(d2, j, bd[pos - 1], bj[pos - 1])) {
        bd[pos] = bd[pos - 1];
        bj[pos] = bj[pos - 1];
        --pos;
      }
      bd[pos] = d2;
      bj[pos] = j;
      if (have < k) ++have;
    }
    for (int32_t t = have; t < k; ++t) {
      bj[t] = -1;
      bd[t] = INFINITY;
    }
    if (out_dist)
      for (int32_t t = 0; t < k; ++t) out_dist[i * k + t] = (float)sqrt(bd[t]);
  }
  return ORC_OK;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
