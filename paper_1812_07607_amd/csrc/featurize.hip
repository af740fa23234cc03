// featurize.hip -- colour-histogram transformer over uint8 RGB patches.
//
// Paper: section "Visual ETL", Transformers (colour histogram features for
// image matching); the patches are crops of frames given by bounding boxes
// (section "Iterator API for Patches": a patch refers to a region of an
// image), either already cut out (n patches of h x w pixels) or as boxes over
// full frames.  One wavefront builds the histogram of one patch in a
// wave-private LDS array, so no histogram crosses waves: the waves of a
// workgroup never wait for one another (wave-level LDS ordering only), and
// the only global traffic is one read of the pixels and one coalesced write
// of the normalised bins.  HBM-bound: algorithmic bytes per patch are
// h*w*3 read plus bins^3*4 written.
//
// The fused kernel (materialise into a store, section "Visual ETL") hands
// each bin straight from LDS to the operand prep of the join (operand copy
// and row statistics), so the float32 histograms are written once and never
// read back.
#include "prep_row.hpp"

namespace dl {

constexpr int kHistWaves = 4;  // patches (waves) per workgroup

// This wave's LDS operations are complete and every lane has reached this
// point (the histogram is private to the wave).  Only the LDS counter is
// waited for (s_waitcnt lgkmcnt(0); vmcnt and expcnt at their no-wait
// values): the wave's global stores of the previous patch need not land
// before it clears and counts the next one.
__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_wave_barrier();
}

// Counts of one 16-pixel group (48 bytes = 12 dwords) into the wave's bins.
// Neighbouring pixels often share a bin, so a run of equal bins is added
// with one LDS atomic (fewer atomics, and fewer lanes colliding on the
// same bin in one instruction; measured 0.157 -> 0.127 ms on 100,000
// palette patches).
__device__ inline void count16(uint32_t* __restrict__ hist, const uint32_t w[12], int shift, int bins) {
  uint32_t prev = 0xffffffffu, run = 0;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int b0 = 3 * p, b1 = 3 * p + 1, b2 = 3 * p + 2;
    uint32_t r = (w[b0 >> 2] >> ((b0 & 3) * 8)) & 0xffu;
    uint32_t g = (w[b1 >> 2] >> ((b1 & 3) * 8)) & 0xffu;
    uint32_t b = (w[b2 >> 2] >> ((b2 & 3) * 8)) & 0xffu;
    uint32_t bin = (((r >> shift) * bins) + (g >> shift)) * bins + (b >> shift);
    if (bin == prev) {
      ++run;
    } else {
      if (run) atomicAdd(&hist[prev], run);
      prev = bin;
      run = 1;
    }
  }
  atomicAdd(&hist[prev], run);
}

// Pixel sources.  kSrcPatch48: contiguous patches whose pixel count is a
// multiple of 16, 16-byte aligned (three 16-byte loads per 16 pixels);
// kSrcPatch: any contiguous patches; kSrcCrop: boxes over frames.
enum : int { kSrcPatch48 = 0, kSrcPatch = 1, kSrcCrop = 2 };

struct PixelSource {
  const uint8_t* pix;      // patches (n x h x w x 3) or frames (nframes x h x w x 3)
  int32_t h, w;            // patch size, or frame size for crops
  const dl_box* boxes;     // crops: one box per patch
  int64_t nframes;
  int* bad_box;            // crops: set when a box is not inside its frame
};

// Counts the pixels of patch p into the wave's bins; returns the pixel
// count (0 for an invalid box, which contributes nothing).
template <int kSrc>
__device__ inline int count_patch(const PixelSource& src, int64_t p, uint32_t* __restrict__ hist, int shift,
                                  int bins, int lane) {
  if constexpr (kSrc == kSrcCrop) {
    const dl_box bx = src.boxes[p];
    const bool ok = bx.frame >= 0 && bx.frame < src.nframes && bx.x0 >= 0 && bx.x0 < bx.x1 && bx.x1 <= src.w &&
                    bx.y0 >= 0 && bx.y0 < bx.y1 && bx.y1 <= src.h;
    if (!ok) {
      if (lane == 0) atomicOr(src.bad_box, 1);
      return 0;
    }
    const int cw = bx.x1 - bx.x0, area = cw * (bx.y1 - bx.y0);
    const uint8_t* base = src.pix + (((int64_t)bx.frame * src.h + bx.y0) * src.w + bx.x0) * 3;
    // row of pixel q by a float reciprocal, then one correction step each
    // way (q < 2^24, so the estimate is off by at most one)
    const float rcw = 1.0f / (float)cw;
    auto at = [&](int q) {
      int y = (int)((float)q * rcw);
      int x = q - y * cw;
      if (x < 0) {
        --y;
        x += cw;
      } else if (x >= cw) {
        ++y;
        x -= cw;
      }
      return base + ((int64_t)y * src.w + x) * 3;
    };
    auto bin_of = [&](uint32_t r, uint32_t g, uint32_t b) {
      return (((r >> shift) * bins) + (g >> shift)) * bins + (b >> shift);
    };
    // eight (then four) pixels' loads in flight per lane, then their counts (a box's
    // rows are short strided runs, so the loads' latency, not their bytes,
    // bounds a wave)
    int q = lane;
    for (; q + 7 * 64 < area; q += 8 * 64) {
      uint32_t c[8][3];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint8_t* px = at(q + 64 * u);
        c[u][0] = px[0];
        c[u][1] = px[1];
        c[u][2] = px[2];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) atomicAdd(&hist[bin_of(c[u][0], c[u][1], c[u][2])], 1u);
    }
    for (; q + 3 * 64 < area; q += 4 * 64) {
      uint32_t c[4][3];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint8_t* px = at(q + 64 * u);
        c[u][0] = px[0];
        c[u][1] = px[1];
        c[u][2] = px[2];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) atomicAdd(&hist[bin_of(c[u][0], c[u][1], c[u][2])], 1u);
    }
    for (; q < area; q += 64) {
      const uint8_t* px = at(q);
      atomicAdd(&hist[bin_of(px[0], px[1], px[2])], 1u);
    }
    return area;
  } else {
    const int npx = src.h * src.w;
    const uint8_t* s = src.pix + p * (int64_t)npx * 3;
    if constexpr (kSrc == kSrcPatch48) {
      typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
      const u32x4* v = reinterpret_cast<const u32x4*>(s);
      const int groups = npx / 16;  // 16 pixels = 48 bytes = 3 x 16 bytes
      for (int c = lane; c < groups; c += 64) {
        const u32x4 x0 = __builtin_nontemporal_load(v + 3 * c + 0);
        const u32x4 x1 = __builtin_nontemporal_load(v + 3 * c + 1);
        const u32x4 x2 = __builtin_nontemporal_load(v + 3 * c + 2);
        uint32_t w[12] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w, x2.x, x2.y, x2.z, x2.w};
        count16(hist, w, shift, bins);
      }
    } else {
      for (int q = lane; q < npx; q += 64) {
        const uint32_t r = s[3 * q], g = s[3 * q + 1], b = s[3 * q + 2];
        const uint32_t bin = (((r >> shift) * bins) + (g >> shift)) * bins + (b >> shift);
        atomicAdd(&hist[bin], 1u);
      }
    }
    return npx;
  }
}

// Histograms only: bin / pixel count, rounded once (IEEE division).
template <int kSrc>
__global__ __launch_bounds__(64 * kHistWaves) void hist_rgb8_kernel(PixelSource src, int64_t n, int32_t bins,
                                                                    int32_t shift, float* __restrict__ out) {
  extern __shared__ uint32_t lds_hist[];
  const int nb = bins * bins * bins;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* hist = lds_hist + wave * nb;
  const int64_t ngroups = (n + kHistWaves - 1) / kHistWaves;
  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int64_t p = g * kHistWaves + wave;
    if (p >= n) break;
    for (int b = lane; b < nb; b += 64) hist[b] = 0u;
    wave_lds_fence();
    const int npx = count_patch<kSrc>(src, p, hist, shift, bins, lane);
    wave_lds_fence();
    const float fnpx = (float)(npx > 0 ? npx : 1);  // exact: npx < 2^24
    float* dst = out + p * (int64_t)nb;
    for (int b = lane; b < nb; b += 64) dst[b] = (float)hist[b] / fnpx;  // IEEE division
    wave_lds_fence();  // the bins are read before the next patch clears them
  }
}

// Histograms plus the join's operand prep of each histogram row (rows n..npad
// of the operand copy are zero padding, as the prep kernel writes them).
template <int kSrc, int kPrec>
__global__ __launch_bounds__(64 * kHistWaves) void hist_prep_kernel(PixelSource src, int64_t n, int32_t bins,
                                                                    int32_t shift, float* __restrict__ out,
                                                                    int64_t dpad, Prep P, RelStats* rs) {
  extern __shared__ uint32_t lds_hist[];
  const int nb = bins * bins * bins;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* hist = lds_hist + wave * nb;
  const int64_t ngroups = (P.npad + kHistWaves - 1) / kHistWaves;
  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int64_t p = g * kHistWaves + wave;
    if (p >= P.npad) break;
    const bool real = p < n;
    int npx = 0;
    if (real) {
      for (int b = lane; b < nb; b += 64) hist[b] = 0u;
      wave_lds_fence();
      npx = count_patch<kSrc>(src, p, hist, shift, bins, lane);
      wave_lds_fence();
    }
    const float fnpx = (float)(npx > 0 ? npx : 1);
    int sexp = 0;
    if (kPrec == DL_FP8 && real) {
      // the largest bin, divided as the bins are (rounding is monotone)
      uint32_t cmax = 0;
      for (int b = lane; b < nb; b += 64) cmax = max(cmax, hist[b]);
      sexp = e4m3_row_scale(wave_max((float)cmax / fnpx));
    }
    RowPrep<kPrec> rp(P, p, sexp);
    float* dst = out + p * (int64_t)nb;
    for (int64_t k = lane; k < dpad; k += 64) {
      float v = 0.0f;
      if (real && k < nb) {
        v = (float)hist[k] / fnpx;  // IEEE division
        dst[k] = v;
      }
      rp.element(v, k);
    }
    rp.finish(P, p, dpad, real, rs, lane);
    wave_lds_fence();
  }
}

static int bin_shift(int bins) {
  int shift = 0;
  while ((256 >> shift) > bins) ++shift;
  return shift;
}

// Host launchers; arguments validated by the caller.
hipError_t launch_hist_rgb8(const uint8_t* patches, int64_t n, int32_t h, int32_t w, int32_t bins,
                            float* out, hipStream_t st, int cu_count) {
  if (n == 0) return hipSuccess;
  const int32_t npx = h * w;
  const int nb = bins * bins * bins;
  const size_t lds = (size_t)kHistWaves * nb * sizeof(uint32_t);
  const int64_t ngroups = (n + kHistWaves - 1) / kHistWaves;
  const int grid = (int)(ngroups < (int64_t)cu_count * 64 ? ngroups : (int64_t)cu_count * 64);
  const PixelSource src{patches, h, w, nullptr, 0, nullptr};
  const bool vec = (npx % 16 == 0) && ((reinterpret_cast<uintptr_t>(patches) & 15) == 0);
  if (vec)
    hipLaunchKernelGGL(hist_rgb8_kernel<kSrcPatch48>, dim3(grid), dim3(64 * kHistWaves), lds, st, src, n, bins,
                       bin_shift(bins), out);
  else
    hipLaunchKernelGGL(hist_rgb8_kernel<kSrcPatch>, dim3(grid), dim3(64 * kHistWaves), lds, st, src, n, bins,
                       bin_shift(bins), out);
  return hipGetLastError();
}

hipError_t launch_hist_crops(const uint8_t* frames, int64_t nframes, int32_t height, int32_t width,
                             const dl_box* boxes, int64_t n, int32_t bins, float* out, int* bad_box, hipStream_t st,
                             int cu_count) {
  if (n == 0) return hipSuccess;
  const int nb = bins * bins * bins;
  const size_t lds = (size_t)kHistWaves * nb * sizeof(uint32_t);
  const int64_t ngroups = (n + kHistWaves - 1) / kHistWaves;
  const int grid = (int)(ngroups < (int64_t)cu_count * 64 ? ngroups : (int64_t)cu_count * 64);
  const PixelSource src{frames, height, width, boxes, nframes, bad_box};
  hipLaunchKernelGGL(hist_rgb8_kernel<kSrcCrop>, dim3(grid), dim3(64 * kHistWaves), lds, st, src, n, bins,
                     bin_shift(bins), out);
  return hipGetLastError();
}

template <int kSrc>
static void launch_hist_prep_src(const PixelSource& src, int64_t n, int32_t bins, float* out, dl_prec prec,
                                 const Prep& P, RelStats* rs, dim3 grid, size_t lds, hipStream_t st) {
  const int64_t dpad = dpad_of(bins * bins * bins, prec);
  const int shift = bin_shift(bins);
  switch (prec) {
    case DL_FP32:
      hipLaunchKernelGGL((hist_prep_kernel<kSrc, DL_FP32>), grid, dim3(64 * kHistWaves), lds, st, src, n, bins, shift,
                         out, dpad, P, rs);
      break;
    case DL_BF16:
      hipLaunchKernelGGL((hist_prep_kernel<kSrc, DL_BF16>), grid, dim3(64 * kHistWaves), lds, st, src, n, bins, shift,
                         out, dpad, P, rs);
      break;
    case DL_FP16:
      hipLaunchKernelGGL((hist_prep_kernel<kSrc, DL_FP16>), grid, dim3(64 * kHistWaves), lds, st, src, n, bins, shift,
                         out, dpad, P, rs);
      break;
    case DL_FP8:
      hipLaunchKernelGGL((hist_prep_kernel<kSrc, DL_FP8>), grid, dim3(64 * kHistWaves), lds, st, src, n, bins, shift,
                         out, dpad, P, rs);
      break;
  }
}

// Fused featurise + prep into P (npad rows); the caller runs the statistics
// reduction after it.  frames/boxes null: patches of h x w.
hipError_t launch_hist_prep(const uint8_t* pix, int64_t nframes, int32_t h, int32_t w, const dl_box* boxes, int64_t n,
                            int32_t bins, float* out, int* bad_box, dl_prec prec, const Prep& P, RelStats* rs,
                            hipStream_t st, int cu_count) {
  const int nb = bins * bins * bins;
  const size_t lds = (size_t)kHistWaves * nb * sizeof(uint32_t);
  const int64_t ngroups = (P.npad + kHistWaves - 1) / kHistWaves;
  const dim3 grid((unsigned)(ngroups < (int64_t)cu_count * 64 ? ngroups : (int64_t)cu_count * 64));
  if (boxes) {
    launch_hist_prep_src<kSrcCrop>(PixelSource{pix, h, w, boxes, nframes, bad_box}, n, bins, out, prec, P, rs, grid,
                                   lds, st);
  } else {
    const PixelSource src{pix, h, w, nullptr, 0, nullptr};
    if (((int64_t)h * w) % 16 == 0 && (reinterpret_cast<uintptr_t>(pix) & 15) == 0)
      launch_hist_prep_src<kSrcPatch48>(src, n, bins, out, prec, P, rs, grid, lds, st);
    else
      launch_hist_prep_src<kSrcPatch>(src, n, bins, out, prec, P, rs, grid, lds, st);
  }
  return hipGetLastError();
}

}  // namespace dl
