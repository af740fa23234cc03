// join_mfma.hip -- candidate pass of the similarity join on CDNA4 matrix cores.
//
// Paper: section "Query Processing" (Nested Loop Join over all pairs of two
// patch collections) with the Euclidean predicate of section "Derived Data"
// and the closest-image query q1 of section "Queries".  The nested loop is
// recast as a tiled product G = A B^T of the two relations' operand copies:
// each 256 x 256 tile of pairs accumulates P~ = a.b - |b|^2/2 (the
// accumulator starts at -h_j) over K-chunks of 128 bytes on the matrix
// cores, and the epilogue compares P~ with one per-row float:
//   eps mode   P~ >= thr_i  (thr_i folds |a|^2, the threshold T and the
//              rigorous margin E_i) -> append (i, j) to the candidate list;
//   band mode  P~ >= band_i, a running top-k band per row kept in LDS ->
//              append (P~, j) to the row's band buffer, tightening band_i
//              to P~_(k) - E_i whenever the buffer fills.
// Candidates are a superset of the exact result; the recheck kernels decide
// exactly.
//
// Layout: 512 threads = 8 waves in a 2 x 4 grid, each wave owns 128 x 64
// outputs as 8 x 4 blocks of 16 x 16 (v_mfma_*_16x16x*), 32 f32x4
// accumulators.  Operands move global -> LDS directly
// (global_load_lds_dwordx4, no staging registers) into a two-stage ring of
// 2 x 256 rows x 128 bytes per stage; the 16-byte slot of logical piece c of
// row r is stored at c ^ ((r >> 1) & 7), which makes the 16-row fragment
// reads conflict-free.  The loads of step s+1 are issued right after the
// barrier that opens step s, so they overlap its MFMAs and epilogue, across
// tile boundaries too.  Workgroups are persistent; tiles are ordered in
// groups of GM row tiles and dealt to the 8 XCDs in contiguous runs so that
// each XCD's L2 holds the row tiles of its group while S tiles stream past.
#include "join_params.hpp"

namespace dl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 512;
constexpr int kStageBytes = kTile * kChunkBytes;  // one operand, one K-chunk
constexpr int kWaveM = 128, kWaveN = 64;          // outputs per wave

typedef __attribute__((address_space(1))) void gvoid_t;
typedef __attribute__((address_space(3))) void lvoid_t;

// 16 bytes per lane from global memory into LDS (global_load_lds_dwordx4):
// lane l's bytes land at lds_dst + 16 l.  Issued as inline assembly so that
// the compiler's wait-count insertion does not treat the transfer as a
// write to the stage being read; the kernel orders it explicitly (vmcnt(0)
// and a barrier before a stage is read or overwritten).
__device__ inline void lds_dma16(const void* gsrc, void* lds_dst) {
  const uint32_t m0 = __builtin_amdgcn_readfirstlane(
      (uint32_t)reinterpret_cast<uintptr_t>((lvoid_t*)lds_dst));
  // M0 (the LDS base of the transfer) is saved and restored around the
  // transfer, and one wait state separates the M0 write from the LDS-DMA
  // instruction that reads it.
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %2\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %1, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "v"(gsrc), "s"(m0)
      : "memory");
}

// LDS byte offset of logical 16-byte piece c of tile row r.
__device__ inline int lds_off(int r, int c) { return r * kChunkBytes + ((c ^ ((r >> 1) & 7)) << 4); }

enum : int { kModeEps = 0, kModeBand = 1 };



// ------------------------------------------------------------- tile order
// Logical index -> (ti, tj) for the eps mode (see file comment).  Returns
// false for the skipped lower-triangle tiles of a self-join's diagonal groups.
__device__ inline bool tile_of(const CandParams& p, int64_t L, int64_t& ti, int64_t& tj) {
  const int64_t GM = p.GM;
  if (!p.self_join) {
    const int64_t g = L / (GM * p.nTS);
    const int64_t rem = L - g * GM * p.nTS;
    const int64_t gm = min(GM, p.nTR - g * GM);
    tj = rem / gm;
    ti = g * GM + rem % gm;
    return true;
  }
  // self-join: group g covers ti in [g*GM, g*GM+gm) and tj in [g*GM, nT)
  const int64_t nT = p.nTR;
  int64_t lo = 0, hi = p.ngroups - 1;
  while (lo < hi) {  // largest g with prefix(g) <= L
    const int64_t mid = (lo + hi + 1) >> 1;
    const int64_t pre = GM * (mid * nT - GM * mid * (mid - 1) / 2);
    if (pre <= L) lo = mid; else hi = mid - 1;
  }
  const int64_t g = lo;
  const int64_t rem = L - GM * (g * nT - GM * g * (g - 1) / 2);
  const int64_t gm = min(GM, nT - g * GM);
  tj = g * GM + rem / gm;
  ti = g * GM + rem % gm;
  return ti <= tj && tj < nT;
}

// Marks a block-uniform 64-bit value as such, so that it lives in scalar
// registers (the uniformity analysis loses tile indices carried around the
// persistent loop, and 64-bit vector copies of them crowd out the
// accumulators).
__device__ inline int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Block-uniform iterator over this workgroup's tiles.
struct TileIter {
  int64_t step;  // eps: logical round; band: S tile within split
  __device__ bool next(const CandParams& p, int mode, int64_t& ti, int64_t& tj) {
    if (mode == kModeEps) {
      const int64_t G = gridDim.x;
      const int64_t slot = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
      for (;;) {
        const int64_t L = step * G + slot;
        ++step;
        if (L >= p.nlogical) return false;
        if (tile_of(p, L, ti, tj)) {
          ti = uniform64(ti);
          tj = uniform64(tj);
          return true;
        }
      }
    } else {
      // work item: consecutive items share a split (S range), so the
      // concurrently running items of one XCD read the same S tiles
      const int64_t nb = gridDim.x;
      const int64_t w = (int64_t)(blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
      const int64_t split = w / p.nTR;
      ti = w % p.nTR;
      const int64_t t = split * p.tps + step;
      ++step;
      if (step > p.tps || t >= p.nTS) return false;
      ti = uniform64(ti);
      tj = uniform64(t);
      return true;
    }
  }
};

// ----------------------------------------------------- operand movement
// One K-chunk of both operand tiles, global -> LDS.  Each wave moves rows
// [8q, 8q+8) for q = 4 * wave + t (t < 4) of each operand with one 1 KiB
// global_load_lds_dwordx4: lane l fills LDS slot l of that block, i.e.
// row 8q + l/8, physical piece l%8, so it fetches logical piece
// (l%8) ^ ((row >> 1) & 7) of that row.
__device__ inline void issue_loads(const CandParams& p, int64_t ti, int64_t tj, int chunk, uint8_t* la, uint8_t* lb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave-uniform tile bases (scalar registers) + a 32-bit in-tile offset per
  // lane and t: few live registers, nothing worth hoisting across steps
  const uint8_t* ga0 = p.qa + (ti * kTile) * p.qld + (int64_t)chunk * kChunkBytes;
  const uint8_t* gb0 = p.qb + (tj * kTile) * p.qld + (int64_t)chunk * kChunkBytes;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int q = wave * 4 + t;
    const int row = q * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((row >> 1) & 7);
    const uint32_t off = (uint32_t)row * (uint32_t)p.qld + (uint32_t)(c * 16);
    lds_dma16(ga0 + off, la + q * 8 * kChunkBytes);
    lds_dma16(gb0 + off, lb + q * 8 * kChunkBytes);
  }
}

// ------------------------------------------------------ one K-chunk of MMA
// Every lane reads 16-byte pieces at (row = lane % 16, byte = group * 16)
// with group = lane / 16.  A and B use the same (lane, slot) -> k mapping,
// so the dot product is over all k of the chunk whatever order the matrix
// core assigns to the slots.
template <int kPrec>
__device__ inline void mma_chunk(f32x4 (&acc)[8][4], const uint8_t* la, const uint8_t* lb, int ra0, int rb0,
                                 const int (&sa)[8], const int (&sb)[4]) {
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, grp = lane >> 4;
  if constexpr (kPrec == DL_BF16 || kPrec == DL_FP16) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      uint4 bq[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        bq[nb] = *reinterpret_cast<const uint4*>(lb + lds_off(rb0 + nb * 16 + r16, ks * 4 + grp));
#pragma unroll
      for (int mb = 0; mb < 8; ++mb) {
        const uint4 aq = *reinterpret_cast<const uint4*>(la + lds_off(ra0 + mb * 16 + r16, ks * 4 + grp));
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          if constexpr (kPrec == DL_BF16)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, aq),
                                                                  __builtin_bit_cast(bf16x8, bq[nb]),
                                                                  acc[mb][nb], 0, 0, 0);
          else
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, aq),
                                                                 __builtin_bit_cast(f16x8, bq[nb]),
                                                                 acc[mb][nb], 0, 0, 0);
        }
      }
    }
  } else if constexpr (kPrec == DL_FP8) {
    // 16x16x128 E4M3 with per-row E8M0 scales; each lane reads 32 bytes
    i32x8 bq[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int r = rb0 + nb * 16 + r16;
      const uint4 x0 = *reinterpret_cast<const uint4*>(lb + lds_off(r, 2 * grp));
      const uint4 x1 = *reinterpret_cast<const uint4*>(lb + lds_off(r, 2 * grp + 1));
      bq[nb] = i32x8{(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w, (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
    }
#pragma unroll
    for (int mb = 0; mb < 8; ++mb) {
      const int r = ra0 + mb * 16 + r16;
      const uint4 x0 = *reinterpret_cast<const uint4*>(la + lds_off(r, 2 * grp));
      const uint4 x1 = *reinterpret_cast<const uint4*>(la + lds_off(r, 2 * grp + 1));
      const i32x8 aq = {(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w, (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(aq, bq[nb], acc[mb][nb], 0, 0, 0, sa[mb], 0,
                                                                      sb[nb]);
      // keep at most two 32-byte A fragments live (register pressure)
      if (mb & 1) __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    // fp32: 16x16x4; a 16-byte read gives 4 k-steps
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      float4 bq[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        bq[nb] = *reinterpret_cast<const float4*>(lb + lds_off(rb0 + nb * 16 + r16, half * 4 + grp));
#pragma unroll
      for (int mb = 0; mb < 8; ++mb) {
        const float4 aq = *reinterpret_cast<const float4*>(la + lds_off(ra0 + mb * 16 + r16, half * 4 + grp));
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.x, bq[nb].x, acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.y, bq[nb].y, acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.z, bq[nb].z, acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.w, bq[nb].w, acc[mb][nb], 0, 0, 0);
        }
      }
    }
  }
}

// -------------------------------------------------------------- epilogues
// Output element (mb, nb, r) of a lane sits at tile row wm*128 + mb*16 +
// 4*(lane/16) + r and tile column wn*64 + nb*16 + lane%16.
__device__ inline void epilogue_eps(const CandParams& p, int64_t ti, int64_t tj, const f32x4 (&acc)[8][4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int64_t row0 = ti * kTile + wm * kWaveM + 4 * (lane >> 4);
  const int64_t col0 = tj * kTile + wn * kWaveN + (lane & 15);
  float4 th[8];
  bool any = false;
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
    th[mb] = *reinterpret_cast<const float4*>(p.thr + row0 + mb * 16);
    // row maxima over the 4 column blocks, then one compare per row
    float m[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
      m[r] = fmaxf(fmaxf(acc[mb][0][r], acc[mb][1][r]), fmaxf(acc[mb][2][r], acc[mb][3][r]));
    any |= (m[0] >= th[mb].x) | (m[1] >= th[mb].y) | (m[2] >= th[mb].z) | (m[3] >= th[mb].w);
  }
  if (!__any(any)) return;
  // slow path: 128 hit bits per lane (bit (mb & 1) * 16 + nb * 4 + r of
  // word mb / 2), one wave-wide atomic for the whole tile, then each lane
  // writes its own hits.
  uint32_t hm[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
    const float tv[4] = {th[mb].x, th[mb].y, th[mb].z, th[mb].w};
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = row0 + mb * 16 + r, j = col0 + nb * 16;
        const bool v = acc[mb][nb][r] >= tv[r] && i < p.nR && j < p.nS && (!p.self_join || j > i);
        hm[mb >> 1] |= (uint32_t)v << ((mb & 1) * 16 + nb * 4 + r);
      }
    }
  }
  const uint32_t mine = __popc(hm[0]) + __popc(hm[1]) + __popc(hm[2]) + __popc(hm[3]);
  uint32_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  if (total == 0) return;
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(p.ccount, (unsigned long long)total);
  base = __shfl(base, 0, 64);
  unsigned long long pos = base + incl - mine;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t bits = hm[w];
    while (bits) {
      const int b = __builtin_ctz(bits);
      bits &= bits - 1;
      const int mb = 2 * w + (b >> 4), nb = (b >> 2) & 3, r = b & 3;
      if (pos < (unsigned long long)p.ccap)
        p.cand[pos] = make_uint2((uint32_t)(row0 + mb * 16 + r), (uint32_t)(col0 + nb * 16));
      ++pos;
    }
  }
}

__device__ inline uint32_t order_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float key_float(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

constexpr int kSelPerLane = 8;  // entries per lane in the k-selection subset

// Tighten one row's band and drop what falls below it (one wave).  The new
// threshold is P~_(k) - E_i with P~_(k) the k-th largest value of the first
// 64 * kSelPerLane entries: the k-th largest of a subset is at most the k-th
// largest of the whole buffer, so the band stays a superset of the exact
// one, and the selection runs on registers only.
// Scalar arguments only (a reference to the kernel's parameter block would
// force the block into scratch memory).
__device__ inline void compact_row(uint2* e, int n, float marg, float* bthr, int* bcnt, int k,
                                                      int cap, int* overflow) {
  const int lane = threadIdx.x & 63;
  float thr = *bthr;
  const int m = min(n, 64 * kSelPerLane);
  if (m >= k) {
    uint32_t key[kSelPerLane];
#pragma unroll
    for (int t = 0; t < kSelPerLane; ++t) {
      const int s = t * 64 + lane;
      key[t] = s < m ? order_key(__uint_as_float(e[s].x)) : 0u;
    }
    uint32_t kk = 0;  // largest key with at least k entries >= it
    for (int b = 31; b >= 0; --b) {
      const uint32_t cand = kk | (1u << b);
      int c = 0;
#pragma unroll
      for (int t = 0; t < kSelPerLane; ++t) c += key[t] >= cand;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
      if (c >= k) kk = cand;
    }
    thr = fmaxf(thr, f32_down((double)key_float(kk) - (double)marg));
  }
  int w = 0;
  const uint64_t lt = __lanemask_lt();
  for (int base = 0; base < n; base += 64) {
    const int s = base + lane;
    uint2 v = make_uint2(0, 0);
    bool keep = false;
    if (s < n) {
      v = e[s];
      keep = __uint_as_float(v.x) >= thr;
    }
    const uint64_t mm = __ballot(keep);
    if (keep) e[w + __popcll(mm & lt)] = v;
    w += __popcll(mm);
  }
  if (lane == 0) {
    *bthr = thr;
    *bcnt = w;
    if (w > cap - kTile) atomicOr(overflow, 1);
  }
}

// Band epilogue.  For each of the wave's 32 (row block, row) slots the row
// maximum over the four column blocks is tested against the row's band
// threshold; only a slot with a hit walks its four outputs.  Hits of one row
// are appended with one LDS atomic per 16-lane row group; an append that
// takes a row's buffer past cap - 256 queues the row for tightening (the
// buffer still has room for one more tile).
__device__ inline void epilogue_band(const CandParams& p, int64_t ti, int64_t tj, int64_t split, bool full,
                                     const f32x4 (&acc)[8][4], const float* lds_thr, int* lds_cnt, int* lds_list) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int lrow0 = wm * kWaveM + 4 * (lane >> 4);
  const uint32_t row0 = (uint32_t)(ti * kTile + lrow0);
  const uint32_t col0 = (uint32_t)(tj * kTile + wn * kWaveN + (lane & 15));
  const int limit = p.cap - kTile;
  const uint64_t lt = __lanemask_lt();
  const uint64_t gmask = 0xffffull << (lane & 48);  // the 16 lanes sharing this lane's row
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
    const float4 th = *reinterpret_cast<const float4*>(lds_thr + lrow0 + mb * 16);
    const float tv[4] = {th.x, th.y, th.z, th.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float mx = fmaxf(fmaxf(acc[mb][0][r], acc[mb][1][r]), fmaxf(acc[mb][2][r], acc[mb][3][r]));
      if (!__ballot(mx >= tv[r])) continue;
      const int lr = lrow0 + mb * 16 + r;
      const uint32_t i = row0 + mb * 16 + r;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const uint32_t j = col0 + nb * 16;
        bool hit = acc[mb][nb][r] >= tv[r];
        if (!full) hit = hit && i < (uint64_t)p.nR && j < (uint64_t)p.nS && !(p.exclude_self && i == j);
        const uint64_t m = __ballot(hit);
        if (!m) continue;
        const uint64_t gm = m & gmask;
        const int first = gm ? __ffsll((unsigned long long)gm) - 1 : 0;
        int base = 0;
        if (hit && lane == first) {
          const int cnt = __popcll(gm);
          base = atomicAdd(&lds_cnt[lr], cnt);
          if (base <= limit && limit < base + cnt) lds_list[1 + atomicAdd(&lds_list[0], 1)] = lr;
        }
        base = __shfl(base, first, 64);
        if (hit) {
          const int pos = base + __popcll(gm & lt);
          // the row's buffer address is formed here: hoisted out of the
          // tile loop for all 32 row slots it would be spilled to scratch
          uint32_t ii = i;
          asm volatile("" : "+v"(ii));
          if (pos < p.cap)
            p.band[((int64_t)ii * p.P + split) * (int64_t)p.cap + pos] = make_uint2(__float_as_uint(acc[mb][nb][r]), j);
        }
      }
    }
  }
}

// Rows queued by the band epilogue are tightened by one wave each; called by
// the whole workgroup right after a barrier, so lds_list[0] is uniform, and
// only at the first K-chunk of a tile, where the accumulators are dead (the
// queued rows are still tightened before the next epilogue appends).
__device__ inline void tighten_rows(const CandParams& p, int64_t ti, int64_t split, float* lds_thr, int* lds_cnt,
                                    int* lds_list) {
  const int nq = lds_list[0];
  if (nq == 0) return;
  const int wave = threadIdx.x >> 6;
  for (int q = wave; q < nq; q += kThreads / 64) {
    const int lr = lds_list[1 + q];
    const int64_t i = ti * kTile + lr;
    const int n = min(lds_cnt[lr], p.cap);
    compact_row(p.band + ((i * p.P) + split) * (int64_t)p.cap, n, p.marg[i], &lds_thr[lr], &lds_cnt[lr], p.k, p.cap,
                p.overflow);
  }
  __syncthreads();
  if (threadIdx.x == 0) lds_list[0] = 0;
  __syncthreads();
}

// ------------------------------------------------------------------ kernel
template <int kPrec, int kMode>
__global__ __launch_bounds__(kThreads, 1) void cand_kernel(CandParams p) {
  // two stages of (A chunk, B chunk)
  __shared__ __attribute__((aligned(1024))) uint8_t lds_ab[2][2][kStageBytes];
  __shared__ __attribute__((aligned(16))) float lds_thr[kMode == kModeBand ? kTile : 1];
  __shared__ int lds_cnt[kMode == kModeBand ? kTile : 1];
  __shared__ int lds_list[kMode == kModeBand ? kTile + 1 : 1];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  TileIter it{0};
  int64_t ti, tj;
  if (!it.next(p, kMode, ti, tj)) return;
  int64_t split = 0;
  if constexpr (kMode == kModeBand) {
    const int64_t nb = gridDim.x;
    const int64_t w = (int64_t)(blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    split = uniform64(w / p.nTR);
    for (int r = threadIdx.x; r < kTile; r += kThreads) {
      lds_thr[r] = -INFINITY;
      lds_cnt[r] = 0;
    }
    if (threadIdx.x == 0) lds_list[0] = 0;
  }
  int chunk = 0, stage = 0;
  bool full = true;  // band mode: the tile needs no bounds or self checks
  issue_loads(p, ti, tj, 0, lds_ab[0][0], lds_ab[0][1]);
  f32x4 acc[8][4];
  int sa[8], sb[4];
  for (;;) {
    int64_t nti = ti, ntj = tj;
    int nchunk = chunk + 1;
    bool more = true;
    if (nchunk == p.nchunks) {
      nchunk = 0;
      more = it.next(p, kMode, nti, ntj);
    }
    // This step's operands are in LDS once this wave's loads have landed
    // (vmcnt) and every wave has passed the barrier; the barrier also means
    // every wave is done reading the other stage (it computed the previous
    // step before arriving), so the next step's loads may overwrite it.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (chunk == 0) {
      if constexpr (kMode == kModeBand) {
        tighten_rows(p, ti, split, lds_thr, lds_cnt, lds_list);
        full = (ti + 1) * kTile <= p.nR && (tj + 1) * kTile <= p.nS && !(p.exclude_self && ti == tj);
      }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int64_t j = tj * kTile + wn * kWaveN + nb * 16 + (lane & 15);
        const float init = -p.hb[j];
#pragma unroll
        for (int mb = 0; mb < 8; ++mb) acc[mb][nb] = f32x4{init, init, init, init};
        if constexpr (kPrec == DL_FP8) sb[nb] = p.sexb[j] + 127;
      }
      if constexpr (kPrec == DL_FP8) {
#pragma unroll
        for (int mb = 0; mb < 8; ++mb) sa[mb] = p.sexa[ti * kTile + wm * kWaveM + mb * 16 + (lane & 15)] + 127;
      }
      // the initial values are in registers before the next step's
      // transfers are queued behind them
      __builtin_amdgcn_s_waitcnt(0);
    }
    if (more) issue_loads(p, nti, ntj, nchunk, lds_ab[stage ^ 1][0], lds_ab[stage ^ 1][1]);
    mma_chunk<kPrec>(acc, lds_ab[stage][0], lds_ab[stage][1], wm * kWaveM, wn * kWaveN, sa, sb);
    if (chunk == p.nchunks - 1) {
      if constexpr (kMode == kModeEps) epilogue_eps(p, ti, tj, acc);
      else epilogue_band(p, ti, tj, split, full, acc, lds_thr, lds_cnt, lds_list);
    }
    if (!more) break;
    ti = nti;
    tj = ntj;
    chunk = nchunk;
    stage ^= 1;
  }
  if constexpr (kMode == kModeBand) {
    __syncthreads();
    tighten_rows(p, ti, split, lds_thr, lds_cnt, lds_list);
    for (int r = threadIdx.x; r < kTile; r += kThreads) {
      const int64_t i = ti * kTile + r;
      if (i < p.nR) p.bcount[i * p.P + split] = min(lds_cnt[r], p.cap);
    }
  }
}

// ------------------------------------------------------------ host launch
template <int kMode>
static hipError_t launch_mode(dl_prec prec, const CandParams& p, dim3 grid, hipStream_t st) {
  switch (prec) {
    case DL_FP32: hipLaunchKernelGGL((cand_kernel<DL_FP32, kMode>), grid, dim3(kThreads), 0, st, p); break;
    case DL_BF16: hipLaunchKernelGGL((cand_kernel<DL_BF16, kMode>), grid, dim3(kThreads), 0, st, p); break;
    case DL_FP16: hipLaunchKernelGGL((cand_kernel<DL_FP16, kMode>), grid, dim3(kThreads), 0, st, p); break;
    case DL_FP8: hipLaunchKernelGGL((cand_kernel<DL_FP8, kMode>), grid, dim3(kThreads), 0, st, p); break;
  }
  return hipGetLastError();
}

// Row tiles per group: keep the group's row tiles within about 1 MiB so they
// stay resident in an XCD's 4 MiB L2 beside the streaming S tiles.
static int group_rows(int64_t qld, int64_t nTR) {
  int64_t gm = (int64_t)(1 << 20) / (kTile * qld);
  gm = gm < 1 ? 1 : (gm > 16 ? 16 : gm);
  if (gm > nTR) gm = nTR;
  return (int)gm;
}

hipError_t launch_cand_eps(dl_prec prec, CandParams p, hipStream_t st, int cu_count) {
  p.nTR = (p.nR + kTile - 1) / kTile;
  p.nTS = (p.nS + kTile - 1) / kTile;
  if (p.nTR == 0 || p.nTS == 0) return hipSuccess;
  p.GM = group_rows(p.qld, p.nTR);
  p.ngroups = (p.nTR + p.GM - 1) / p.GM;
  if (p.self_join) {
    const int64_t g = p.ngroups;
    p.nlogical = (int64_t)p.GM * (g * p.nTR - (int64_t)p.GM * g * (g - 1) / 2);
  } else {
    p.nlogical = p.nTR * p.nTS;
  }
  int64_t G = cu_count;  // one 512-thread workgroup per CU
  const int64_t need = (p.nlogical + 7) / 8 * 8;
  if (G > need) G = need;
  G = (G + 7) / 8 * 8;
  return launch_mode<kModeEps>(prec, p, dim3((unsigned)G), st);
}

hipError_t launch_cand_band(dl_prec prec, CandParams p, hipStream_t st) {
  p.nTR = (p.nR + kTile - 1) / kTile;
  p.nTS = (p.nS + kTile - 1) / kTile;
  if (p.nTR == 0 || p.nTS == 0) return hipSuccess;
  p.tps = (p.nTS + p.P - 1) / p.P;
  const int64_t items = p.nTR * p.P;
  // the XCD dealing in TileIter needs a multiple of 8 workgroups; the extra
  // ones find no S tiles and exit
  const int64_t G = (items + 7) / 8 * 8;
  return launch_mode<kModeBand>(prec, p, dim3((unsigned)G), st);
}

}  // namespace dl
