// join_mfma.hip -- candidate pass of the similarity join on CDNA4 matrix cores.
//
// Paper: section "Query Processing" (Nested Loop Join over all pairs of two
// patch collections) with the Euclidean predicate of section "Derived Data"
// and the closest-image query q1 of section "Queries".  The nested loop is
// recast as a tiled product G = A B^T of the two relations' operand copies:
// each 256 x 256 tile of pairs accumulates P~ = a.b - |b|^2/2 (the
// accumulator starts at -h_j) over K-steps of 128 bytes on the matrix
// cores, and the epilogue compares P~ with one per-row float:
//   eps mode   P~ >= thr_i  (thr_i folds |a|^2, the threshold T and the
//              rigorous margin E_i) -> append (i, j) to the candidate list;
//   band mode  P~ >= band_i, a running top-k band per row kept in LDS ->
//              append (P~, j) to the row's band buffer, tightening band_i
//              to (a lower bound of) P~_(k) - E_i every few dozen appends.
// Candidates are a superset of the exact result; the recheck kernels decide
// exactly.
//
// Layout: 512 threads = 8 waves in a 2 x 4 grid, each wave owns 128 x 64
// outputs as 8 x 4 blocks of 16 x 16 (v_mfma_*_16x16x*), 32 f32x4
// accumulators.  Operands move global -> LDS directly
// (global_load_lds_dwordx4, no staging registers) into a 128 KiB ring of
// two stages of 256 rows x 128 bytes per operand.  The 16-byte piece c of row r is
// stored at a slot c ^ f(r) that makes the 16-row fragment reads
// conflict-free.  The loader runs kStages - 1 K-steps ahead of the matrix
// cores, across tile boundaries too; per-tile side data (h_j, thresholds,
// E4M3 scales) travels the same way, so the loop waits only on its own
// transfer counts.  Workgroups are persistent; tiles are ordered in groups of
// GM row tiles and dealt to the 8 XCDs in contiguous runs so that each XCD's
// L2 holds the row tiles of its group while S tiles stream past.
#include "join_params.hpp"

namespace dl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 512;
constexpr int kWaveM = 128, kWaveN = 64;  // outputs per wave
constexpr int kRingBytes = 128 * 1024;   // LDS operand ring, all stages

// K-step geometry.  A K-step moves kCB bytes of each of the 256 A rows and
// 256 B rows into one stage of the ring.  128-byte steps (two stages) are
// used for every format: E4M3 needs them (the scaled matrix instruction has
// K = 128), and for the others they measured faster than 64-byte steps with
// four stages, whose extra barrier per 32 matrix instructions cost more than
// the deeper prefetch saved.  The code below handles either geometry.
template <int kPrec>
struct Pipe {
  static constexpr int kCB = 128;
  static constexpr int kSlots = kCB / 16;                         // 16-byte pieces per row
  static constexpr int kStageBytes = kTile * kCB;                 // one operand, one step
  static constexpr int kStages = kRingBytes / (2 * kStageBytes);  // 2 or 4
  static constexpr int kRowsPerDma = 1024 / kCB;                  // rows per 1 KiB transfer
};

typedef __attribute__((address_space(1))) void gvoid_t;
typedef __attribute__((address_space(3))) void lvoid_t;

// 16 bytes per lane from global memory into LDS (global_load_lds_dwordx4):
// lane l's bytes land at lds_dst + 16 l.  Issued as inline assembly so that
// the compiler's wait-count insertion does not treat the transfer as a
// write to the stage being read; the kernel orders it explicitly (vmcnt(0)
// and a barrier before a stage is read or overwritten).
__device__ inline uint32_t lds_addr(const void* lds_ptr) {
  return __builtin_amdgcn_readfirstlane((uint32_t)reinterpret_cast<uintptr_t>((const lvoid_t*)lds_ptr));
}
// the same with the LDS destination given as a wave-uniform LDS address
__device__ inline void lds_dma16_at(const void* gsrc, uint32_t m0) {
  // M0 (the LDS base of the transfer) is an operand bound to the register,
  // so the compiler knows it is written; one wait state separates the M0
  // write from the LDS-DMA instruction that reads it.
  asm volatile(
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %0, off"
      :
      : "v"(gsrc), "{m0}"(m0)
      : "memory");
}
__device__ inline void lds_dma16(const void* gsrc, void* lds_dst) { lds_dma16_at(gsrc, lds_addr(lds_dst)); }

// LDS byte offset of logical 16-byte piece c of tile row r in a stage with
// kCB bytes per row.  The piece is stored at slot c ^ f(r), which spreads the
// 16 rows read by one 16-lane group over all 64 banks.
template <int kCB>
__device__ inline int lds_off(int r, int c) {
  if constexpr (kCB == 128) return r * 128 + ((c ^ ((r >> 1) & 7)) << 4);
  else return r * 64 + ((c ^ ((r >> 2) & 3)) << 4);
}

// eps: append candidates; band: top-k band; mark: the bound pass of the
// index-pruned join (rows are block centroids, columns data rows; a hit sets
// the block's bit for the data row's tile); nearest: each row's column of
// largest P~ (the pivot assignment of the index-pruned join).
enum : int { kModeEps = 0, kModeBand = 1, kModeMark = 2, kModeNearest = 3 };

// Waves that issue the operand transfers (waves w and w + 4 share a SIMD).
// Fewer issuing waves leave more waves free of transfers to feed the matrix
// cores while the issuers wait on the vector-memory queue.  Measured: eps
// mode is 1-2% faster with two issuers than with four (eight lose 6%); band
// mode, whose epilogue and tightening already load waves unevenly, is 1%
// faster with four.
template <int kMode>
constexpr int dma_waves() { return kMode == kModeBand ? 4 : 2; }
template <int kMode>
constexpr int dma_per_op(int rows_per_dma) { return kTile / rows_per_dma / dma_waves<kMode>(); }



// ------------------------------------------------------------- tile order
// Logical index -> (ti, tj) for the eps mode (see file comment).  Returns
// false for the skipped lower-triangle tiles of a self-join's diagonal
// groups.  (Measured: this closed form, whose divisions by block-uniform
// values compile to scalar code, beats carrying (group, offset) forward
// with vector-unit 32-bit divisions.)
// Division of a 32-bit block-uniform n by an invariant d through a
// multiply-high and shifts (Granlund and Montgomery, "Division by Invariant
// Integers using Multiplication", PLDI 1994): q = (t + ((n - t) >> s1)) >> s2
// with t = mulhi(m, n); m, s1, s2 come from the host (div_magic).
__device__ inline uint32_t udiv32(uint32_t n, uint32_t m, uint32_t s1, uint32_t s2) {
  const uint32_t t = __umulhi(n, m);
  return (t + ((n - t) >> s1)) >> s2;
}

__device__ inline bool tile_of(const CandParams& p, int64_t L, int64_t& ti, int64_t& tj) {
  const int64_t GM = p.GM;
  if (p.small32) {
    // every index below fits 32 bits: scalar multiply-high divisions
    const uint32_t l = (uint32_t)L, gmax = (uint32_t)GM;
    uint32_t g, rem;
    if (!p.self_join) {
      g = udiv32(l, p.dv_grp_m, p.dv_grp_s1, p.dv_grp_s2);
      rem = l - g * (gmax * (uint32_t)p.nTS);
    } else {
      const int64_t nT = p.nTR;
      int64_t lo = 0, hi = p.ngroups - 1;
      while (lo < hi) {  // largest g with prefix(g) <= L
        const int64_t mid = (lo + hi + 1) >> 1;
        const int64_t pre = GM * (mid * nT - GM * mid * (mid - 1) / 2);
        if (pre <= L) lo = mid; else hi = mid - 1;
      }
      g = (uint32_t)lo;
      rem = (uint32_t)(L - GM * ((int64_t)g * nT - GM * (int64_t)g * (g - 1) / 2));
    }
    const bool last = (int64_t)g == p.ngroups - 1;
    const uint32_t gm = last ? (uint32_t)(p.nTR - (int64_t)g * GM) : gmax;
    const uint32_t q = last ? udiv32(rem, p.dv_gl_m, p.dv_gl_s1, p.dv_gl_s2) : udiv32(rem, p.dv_gm_m, p.dv_gm_s1, p.dv_gm_s2);
    const int64_t g0 = (int64_t)g * GM;
    tj = (p.self_join ? g0 : 0) + (int64_t)q;
    ti = g0 + (int64_t)(rem - q * gm);
    return !p.self_join || (ti <= tj && tj < p.nTR);
  }
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

// This lane's index (0..63), recomputed from the lane-count instructions at
// every use.  Lane-derived offsets formed from it are not hoisted out of the
// persistent loop, where they would stay live beside the 128 accumulator
// registers and be spilled.
__device__ inline int fresh_lane() {
  int l;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
  return l;
}

// Block-uniform iterator over this workgroup's tiles: eps (and mark) mode
// walks logical tiles slot, slot + G, ... (G workgroups; slot = the
// workgroup's place in the XCD dealing), either all tiles in the group order
// or the entries of a tile list (p.tiles, *p.ntiles of them); band mode walks
// the S tiles of one (row tile, split) work item, fixed at the first call.
struct TileIter {
  int64_t step = 0;                              // eps: logical round
  int64_t lim = -1;                              // eps: logical tiles
  int64_t ti = 0, split = 0, t = 0, t_end = 0;   // band
  bool list = false;                             // eps: walking the tile list
  __device__ bool next(const CandParams& p, int mode, int64_t& oti, int64_t& otj) {
    const int64_t G = gridDim.x;
    const int64_t slot = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
    if (mode != kModeBand) {
      if (lim < 0) {
        // a long list costs a cache-missing read per tile that the grid's
        // order computes, so when most tiles are listed the grid is walked
        const int64_t nl = p.tiles ? uniform64((int64_t)*p.ntiles) : 0;
        list = p.tiles && (p.list_all == 0 || 2 * nl < p.list_all);
        lim = list ? nl : p.nlogical;
      }
      for (;;) {
        const int64_t L = step * G + slot;
        ++step;
        if (L >= lim) return false;
        int64_t ti_, tj_;
        if (list) {
          const uint2 t2 = p.tiles[L];
          oti = uniform64((int64_t)t2.x);
          otj = uniform64((int64_t)t2.y);
          return true;
        }
        if (tile_of(p, L, ti_, tj_)) {
          oti = uniform64(ti_);
          otj = uniform64(tj_);
          return true;
        }
      }
    } else {
      if (t_end == 0) {
        // consecutive items share a split (S range), so the concurrently
        // running items of one XCD read the same S tiles
        split = slot / p.nTR;
        ti = slot % p.nTR;
        t = split * p.tps;
        t_end = min(t + p.tps, p.nTS);
        if (t >= t_end) t_end = -1;  // no S tiles for this workgroup
      }
      // tiles the index cannot rule out only (a row tile's survivor bits)
      if (p.surv)
        while (t < t_end && !((p.surv[ti * p.sw + (t >> 5)] >> (t & 31)) & 1u)) ++t;
      if (t_end < 0 || t >= t_end) return false;
      oti = uniform64(ti);
      otj = uniform64(t);
      ++t;
      return true;
    }
  }
};

// K-steps of tile (ti, tj), bit s for step s.  With the per-tile masks a
// step where every row of one of the two tiles is zero is dropped: each of
// its products is zero, and adding zero leaves every accumulator as it was
// (the inputs are finite).  A tile keeps at least one step, whose products
// are then all zero, so its epilogue still runs on the initial values.
__device__ inline uint64_t tile_steps(const CandParams& p, int64_t ti, int64_t tj) {
  const uint64_t m = p.kmaskA[ti] & p.kmaskB[tj];
  return m ? m : 1ull;
}

// ----------------------------------------------------- operand movement
// One K-step of both operand tiles, global -> LDS.  Each wave moves blocks
// q = kDmaPerOp * wave + t of each operand, kRowsPerDma rows per block, with
// one 1 KiB global_load_lds_dwordx4: lane l fills LDS slot l of the block,
// i.e. row q * kRowsPerDma + l / kSlots, physical piece l % kSlots, so it
// fetches the logical piece that the swizzle puts there.

template <int kPrec, int kMode>
__device__ inline void issue_loads(const CandParams& p, int64_t ti, int64_t tj, int step, uint8_t* la, uint8_t* lb) {
  constexpr int kDmaWaves = dma_waves<kMode>();
  using Q = Pipe<kPrec>;
  // wave-uniform tile bases and LDS destinations (scalar registers) + a
  // 32-bit in-tile offset per lane and block, recomputed from an opaque lane
  // index at every call: hoisted out of the loop, the offsets would stay
  // live (and be spilled) beside the accumulators
  const int lane = fresh_lane();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wave >= kDmaWaves) return;
  constexpr int kPer = dma_per_op<kMode>(Q::kRowsPerDma);  // blocks per issuing wave and operand
  const uint8_t* ga0 = p.qa + (ti * kTile) * p.qld + (int64_t)step * Q::kCB;
  const int64_t dba = (p.qb + (tj * kTile) * p.qld) - (p.qa + (ti * kTile) * p.qld);  // B source - A source
  // The swizzle key of a row repeats every 2 * kRowsPerDma rows, so block t
  // reads at the lane offset of block t & 1 plus (t - (t & 1)) *
  // kRowsPerDma rows: two per-lane addresses, the rest is scalar.
  static_assert(Q::kCB == 128 ? (2 * Q::kRowsPerDma) % 16 == 0 : (2 * Q::kRowsPerDma) % 32 == 0,
                "swizzle period");
  auto lane_src = [&](int u) {
    const int row = (wave * kPer + u) * Q::kRowsPerDma + lane / Q::kSlots;
    const int phys = lane % Q::kSlots;
    const int c = (lds_off<Q::kCB>(row, phys) - row * Q::kCB) >> 4;  // the swizzle is an involution
    return ga0 + ((uint32_t)row * (uint32_t)p.qld + (uint32_t)(c * 16));
  };
  const uint8_t* const pa0 = lane_src(0);
  const uint8_t* const pa1 = lane_src(1);
  const uint32_t la0 = lds_addr(la) + wave * kPer * 1024, lb0 = lds_addr(lb) + wave * kPer * 1024;
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const uint8_t* a = ((t & 1) ? pa1 : pa0) + (int64_t)((t & ~1) * Q::kRowsPerDma) * p.qld;
    lds_dma16_at(a, la0 + t * 1024);
    lds_dma16_at(a + dba, lb0 + t * 1024);
  }
}

// Per-tile side data moved with the first K-step of a tile, one 1 KiB
// transfer each (256 four-byte values): h_j of the S tile, the eps
// thresholds of the R tile, the E4M3 row scales of both.  Keeping them in
// LDS means the loop's only global reads are these transfers, ordered by
// the kernel's own wait counts.
struct SideRefs {
  float* hb;
  float* thr;
  int* sa;
  int* sb;
};
template <int kPrec, int kMode>
__device__ inline void issue_side(const CandParams& p, int64_t ti, int64_t tj, const SideRefs& d) {
  // by the waves that issue no operand transfers, if there are such
  constexpr int kDmaWaves = dma_waves<kMode>();
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) - (kDmaWaves < 8 ? kDmaWaves : 0);
  const int e = 4 * fresh_lane();
  if (w == 0) lds_dma16(p.hb + tj * kTile + e, d.hb);
  if constexpr (kMode == kModeEps || kMode == kModeMark)
    if (w == 1) lds_dma16(p.thr + ti * kTile + e, d.thr);
  if constexpr (kPrec == DL_FP8) {
    if (w == 2) lds_dma16(p.sexa + ti * kTile + e, d.sa);
    if (w == 3) lds_dma16(p.sexb + tj * kTile + e, d.sb);
  }
}

// ------------------------------------------------------- one K-step of MMA
// Every lane reads 16-byte pieces at (row = lane % 16, piece = lane / 16 +
// 4 * sub-step).  A and B use the same (lane, slot) -> k mapping, so the dot
// product is over all k of the step whatever order the matrix core assigns
// to the slots.
//
// Fragment reads run ahead of the matrix instructions in a rolling window:
// the first sub-step's fragments are requested up front, in the order the
// matrix instructions use them (A0, B0..B3, A1..A7); the second
// sub-step's A fragment mb (and B fragment nb) is requested right after the
// instructions that consume the register it replaces.  The LDS latency is
// then paid about once per step instead of once per pair of A fragments,
// with 64 fragment registers beside the 128 accumulator registers.
//
// kFirst (a tile's first K-step): the first instruction of each block reads
// its C operand from init[nb] (the block's initial value -h_j, one register
// quad per column block) and writes the accumulator, so no per-tile copy of
// the initial values into the 128 accumulator registers is needed.

// Fragment registers of a K-step (16-bit formats and fp32): the first
// sub-step's A and B fragments, then the second sub-step's.  They live
// across the barrier between K-steps: the second sub-step's products of A
// blocks kTailFrom..7 are issued at the start of the next K-step (kTailIn),
// after that step's first fragment reads, so the matrix core has work while
// those reads land; a tile's last K-step leaves them to mma_tail, before the
// epilogue.
struct Frags {
  uint4 a[8], b0[4], b1[4];
};
constexpr int kTailFrom = 4;  // first A block whose second-sub-step products are deferred

// one block product c = c0 + x.y: 16x16x32 for the 16-bit formats, four
// 16x16x4 for fp32
template <int kPrec>
__device__ inline void mac_block(f32x4& c, const f32x4& c0, const uint4& x, const uint4& y) {
  if constexpr (kPrec == DL_BF16) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, x), __builtin_bit_cast(bf16x8, y), c0, 0,
                                                0, 0);
  } else if constexpr (kPrec == DL_FP16) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, x), __builtin_bit_cast(f16x8, y), c0, 0, 0,
                                               0);
  } else {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.x), __uint_as_float(y.x), c0, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.y), __uint_as_float(y.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.z), __uint_as_float(y.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.w), __uint_as_float(y.w), c, 0, 0, 0);
  }
}

// The products a K-step leaves for later: second sub-step, A blocks
// kTailFrom..7.
template <int kPrec>
__device__ inline void mma_tail(f32x4 (&acc)[8][4], const Frags& fr) {
  if constexpr (kPrec != DL_FP8) {
#pragma unroll
    for (int mb = kTailFrom; mb < 8; ++mb) {
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) mac_block<kPrec>(acc[mb][nb], acc[mb][nb], fr.a[mb], fr.b1[nb]);
    }
  }
}

// The first sub-step's first fragments of a 16-bit K-step (A0, B0..B3,
// A1..A3), in the order of first use: the first instruction waits for two
// reads.  mma_step issues them itself unless kReadsDone (the eps pass issues
// them, then runs the previous tile's epilogue while they land).
template <int kPrec>
__device__ inline void mma_first_reads(const uint8_t* la, const uint8_t* lb, int ra0, int rb0, Frags& fr) {
  constexpr int kCB = Pipe<kPrec>::kCB;
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, grp = lane >> 4;
  fr.a[0] = *reinterpret_cast<const uint4*>(la + lds_off<kCB>(ra0 + r16, grp));
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) fr.b0[nb] = *reinterpret_cast<const uint4*>(lb + lds_off<kCB>(rb0 + nb * 16 + r16, grp));
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int mb = 1; mb < kTailFrom; ++mb)
    fr.a[mb] = *reinterpret_cast<const uint4*>(la + lds_off<kCB>(ra0 + mb * 16 + r16, grp));
  __builtin_amdgcn_sched_barrier(0);
}

template <int kPrec, bool kFirst, bool kTailIn, bool kReadsDone = false>
__device__ inline void mma_step(f32x4 (&acc)[8][4], const uint8_t* la, const uint8_t* lb, int ra0, int rb0,
                                const int (&sa)[8], const int (&sb)[4], const f32x4 (&init)[4], Frags& fr) {
  constexpr int kCB = Pipe<kPrec>::kCB;
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, grp = lane >> 4;
  auto ldA = [&](int mb, int piece) {
    return *reinterpret_cast<const uint4*>(la + lds_off<kCB>(ra0 + mb * 16 + r16, piece));
  };
  auto ldB = [&](int nb, int piece) {
    return *reinterpret_cast<const uint4*>(lb + lds_off<kCB>(rb0 + nb * 16 + r16, piece));
  };
  if constexpr (kPrec == DL_BF16 || kPrec == DL_FP16 || kPrec == DL_FP32) {
    static_assert(kCB == 128, "two sub-steps of 64 bytes");
    static_assert(!(kFirst && kTailIn), "a tile's first K-step has no earlier products pending");
    constexpr int kPerBlock = kPrec == DL_FP32 ? 4 : 1;  // matrix instructions per block product
    uint4(&a)[8] = fr.a;
    uint4(&b0)[4] = fr.b0;
    uint4(&b1)[4] = fr.b1;
    if constexpr (!kReadsDone) mma_first_reads<kPrec>(la, lb, ra0, rb0, fr);
    if constexpr (kTailIn) {
      mma_tail<kPrec>(acc, fr);  // the previous K-step's pending products
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int mb = kTailFrom; mb < 8; ++mb) a[mb] = ldA(mb, grp);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int mb = 0; mb < 8; ++mb) {
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) mac_block<kPrec>(acc[mb][nb], kFirst ? init[nb] : acc[mb][nb], a[mb], b0[nb]);
      a[mb] = ldA(mb, 4 + grp);
      if (mb < 4) b1[mb] = ldB(mb, 4 + grp);
      __builtin_amdgcn_sched_group_barrier(0x008, 4 * kPerBlock, 0);  // matrix
      if (mb < 4) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);   // LDS reads
      else __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
#pragma unroll
    for (int mb = 0; mb < kTailFrom; ++mb) {
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) mac_block<kPrec>(acc[mb][nb], acc[mb][nb], a[mb], b1[nb]);
    }
    // A blocks kTailFrom..7 of the second sub-step: mma_tail, at the next
    // K-step or before the epilogue
  } else {
    // E4M3, 128 bytes = 128 values per row: 16x16x128 with per-row E8M0
    // scales; each lane reads 32 bytes per fragment; a window of four A
    // fragments
    auto ld8 = [&](const uint4& x0, const uint4& x1) {
      return i32x8{(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w, (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
    };
    i32x8 b[4], a[4];
    a[0] = ld8(ldA(0, 2 * grp), ldA(0, 2 * grp + 1));
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) b[nb] = ld8(ldB(nb, 2 * grp), ldB(nb, 2 * grp + 1));
#pragma unroll
    for (int mb = 1; mb < 4; ++mb) a[mb] = ld8(ldA(mb, 2 * grp), ldA(mb, 2 * grp + 1));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int mb = 0; mb < 8; ++mb) {
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[mb & 3], b[nb],
                                                                      kFirst ? init[nb] : acc[mb][nb], 0, 0, 0,
                                                                      sa[mb], 0, sb[nb]);
      if (mb < 4) a[mb] = ld8(ldA(mb + 4, 2 * grp), ldA(mb + 4, 2 * grp + 1));
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
      if (mb < 4) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
    }
  }
}

// -------------------------------------------------------------- epilogues
// Output element (mb, nb, r) of a lane sits at tile row wm*128 + mb*16 +
// 4*(lane/16) + r and tile column wn*64 + nb*16 + lane%16.
constexpr int kQueue = 256;  // staged hits per wave (eps candidates or band entries)

// Appends a wave's staged (i, j) candidates to the global list: one atomic
// for the whole batch, then coalesced stores.  Positions past the list's
// capacity are counted but not written (the caller then retries with room).
// With kP, each record's P~ (qp, staged beside q) goes to p.candp too.
template <bool kP>
__device__ inline void flush_eps(const CandParams& p, const uint2* q, const uint32_t* qp, int nq) {
  const int lane = fresh_lane();
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(p.ccount, (unsigned long long)nq);
  base = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
         __builtin_amdgcn_readfirstlane((uint32_t)base);
  for (int s = lane; s < nq; s += 64) {
    const unsigned long long pos = base + (unsigned long long)s;
    if (pos < (unsigned long long)p.ccap) {
      p.cand[pos] = q[s];
      if constexpr (kP)
        if (p.candp) p.candp[pos] = __uint_as_float(qp[s]);
    }
  }
}

// Eps epilogue.  A fast test (each row's maximum over the wave's four
// column blocks against the row threshold) lets most waves skip the tile,
// and records which of the eight row blocks hold a hit.  Only those blocks
// are visited after it: each of their (row block, row) slots with a hit
// forms its four hit masks and stages its (i, j) in the wave's LDS queue
// (ballot prefix, no atomics); the queue persists across tiles and goes to
// global memory only when full and at the end.  Bounds (rows and columns
// left in the tile) and the self-join's j > i (only on a diagonal tile) are
// checked in 32-bit tile coordinates, and only on tiles that need them.
// With kP each record's P~ is staged too (qp).  Returns whether this wave
// wrote to global memory.
template <bool kP>
__device__ inline bool epilogue_eps(const CandParams& p, int64_t ti, int64_t tj, const f32x4 (&acc)[8][4],
                                    const float* thr_tile, uint2* q, uint32_t* qp, int& nq) {
  const int lane = fresh_lane(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 2, wn = wave & 3;
  const int lrow0 = wm * kWaveM + 4 * (lane >> 4);
  const int lcol0 = wn * kWaveN + (lane & 15);
  float4 th[8];
  uint32_t hit_mb = 0;  // bit mb: row block mb holds a hit (wave-uniform)
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
    th[mb] = *reinterpret_cast<const float4*>(thr_tile + lrow0 + mb * 16);
    float m[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) m[r] = max4_nan(acc[mb][0][r], acc[mb][1][r], acc[mb][2][r], acc[mb][3][r]);
    const uint64_t h =
        mask_uge(m[0], th[mb].x) | mask_uge(m[1], th[mb].y) | mask_uge(m[2], th[mb].z) | mask_uge(m[3], th[mb].w);
    hit_mb |= (h != 0 ? 1u : 0u) << mb;
  }
  if (!hit_mb) return false;
  const int rrem = (int)min(p.nR - ti * kTile, (int64_t)kTile);
  const int crem = (int)min(p.nS - tj * kTile, (int64_t)kTile);
  const bool diag = p.self_join && ti == tj;
  const bool full = rrem == kTile && crem == kTile && !diag;
  const uint32_t i0 = (uint32_t)(ti * kTile), j0 = (uint32_t)(tj * kTile);
  const uint64_t lt = __lanemask_lt(), lbit = lt + 1;
  bool wrote = false;
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
    if (!(hit_mb & (1u << mb))) continue;
    const float tv[4] = {th[mb].x, th[mb].y, th[mb].z, th[mb].w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (!mask_uge(max4_nan(acc[mb][0][r], acc[mb][1][r], acc[mb][2][r], acc[mb][3][r]), tv[r])) continue;
      const int lr = lrow0 + mb * 16 + r;
      uint64_t m[4];
      int tot = 0;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        m[nb] = mask_ge(acc[mb][nb][r], tv[r]);
        if (!full) {
          const int lc = lcol0 + nb * 16;
          m[nb] &= __builtin_amdgcn_ballot_w64(lr < rrem && lc < crem && (!diag || lc > lr));
        }
        tot += __popcll(m[nb]);
      }
      if (nq + tot > kQueue) {
        flush_eps<kP>(p, q, qp, nq);
        nq = 0;
        wrote = true;
      }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        if (m[nb] & lbit) {
          const int at = nq + __popcll(m[nb] & lt);
          q[at] = make_uint2(i0 + (uint32_t)lr, j0 + (uint32_t)(lcol0 + nb * 16));
          if constexpr (kP) qp[at] = __float_as_uint(acc[mb][nb][r]);
        }
        nq += __popcll(m[nb]);
      }
    }
  }
  return wrote;
}

// Mark epilogue (the bound pass of the index-pruned join).  Rows of the
// tile are block centroids, columns the data rows of tile tj; every row with
// a hit in any valid column sets its bit in tj's row of p.mark.  A lane's
// outputs of (mb, r) lie on row mb*16 + 4*(lane/16) + r of the wave, so each
// 16-lane group of a hit mask is one row.  Rows past the centroids have an
// infinite threshold and never hit.
__device__ inline void epilogue_mark(const CandParams& p, int64_t ti, int64_t tj, const f32x4 (&acc)[8][4],
                                     const float* thr_tile) {
  const int lane = fresh_lane(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 2, wn = wave & 3;
  const int lrow0 = wm * kWaveM + 4 * (lane >> 4);
  const int lcol0 = wn * kWaveN + (lane & 15);
  const int crem = (int)min(p.nS - tj * kTile, (int64_t)kTile);
  uint64_t colok[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) colok[nb] = __builtin_amdgcn_ballot_w64(lcol0 + nb * 16 < crem);
  uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;  // the wave's 128 rows
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
    const float4 th = *reinterpret_cast<const float4*>(thr_tile + lrow0 + mb * 16);
    const float tv[4] = {th.x, th.y, th.z, th.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint64_t m = 0;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) m |= mask_ge(acc[mb][nb][r], tv[r]) & colok[nb];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        if ((m >> (16 * g)) & 0xffffull) {
          const int q = mb * 16 + 4 * g + r;  // row in the wave
          const uint32_t bit = 1u << (q & 31);
          if ((q >> 5) == 0) w0 |= bit;
          else if ((q >> 5) == 1) w1 |= bit;
          else if ((q >> 5) == 2) w2 |= bit;
          else w3 |= bit;
        }
      }
    }
  }
  const uint32_t mine = lane == 0 ? w0 : lane == 1 ? w1 : lane == 2 ? w2 : w3;
  if (lane < 4 && mine)
    atomicOr(p.mark + tj * p.mark_words + ((ti * kTile + wm * kWaveM) >> 5) + lane, mine);
}

// Nearest epilogue (pivot assignment): per row the column of largest P~ =
// a.b - |b|^2/2, i.e. of smallest distance (ties to the smaller column),
// reduced over the 16 lanes that share the row, then folded into the row's
// 64-bit key (order bits of P~, then the complement of the column) with one
// atomic maximum per row and wave.  An approximate answer is fine here: the
// assignment only orders rows, and the pruning it enables is exact anyway.
__device__ inline void epilogue_nearest(const CandParams& p, int64_t ti, int64_t tj, const f32x4 (&acc)[8][4]) {
  const int lane = fresh_lane(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 2, wn = wave & 3;
  const int lrow0 = wm * kWaveM + 4 * (lane >> 4);
  const int lcol0 = wn * kWaveN + (lane & 15);
  const int rrem = (int)min(p.nR - ti * kTile, (int64_t)kTile);
  const int crem = (int)min(p.nS - tj * kTile, (int64_t)kTile);
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float best = -INFINITY;
      uint32_t bc = 0xffffffffu;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const float v = acc[mb][nb][r];
        if (lcol0 + nb * 16 < crem && v > best) {  // a NaN never wins
          best = v;
          bc = (uint32_t)(lcol0 + nb * 16);
        }
      }
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const float ov = __shfl_xor(best, o, 64);
        const uint32_t oc = __shfl_xor(bc, o, 64);
        if (ov > best || (ov == best && oc < bc)) {
          best = ov;
          bc = oc;
        }
      }
      const int lr = lrow0 + mb * 16 + r;
      if ((lane & 15) == 0 && lr < rrem && bc != 0xffffffffu) {
        const unsigned long long key =
            ((unsigned long long)order_key(best) << 32) | (0xffffffffull - (uint64_t)(tj * kTile + bc));
        atomicMax(p.argkey + ti * kTile + lr, key);
      }
    }
  }
}

constexpr int kSelPerLane = 8;  // entries per lane in the k-selection subset
constexpr int kSelBits = 24;    // key bits resolved by the selection

// Largest key prefix (top kSelBits bits) with at least k of the first
// 64 * kT keys at or above it: one bit per step, each step a few compares
// whose masks are counted on the scalar unit.
template <int kT>
__device__ inline uint32_t kth_key(const uint32_t (&key)[kSelPerLane], int k) {
  uint32_t kk = 0;
  for (int b = 31; b >= 32 - kSelBits; --b) {
    const uint32_t cand = kk | (1u << b);
    int c = 0;
#pragma unroll
    for (int t = 0; t < kT; ++t) c += __popcll(mask_ge(key[t], cand));
    if (c >= k) kk = cand;
  }
  return kk;
}

// Tighten one row's band and drop what falls below it (one wave).  The new
// threshold is v - E_i where v is a lower bound of the k-th largest P~ of
// the first 64 * kSelPerLane entries (the k-th largest of a subset is at
// most that of the whole buffer, so the band stays a superset of the exact
// one): the largest key, resolved to its top kSelBits bits, with at least k
// entries at or above it.  Counting uses compare masks, so every step is
// scalar; only the blocks of 64 that hold entries are counted.  n is
// uniform.  Returns the entries kept; the caller re-arms the row's trigger.
// Scalar arguments only (a reference to the kernel's parameter block would
// force the block into scratch memory).
__device__ inline int compact_row(uint2* e, int n, float marg, float* bthr, int k) {
  const int lane = threadIdx.x & 63;
  float thr = *bthr;
  const int m = min(n, 64 * kSelPerLane);
  uint2 v[kSelPerLane];
#pragma unroll
  for (int t = 0; t < kSelPerLane; ++t) {
    const int s = t * 64 + lane;
    v[t] = s < m ? e[s] : make_uint2(0xff800000u, 0);  // -inf sorts below everything kept
  }
  if (m >= k) {
    uint32_t key[kSelPerLane];
#pragma unroll
    for (int t = 0; t < kSelPerLane; ++t) key[t] = (t * 64 + lane) < m ? order_key(__uint_as_float(v[t].x)) : 0u;
    const int tm = (m + 63) >> 6;
    const uint32_t kk = tm <= 2 ? kth_key<2>(key, k) : tm <= 4 ? kth_key<4>(key, k) : kth_key<8>(key, k);
    thr = fmaxf(thr, f32_down((double)key_float(kk) - (double)marg));
  }
  const uint64_t lt = __lanemask_lt(), lbit = 1ull << lane;
  int w = 0;
  // the first entries come from registers; later ones (a buffer larger than
  // the subset) are read block by block before any write can reach them
#pragma unroll
  for (int t = 0; t < kSelPerLane; ++t) {
    if (t * 64 >= m) break;
    const uint64_t mm = mask_ge(__uint_as_float(v[t].x), thr) & lanes_below(m - t * 64);
    if (mm & lbit) e[w + __popcll(mm & lt)] = v[t];
    w += __popcll(mm);
  }
  for (int base = m; base < n; base += 64) {
    const int s = base + lane;
    const uint2 x = s < n ? e[s] : make_uint2(0xff800000u, 0);
    const uint64_t mm = mask_ge(__uint_as_float(x.x), thr) & lanes_below(n - base);
    if (mm & lbit) e[w + __popcll(mm & lt)] = x;
    w += __popcll(mm);
  }
  if (lane == 0) *bthr = thr;
  return w;
}

// Per-workgroup band state in LDS: the threshold, entry count and re-tighten
// trigger of each of the tile's rows, the queue of rows to tighten, and one
// staging queue of hits per wave.
struct BandLds {
  float thr[kTile];
  int cnt[kTile];
  int trig[kTile];
  int list[kTile + 1];
  int urgent;  // a row came within two tiles of the buffer's end
  uint2 q[kThreads / 64][kQueue];  // (P~ bits, row << 8 | column in tile)
};

// Appends a wave's staged hits to their rows' band buffers: one LDS atomic
// per hit for its slot (all 64 lanes at once), then a plain store.  A row
// whose count passes its trigger is queued for tightening.
__device__ inline void flush_band(const CandParams& p, int64_t ti, int64_t tj, int64_t split, BandLds& L,
                                  const uint2* q, int nq) {
  const int lane = threadIdx.x & 63;
  for (int base = 0; base < nq; base += 64) {
    const int s = base + lane;
    if (s < nq) {
      const uint2 h = q[s];
      const int lr = (int)(h.y >> 8);
      const int pos = atomicAdd(&L.cnt[lr], 1);
      if (pos == L.trig[lr]) L.list[1 + atomicAdd(&L.list[0], 1)] = lr;
      if (pos == p.limit) L.urgent = 1;
      if (pos < p.cap) {
        const int64_t i = ti * kTile + lr;
        const uint32_t j = (uint32_t)(tj * kTile) + (h.y & 255u);
        p.band[(i * p.P + split) * (int64_t)p.cap + pos] = make_uint2(h.x, p.jmap ? p.jmap[j] : j);
      }
    }
  }
}

// Band epilogue.  A first test (each row's maximum over the wave's four
// column blocks against its band threshold) finds the row blocks that hold
// an entry; in those, each output is compared with its row's band
// threshold, the 64-lane hit mask of each (row block, row, column block) is
// a single ballot, and only a nonzero mask stages its hits in the wave's LDS
// queue (ballot prefix, no atomics, no waits).  The queue is flushed when
// the next (row block, row) slot might not fit and at the end.  A full tile
// (the common case) carries no bounds or diagonal code; a partial or
// self-diagonal tile checks rows and columns left in the tile in 32-bit tile
// coordinates.  Returns whether this wave wrote to global memory.
template <bool kFull>
__device__ inline bool epilogue_band(const CandParams& p, int64_t ti, int64_t tj, int64_t split,
                                     const f32x4 (&acc)[8][4], BandLds& L) {
  const int lane = fresh_lane(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 2, wn = wave & 3;
  const int lrow0 = wm * kWaveM + 4 * (lane >> 4);
  const int lcol0 = wn * kWaveN + (lane & 15);
  const uint64_t lt = __lanemask_lt(), lbit = lt + 1;
  uint2* q = L.q[wave];
  int nq = 0;
  bool wrote = false;
  // the hit tag (row << 8 | column) is formed from this opaque base: left
  // visible, all 128 tags would be precomputed and kept across the tile loop
  uint32_t tag0 = ((uint32_t)lrow0 << 8) | (uint32_t)lcol0;
  asm volatile("" : "+v"(tag0));
  int rrem = kTile, crem = kTile;
  bool diag = false;
  if constexpr (!kFull) {
    rrem = (int)min(p.nR - ti * kTile, (int64_t)kTile);
    crem = (int)min(p.nS - tj * kTile, (int64_t)kTile);
    diag = p.exclude_self && ti == tj;
  }
  // which row blocks hold an entry: each row's maximum over the wave's four
  // column blocks against its band threshold (NaN passes; bounds are
  // applied below)
  uint32_t hit_mb = 0;
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
    const float4 th = *reinterpret_cast<const float4*>(L.thr + lrow0 + mb * 16);
    const uint64_t h = mask_uge(max4_nan(acc[mb][0][0], acc[mb][1][0], acc[mb][2][0], acc[mb][3][0]), th.x) |
                       mask_uge(max4_nan(acc[mb][0][1], acc[mb][1][1], acc[mb][2][1], acc[mb][3][1]), th.y) |
                       mask_uge(max4_nan(acc[mb][0][2], acc[mb][1][2], acc[mb][2][2], acc[mb][3][2]), th.z) |
                       mask_uge(max4_nan(acc[mb][0][3], acc[mb][1][3], acc[mb][2][3], acc[mb][3][3]), th.w);
    hit_mb |= (h != 0 ? 1u : 0u) << mb;
  }
  if (!hit_mb) return false;
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
    if (!(hit_mb & (1u << mb))) continue;
    const float4 th = *reinterpret_cast<const float4*>(L.thr + lrow0 + mb * 16);
    const float tv[4] = {th.x, th.y, th.z, th.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint64_t m[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        m[nb] = mask_ge(acc[mb][nb][r], tv[r]);
        if constexpr (!kFull) {
          const int lr = lrow0 + mb * 16 + r, lc = lcol0 + nb * 16;
          m[nb] &= __builtin_amdgcn_ballot_w64(lr < rrem && lc < crem && !(diag && lr == lc));
        }
      }
      if (!(m[0] | m[1] | m[2] | m[3])) continue;
      // one capacity check per slot keeps the flush code at 32 sites
      if (nq + __popcll(m[0]) + __popcll(m[1]) + __popcll(m[2]) + __popcll(m[3]) > kQueue) {
        flush_band(p, ti, tj, split, L, q, nq);
        nq = 0;
        wrote = true;
      }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        if (m[nb]) {
          if (m[nb] & lbit)
            q[nq + __popcll(m[nb] & lt)] =
                make_uint2(__float_as_uint(acc[mb][nb][r]), tag0 + (uint32_t)(((mb * 16 + r) << 8) + nb * 16));
          nq += __popcll(m[nb]);
        }
      }
    }
  }
  if (nq) {
    flush_band(p, ti, tj, split, L, q, nq);
    wrote = true;
  }
  return wrote;
}

// The band epilogue of a workgroup's first tile when the tile is full: every
// row's threshold is still -inf, so every output is a hit, and each row's
// buffer takes the tile's 256 outputs in column order straight from the
// registers (no staging, no atomics).  Then each row holds 256 entries and
// is queued if that passed its trigger.  (A NaN output, possible only when
// the inputs overflow, becomes an entry too; no threshold test keeps it
// and the selection sorts it above every number, which can only lower the
// threshold it finds.)
__device__ inline void flood_band(const CandParams& p, int64_t ti, int64_t tj, int64_t split,
                                  const f32x4 (&acc)[8][4], BandLds& L) {
  const int lane = fresh_lane(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 2, wn = wave & 3;
  const int lrow0 = wm * kWaveM + 4 * (lane >> 4);
  const int lcol0 = wn * kWaveN + (lane & 15);
  const int64_t rstride = (int64_t)p.P * p.cap;  // entries from one row's buffer to the next's
  uint2* const e0 = p.band + (ti * kTile * p.P + split) * (int64_t)p.cap + lrow0 * rstride + lcol0;
  const uint32_t j0 = (uint32_t)(tj * kTile) + (uint32_t)lcol0;
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint2* const e = e0 + (mb * 16 + r) * rstride;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) e[nb * 16] = make_uint2(__float_as_uint(acc[mb][nb][r]), j0 + nb * 16);
    }
  }
  for (int r = threadIdx.x; r < kTile; r += kThreads) {
    L.cnt[r] = kTile;
    if (L.trig[r] < kTile) L.list[1 + atomicAdd(&L.list[0], 1)] = r;
    if (p.limit < kTile) L.urgent = 1;
  }
}

// Rows queued by the band epilogue are tightened by one wave each and their
// triggers re-armed retight entries further on (capped at limit).  A round
// waits until batch rows are queued, unless some row has reached limit
// entries.  The host sets limit = cap - 256 when every queued row is
// tightened at once (batch 1), else cap - 512: a tile adds at most 256
// entries to a row, so every row still has room for one more tile when the
// round runs.  Called
// by the whole workgroup right after a barrier, so list[0] and urgent are
// uniform, and only at the first K-chunk of a tile, where the accumulators
// are dead; at the end of the workgroup's tiles every queued row is
// tightened (drain).
// Returns whether any row was tightened (then the workgroup wrote to global
// memory).
__device__ inline bool tighten_rows(const CandParams& p, int64_t ti, int64_t split, BandLds& L, bool drain) {
  // LDS values that are the same in every lane are read into scalars, so
  // that the loops below are uniform
  const int nq = __builtin_amdgcn_readfirstlane(L.list[0]);
  if (nq == 0 || (!drain && nq < p.batch && !__builtin_amdgcn_readfirstlane(L.urgent))) return false;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int limit = p.limit;
  // Every row's band threshold first rises to the best one any split of the
  // row has published (or a seed, see the E4M3 pilot on the host): each is
  // v - E_i with v a lower bound of the k-th largest P~ over a subset of S,
  // so at most the k-th largest over all of S minus E_i (the band stays a
  // superset of the exact one).
  for (int r = threadIdx.x; r < kTile; r += kThreads) {
    const int64_t i = ti * kTile + r;
    if (i < p.nR) {
      const uint32_t g = __hip_atomic_load(p.gkey + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      L.thr[r] = fmaxf(L.thr[r], key_float(g));
    }
  }
  __syncthreads();
  for (int t = wave; t < nq; t += kThreads / 64) {
    const int lr = __builtin_amdgcn_readfirstlane(L.list[1 + t]);
    const int64_t i = ti * kTile + lr;
    const int n = __builtin_amdgcn_readfirstlane(min(L.cnt[lr], p.cap));
    const int w = compact_row(p.band + ((i * p.P) + split) * (int64_t)p.cap, n, p.marg[i], &L.thr[lr], p.k);
    if (lane == 0) {
      L.cnt[lr] = w;
      L.trig[lr] = min(w + p.retight, limit);
      if (w > limit) atomicOr(p.overflow, 1);
      atomicMax(p.gkey + i, order_key(L.thr[lr]));  // publish to the row's other splits
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    L.list[0] = 0;
    L.urgent = 0;
  }
  __syncthreads();
  return true;
}

// ------------------------------------------------------------------ kernel
// Waits until at most n vector-memory operations of this wave are
// outstanding and all of its LDS operations are done, then joins the
// workgroup's barrier.  n is 0 or a multiple of a step's transfers; the
// s_waitcnt immediate packs vmcnt in bits 3:0 and 15:14 (expcnt 6:4 left at
// its no-wait value 7, lgkmcnt 11:8 = 0).
__device__ inline void wait_and_sync(int n) {
  n = __builtin_amdgcn_readfirstlane(n);  // block-uniform: scalar branches
  asm volatile("" ::: "memory");
  if (n >= 8) __builtin_amdgcn_s_waitcnt(0x0078);
  else if (n >= 4) __builtin_amdgcn_s_waitcnt(0x0074);
  else __builtin_amdgcn_s_waitcnt(0x0070);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// kMasked (eps and band modes): the K-step masks p.kmaskA / p.kmaskB are
// set; a separate instantiation, so that the unmasked pass carries none of
// their bookkeeping.
template <int kPrec, int kMode, bool kMasked = false>
__global__ __launch_bounds__(kThreads, 1) void cand_kernel(CandParams p) {
  static_assert(!kMasked || kMode == kModeEps || kMode == kModeBand, "K-step masks in eps and band modes only");
  using Q = Pipe<kPrec>;
  static_assert(Q::kStages == 2 || Q::kStages == 4, "ring depth");
  // operand transfers per issuing wave per step (the count a wait leaves in
  // flight per later step)
  constexpr int kPerStep = 2 * dma_per_op<kMode>(Q::kRowsPerDma);
  static_assert((Q::kStages - 2) * kPerStep <= 8, "wait_and_sync covers two later steps at most");
  // kEps: the eps-like modes (eps and mark), one tile per pass with per-row
  // thresholds; kQueue_: candidates staged in LDS (eps only)
  constexpr bool kFp8 = kPrec == DL_FP8, kEps = kMode != kModeBand, kMark = kMode == kModeMark;
  constexpr bool kQ = kMode == kModeEps;
  // the ring: kStages x (A step, B step)
  __shared__ __attribute__((aligned(1024))) uint8_t lds_ab[Q::kStages][2][Q::kStageBytes];
  // per-tile side data, three tiles deep (the loader runs at most two tiles
  // ahead of the tile being computed)
  __shared__ __attribute__((aligned(16))) float side_hb[3][kTile];
  __shared__ __attribute__((aligned(16))) float side_thr[kEps ? 3 : 1][kEps ? kTile : 4];
  __shared__ __attribute__((aligned(16))) int side_sa[kFp8 ? 3 : 1][kFp8 ? kTile : 4];
  __shared__ __attribute__((aligned(16))) int side_sb[kFp8 ? 3 : 1][kFp8 ? kTile : 4];
  __shared__ __attribute__((aligned(16))) uint8_t lds_band_raw[kEps ? 16 : sizeof(BandLds)];
  BandLds& band = *reinterpret_cast<BandLds*>(lds_band_raw);
  __shared__ __attribute__((aligned(16))) uint2 lds_eq[kQ ? kThreads / 64 : 1][kQ ? kQueue : 1];
  // eps, except E4M3 (LDS budget): the staged candidates' P~
  constexpr bool kStageP = kQ && !kFp8;
  __shared__ uint32_t lds_eqp[kStageP ? kThreads / 64 : 1][kStageP ? kQueue : 1];

  // invalid input (non-finite values, norms out of range): no work at all
  if (p.gate && __builtin_amdgcn_readfirstlane(*p.gate)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 2, wn = wave & 3;
  const int nsteps = (int)(p.qld / Q::kCB);

  // The loader walks the tile sequence one K-step ahead of the matrix
  // cores; the compute side takes its tiles from the loader: the step issued
  // during a tile's last K-step is the next tile's first (one tile_of per
  // tile instead of two).
  static_assert(Q::kStages == 2, "the compute side follows the loader one step behind");
  TileIter lit;
  int64_t ti, tj;
  if (!lit.next(p, kMode, ti, tj)) return;
  // K-step masks (eps and band modes): the loader issues a tile's set steps in
  // order, and the compute side runs as many steps as the loader issued
  constexpr bool masked = kMasked;
  int64_t lti = ti, ltj = tj;  // tile of the loader's next step
  int64_t iti = ti, itj = tj;  // tile of the step issued last
  uint64_t lrem = masked ? tile_steps(p, ti, tj) : 0;  // the loader tile's steps not yet issued
  int lsteps = masked ? __builtin_popcountll(lrem) : nsteps;
  int isteps = lsteps;  // steps of the tile of the step issued last
  int lstep = 0, ltile = 0, issued = 0;
  bool lmore = true;
  auto issue = [&]() {
    if (lstep == 0) {
      const int sb = ltile % 3;
      issue_side<kPrec, kMode>(p, lti, ltj, SideRefs{side_hb[sb], side_thr[kEps ? sb : 0], side_sa[kFp8 ? sb : 0],
                                                      side_sb[kFp8 ? sb : 0]});
    }
    const int st = issued % Q::kStages;
    const int k = masked ? (int)__builtin_ctzll(lrem) : lstep;
    issue_loads<kPrec, kMode>(p, lti, ltj, k, lds_ab[st][0], lds_ab[st][1]);
    iti = lti;
    itj = ltj;
    isteps = lsteps;
    ++issued;
    if (masked) lrem &= lrem - 1;
    if (++lstep == lsteps) {
      lstep = 0;
      ++ltile;
      lmore = lit.next(p, kMode, lti, ltj);
      if (masked && lmore) {
        lrem = tile_steps(p, lti, ltj);
        lsteps = __builtin_popcountll(lrem);
      }
    }
  };

  int64_t split = 0;
  if constexpr (!kEps) {
    split = uniform64(lit.split);
    for (int r = threadIdx.x; r < kTile; r += kThreads) {
      // -inf, or a row's seeded threshold (p.flood == 0)
      band.thr[r] = (!p.flood && ti * kTile + r < p.nR) ? key_float(p.gkey[ti * kTile + r]) : -INFINITY;
      band.cnt[r] = 0;
      band.trig[r] = p.retight;
    }
    if (threadIdx.x == 0) {
      band.list[0] = 0;
      band.urgent = 0;
    }
  }
  for (int s = 0; s < Q::kStages - 1 && lmore; ++s) issue();

  int step = 0, ctile = 0;
  int eq = 0;  // eps: candidates staged in this wave's queue
  bool dirty = true;  // the band set-up above wrote LDS only, but be exact once
  bool full = true;   // band mode: the tile needs no bounds or self checks
  f32x4 acc[8][4];
  Frags fr;
  int sa[8], sb[4];
  // Each K-step starts with a wait: its operands are in LDS once this wave's
  // transfers for it have landed and every wave has passed the barrier;
  // transfers of later steps may stay in flight, unless this wave also wrote
  // to global memory since the last full wait (stores and loads may then
  // retire out of order).  The barrier also means every wave is done with
  // the stage computed in the previous step, so this step's new transfers
  // may overwrite it.
  if constexpr (kEps) {
    // eps mode: one tile per pass; each K-step's last products are issued
    // after the next barrier (mma_step, kTailIn).  A tile's candidate
    // epilogue runs after the barrier that opens the next tile, between that
    // step's first fragment reads and its first matrix instruction: a wave
    // that stages hits then works while the other wave of its SIMD issues
    // matrix instructions, instead of holding every wave at the barrier.
    // (Not for E4M3, whose step has no registers to spare for it.)
    constexpr bool kDefer = kQ && !kFp8;
    int tsteps = isteps;  // K-steps of the current tile (the prologue issued its first step)
    bool pend = false;    // eps: a finished tile (pti, ptj) awaits its epilogue
    int64_t pti = 0, ptj = 0;
    int psbuf = 0;
    for (;;) {  // one tile per pass
      // ---- the tile's first K-step
      wait_and_sync(dirty ? 0 : (issued - step - 1) * kPerStep);
      dirty = false;
      const int sbuf = ctile % 3;
      bool more = lmore;  // a step follows the current one
      {
        const int l16 = fresh_lane() & 15;
        const int cb = wn * kWaveN + l16, rb = wm * kWaveM + l16;
        f32x4 init[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const float h0 = -side_hb[sbuf][cb + nb * 16];
          init[nb] = f32x4{h0, h0, h0, h0};
          if constexpr (kFp8) sb[nb] = side_sb[sbuf][cb + nb * 16] + 127;
        }
        if constexpr (kFp8) {
#pragma unroll
          for (int mb = 0; mb < 8; ++mb) sa[mb] = side_sa[sbuf][rb + mb * 16] + 127;
        }
        if (lmore) issue();
        const int st = step % Q::kStages;
        if constexpr (kDefer) {
          mma_first_reads<kPrec>(lds_ab[st][0], lds_ab[st][1], wm * kWaveM, wn * kWaveN, fr);
          // side_thr[psbuf] is intact: the loader is one step ahead, so it
          // fills at most the next tile's side buffer
          if (pend)
            dirty |= epilogue_eps<kStageP>(p, pti, ptj, acc, side_thr[psbuf], lds_eq[wave],
                                           lds_eqp[kStageP ? wave : 0], eq);
          __builtin_amdgcn_sched_barrier(0);
          mma_step<kPrec, true, false, true>(acc, lds_ab[st][0], lds_ab[st][1], wm * kWaveM, wn * kWaveN, sa, sb,
                                             init, fr);
        } else {
          mma_step<kPrec, true, false>(acc, lds_ab[st][0], lds_ab[st][1], wm * kWaveM, wn * kWaveN, sa, sb, init,
                                       fr);
        }
      }
      ++step;
      // ---- its other K-steps
      for (int c = 1; c < (masked ? tsteps : nsteps); ++c) {
        wait_and_sync(dirty ? 0 : (issued - step - 1) * kPerStep);
        dirty = false;
        more = lmore;
        if (lmore) issue();
        const int st = step % Q::kStages;
        mma_step<kPrec, false, true>(acc, lds_ab[st][0], lds_ab[st][1], wm * kWaveM, wn * kWaveN, sa, sb, acc[0], fr);
        ++step;
      }
      mma_tail<kPrec>(acc, fr);
      // ---- epilogue
      if constexpr (kMark) {
        epilogue_mark(p, ti, tj, acc, side_thr[sbuf]);
        dirty = true;  // atomics to global memory
      } else if constexpr (kMode == kModeNearest) {
        epilogue_nearest(p, ti, tj, acc);
        dirty = true;
      } else if constexpr (kDefer) {
        pend = true;  // after the next tile's first barrier, or below
        pti = ti;
        ptj = tj;
        psbuf = sbuf;
      } else {
        dirty |= epilogue_eps<kStageP>(p, ti, tj, acc, side_thr[sbuf], lds_eq[wave], lds_eqp[kStageP ? wave : 0], eq);
      }
      if (!more) break;
      ti = iti;  // the step just issued opens the next tile
      tj = itj;
      tsteps = isteps;
      ++ctile;
    }
    if constexpr (kDefer) {
      if (pend)
        dirty |= epilogue_eps<kStageP>(p, pti, ptj, acc, side_thr[psbuf], lds_eq[wave], lds_eqp[kStageP ? wave : 0],
                                       eq);
    }
  } else {
    // band mode (more live state beside the accumulators): each K-step's
    // products are all issued before the next barrier
    int chunk = 0;
    int tsteps = isteps;  // K-steps of the current tile (the prologue issued its first step)
    for (;;) {
      wait_and_sync(dirty ? 0 : (issued - step - 1) * kPerStep);
      dirty = false;
      const int sbuf = ctile % 3;
      const bool more = lmore;  // a step follows this one
      if (chunk == 0) {
        dirty |= tighten_rows(p, ti, split, band, false);
        full = (ti + 1) * kTile <= p.nR && (tj + 1) * kTile <= p.nS && !(p.exclude_self && ti == tj);
        const int l16 = fresh_lane() & 15;
        const int cb = wn * kWaveN + l16, rb = wm * kWaveM + l16;
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          // the initial values are copied into the accumulators (measured:
          // reading C from them on the first step spills in band mode)
          const float h0 = -side_hb[sbuf][cb + nb * 16];
#pragma unroll
          for (int mb = 0; mb < 8; ++mb) acc[mb][nb] = f32x4{h0, h0, h0, h0};
          if constexpr (kFp8) sb[nb] = side_sb[sbuf][cb + nb * 16] + 127;
        }
        if constexpr (kFp8) {
#pragma unroll
          for (int mb = 0; mb < 8; ++mb) sa[mb] = side_sa[sbuf][rb + mb * 16] + 127;
        }
      }
      if (lmore) issue();
      const int st = step % Q::kStages;
      mma_step<kPrec, false, false>(acc, lds_ab[st][0], lds_ab[st][1], wm * kWaveM, wn * kWaveN, sa, sb, acc[0], fr);
      mma_tail<kPrec>(acc, fr);
      if (chunk == (masked ? tsteps : nsteps) - 1) {
        if (full && ctile == 0 && p.flood) {
          // the first tile: no round has run, every threshold is -inf
          flood_band(p, ti, tj, split, acc, band);
          dirty = true;
        } else if (full) dirty |= epilogue_band<true>(p, ti, tj, split, acc, band);
        else dirty |= epilogue_band<false>(p, ti, tj, split, acc, band);
      }
      ++step;
      if (++chunk == (masked ? tsteps : nsteps)) {
        if (!more) break;
        chunk = 0;
        ti = iti;  // the step just issued opens the next tile
        tj = itj;
        tsteps = isteps;
        ++ctile;
      }
    }
  }
  if constexpr (kQ) {
    if (eq) flush_eps<kStageP>(p, lds_eq[wave], lds_eqp[kStageP ? wave : 0], eq);
  } else if constexpr (!kEps) {
    __syncthreads();
    tighten_rows(p, ti, split, band, true);
    for (int r = threadIdx.x; r < kTile; r += kThreads) {
      const int64_t i = ti * kTile + r;
      if (i < p.nR) p.bcount[i * p.P + split] = min(band.cnt[r], p.cap);
    }
  }
}

template <int kMode>
static hipError_t launch_mode(dl_prec prec, const CandParams& p, dim3 grid, hipStream_t st) {
  if constexpr (kMode == kModeEps || kMode == kModeBand) {
    if (p.kmaskA) {
      switch (prec) {
        case DL_FP32: hipLaunchKernelGGL((cand_kernel<DL_FP32, kMode, true>), grid, dim3(kThreads), 0, st, p); break;
        case DL_BF16: hipLaunchKernelGGL((cand_kernel<DL_BF16, kMode, true>), grid, dim3(kThreads), 0, st, p); break;
        case DL_FP16: hipLaunchKernelGGL((cand_kernel<DL_FP16, kMode, true>), grid, dim3(kThreads), 0, st, p); break;
        case DL_FP8: hipLaunchKernelGGL((cand_kernel<DL_FP8, kMode, true>), grid, dim3(kThreads), 0, st, p); break;
      }
      return hipGetLastError();
    }
  }
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

int cand_group_rows(int64_t qld, int64_t nTR) { return group_rows(qld, nTR); }

// Multiplier and shifts for udiv32 by d >= 1 (Granlund and Montgomery):
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, s1 = min(l, 1),
// s2 = max(l - 1, 0); exact for every 32-bit dividend.
static void div_magic(uint32_t d, uint32_t& m, uint32_t& s1, uint32_t& s2) {
  uint32_t l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  m = (uint32_t)(((((1ull << l) - d) << 32) / d) + 1);
  s1 = l < 1 ? l : 1;
  s2 = l > 1 ? l - 1 : 0;
}

// eps mode over a device tile list (p.tiles, *p.ntiles entries): persistent
// workgroups, one per CU, walk the list; mark = the bound pass (every tile).
static hipError_t launch_eps_like(dl_prec prec, CandParams p, hipStream_t st, int cu_count, int mode);

// The eps pass over the tile list p.tiles (length *p.ntiles, on the device),
// or over the full grid when p.list_all is set and 2 * *p.ntiles >= it; the
// grid's set-up is made either way, the kernel picks.
hipError_t launch_cand_list(dl_prec prec, CandParams p, hipStream_t st, int cu_count) {
  if (!p.tiles) return hipSuccess;
  return launch_eps_like(prec, p, st, cu_count, kModeEps);
}

hipError_t launch_cand_mark(dl_prec prec, CandParams p, hipStream_t st, int cu_count) {
  p.tiles = nullptr;
  return launch_eps_like(prec, p, st, cu_count, kModeMark);
}

hipError_t launch_cand_nearest(dl_prec prec, CandParams p, hipStream_t st, int cu_count) {
  p.tiles = nullptr;
  p.self_join = 0;
  return launch_eps_like(prec, p, st, cu_count, kModeNearest);
}

hipError_t launch_cand_eps(dl_prec prec, CandParams p, hipStream_t st, int cu_count) {
  p.tiles = nullptr;
  return launch_eps_like(prec, p, st, cu_count, kModeEps);
}

static hipError_t launch_eps_like(dl_prec prec, CandParams p, hipStream_t st, int cu_count, int mode) {
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
  // logical indices, offsets and group sizes all below 2^32 - 2^24 (room for
  // the rounds past the end): 32-bit tile-order arithmetic
  p.small32 = p.nlogical + 8 * (int64_t)cu_count < (1ll << 32) - (1ll << 24) &&
              (int64_t)p.GM * (p.self_join ? p.nTR : p.nTS) < (1ll << 31);
  if (p.small32) {
    div_magic((uint32_t)(p.GM * p.nTS), p.dv_grp_m, p.dv_grp_s1, p.dv_grp_s2);
    div_magic((uint32_t)p.GM, p.dv_gm_m, p.dv_gm_s1, p.dv_gm_s2);
    div_magic((uint32_t)(p.nTR - (p.ngroups - 1) * p.GM), p.dv_gl_m, p.dv_gl_s1, p.dv_gl_s2);
  }
  int64_t G = cu_count;  // one 512-thread workgroup per CU
  const int64_t need = (p.nlogical + 7) / 8 * 8;
  if (G > need) G = need;
  G = (G + 7) / 8 * 8;
  if (mode == kModeMark) return launch_mode<kModeMark>(prec, p, dim3((unsigned)G), st);
  if (mode == kModeNearest) return launch_mode<kModeNearest>(prec, p, dim3((unsigned)G), st);
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
