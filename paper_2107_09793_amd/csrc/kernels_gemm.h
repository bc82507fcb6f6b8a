// Complex GEMM steps on the matrix cores (MFMA), with operands read in
// place through their bit strides (no separate transpose pass).
//
// Complex arithmetic as one real GEMM: with A row-major and complex
// interleaved, A is a real M x 2K matrix; B becomes the real 2K x 2N matrix
//   [[ Br, Bi], [-Bi, Br]]  per complex entry,
// so the real product is C in interleaved form.  On the FP32 matrix path one
// v_mfma_f32_32x32x2f32 covers one complex k for a 32 x 16 complex block:
// lanes 0-31 carry Re A / the first row of the 2x2 block of B, lanes 32-63
// Im A / the second row.
//
// Split-BF16 path: every float x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
// (round to nearest even); a product is hi*hi + hi*lo + lo*hi with float32
// accumulation (the lo*lo term, ~2^-16 relative, is dropped).  One
// v_mfma_f32_32x32x16_bf16 covers 8 complex k for a 32 x 16 complex block.
//
// Tiles: a workgroup of 256 threads (2 x 2 or 4 x 1 waves) owns an MT x NT
// complex output tile and walks k in tiles of KT through double-buffered
// LDS.  At start the workgroup tabulates in LDS the in-tile offsets of rows,
// columns and k of every operand (one bit scatter per entry); afterwards all
// addressing is table lookups and adds.  A tile's elements are enumerated in
// (approximately) increasing stride order so consecutive lanes touch
// consecutive addresses whenever the layout allows.  Workgroup ids are
// remapped so that the tiles one XCD (one L2) runs share their A rows.
#pragma once

#include "kernels_common.h"

namespace tnk {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

struct GemmArgs {
  StepArgs s;
  // Enumeration of a tile's elements: bit j of the element index is a row
  // (A) / column (B) bit if bit j of the mask is set, else a k bit; bits of
  // one class keep their class order.
  uint32_t a_mask, b_mask;
  int32_t xcd_remap;
  // logical tile of workgroup 0: steps with more tiles than one dispatch can
  // hold (2^32 work-items) run as several launches over consecutive ranges
  uint64_t tile0;
  // split k (few output tiles, long sums): 2^kc_log2 chunks of the k tiles,
  // chunk c of every output tile is logical tile c * ntiles + tile and writes
  // its partial result at C + c * part_stride (the reduce adds them up)
  int32_t kc_log2;
  int64_t part_stride;
};

template <int V>
struct ilog2 {
  static constexpr int value = 1 + ilog2<V / 2>::value;
};
template <>
struct ilog2<1> {
  static constexpr int value = 0;
};

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint32_t pack2(uint16_t lo16, uint16_t hi16) {
  return (uint32_t)lo16 | ((uint32_t)hi16 << 16);
}

// Split element index e into (class-1 index, class-2 index) by mask.
__device__ __forceinline__ void split_bits(int e, uint32_t mask, int nbits, int& i1, int& i2) {
  int c1 = 0, c2 = 0;
  i1 = 0;
  i2 = 0;
  for (int j = 0; j < nbits; ++j) {
    int bit = (e >> j) & 1;
    if ((mask >> j) & 1u) { i1 |= bit << c1; ++c1; } else { i2 |= bit << c2; ++c2; }
  }
}

// Per-workgroup LDS copy of the step's bit strides (read once from the kernel
// arguments, then indexed freely) and the tile offset tables.
struct Strides {
  int8_t v[9 * kMaxBits];   // same order as in StepArgs
  __device__ __forceinline__ const int8_t* Ab() const { return v; }
  __device__ __forceinline__ const int8_t* Bb() const { return v + kMaxBits; }
  __device__ __forceinline__ const int8_t* Cb() const { return v + 2 * kMaxBits; }
  __device__ __forceinline__ const int8_t* Am() const { return v + 3 * kMaxBits; }
  __device__ __forceinline__ const int8_t* Cm() const { return v + 4 * kMaxBits; }
  __device__ __forceinline__ const int8_t* Bn() const { return v + 5 * kMaxBits; }
  __device__ __forceinline__ const int8_t* Cn() const { return v + 6 * kMaxBits; }
  __device__ __forceinline__ const int8_t* Ak() const { return v + 7 * kMaxBits; }
  __device__ __forceinline__ const int8_t* Bk() const { return v + 8 * kMaxBits; }
};
static_assert(offsetof(StepArgs, sA_b) % 4 == 0, "stride arrays word aligned");

__device__ __forceinline__ void load_strides(const StepArgs& p, Strides& s) {
  const int32_t* src = reinterpret_cast<const int32_t*>(p.sA_b);
  int32_t* dst = reinterpret_cast<int32_t*>(s.v);
  for (int i = threadIdx.x; i < 9 * kMaxBits / 4; i += 256) dst[i] = src[i];
}

template <int MT, int NT, int KT>
struct GemmTables {
  int64_t am[MT], ak[KT], bk[KT], bn[NT], cm[MT], cn[NT];
};

template <int MT, int NT, int KT>
__device__ __forceinline__ void build_tables(const StepArgs& p, const Strides& S,
                                             GemmTables<MT, NT, KT>& t) {
  constexpr int LM = ilog2<MT>::value, LN = ilog2<NT>::value, LK = ilog2<KT>::value;
  const int tid = threadIdx.x;
  const int nmv = p.nm < LM ? p.nm : LM, nnv = p.nn < LN ? p.nn : LN, nkv = p.nk < LK ? p.nk : LK;
  for (int i = tid; i < MT; i += 256) {
    t.am[i] = scatter(i, S.Am(), nmv);
    t.cm[i] = scatter(i, S.Cm(), nmv);
  }
  for (int i = tid; i < NT; i += 256) {
    t.bn[i] = scatter(i, S.Bn(), nnv);
    t.cn[i] = scatter(i, S.Cn(), nnv);
  }
  for (int i = tid; i < KT; i += 256) {
    t.ak[i] = scatter(i, S.Ak(), nkv);
    t.bk[i] = scatter(i, S.Bk(), nkv);
  }
}

// Coordinates (batch, row tile, column tile) of logical tile t; with the
// remap, tile t runs on XCD t % 8 and each XCD walks a contiguous range of
// tiles (column tiles fastest), so the tiles resident on one L2 share rows of A.
__device__ __forceinline__ void tile_coords(const StepArgs& p, int LM, int LN, uint64_t t,
                                            uint64_t ntiles, int remap, uint64_t& bidx,
                                            uint64_t& mt, uint64_t& nt) {
  if (remap) t = (t & 7) * (ntiles >> 3) + (t >> 3);
  int lnt = p.nn > LN ? p.nn - LN : 0;
  int lmt = p.nm > LM ? p.nm - LM : 0;
  nt = t & ((1ull << lnt) - 1);
  mt = (t >> lnt) & ((1ull << lmt) - 1);
  bidx = t >> (lnt + lmt);
}

// Everything both GEMM kernels share: tables, tile bases, per-thread element
// offsets (independent of the tile), the Gray-code walk over k tiles, and the
// epilogue.  One workgroup per output tile.
template <int MT, int NT, int KT, class OffT>
struct GemmCommon {
  static constexpr int LM = ilog2<MT>::value, LN = ilog2<NT>::value, LK = ilog2<KT>::value;
  static constexpr int AE = MT * KT / 256, BE = NT * KT / 256;
  int64_t baseA, baseB, baseC, kA, kB;
  uint64_t gray, nkt, ntiles, tile;
  int kc_log2;
  int64_t part_stride, cpart;
  OffT a_go[AE], b_go[BE];   // in-tile offsets (32-bit when they fit)
  int a_mk[AE], b_nk[BE];    // packed LDS coordinates: row/col | k << 16
  uint32_t a_ok, b_ok;
  int remap;

  __device__ __forceinline__ void init(const GemmArgs& g, const GemmTables<MT, NT, KT>& t) {
    const StepArgs& p = g.s;
    const int tid = threadIdx.x;
    const int mlim = 1 << (p.nm < LM ? p.nm : LM), nlim = 1 << (p.nn < LN ? p.nn : LN);
    const int klim = 1 << (p.nk < LK ? p.nk : LK);
    a_ok = 0;
    b_ok = 0;
#pragma unroll
    for (int r = 0; r < AE; ++r) {
      int mi, ki;
      split_bits(tid + 256 * r, g.a_mask, LM + LK, mi, ki);
      a_mk[r] = mi | (ki << 16);
      a_go[r] = (OffT)(t.am[mi] + t.ak[ki]);
      if (mi < mlim && ki < klim) a_ok |= 1u << r;
    }
#pragma unroll
    for (int r = 0; r < BE; ++r) {
      int ni, ki;
      split_bits(tid + 256 * r, g.b_mask, LN + LK, ni, ki);
      b_nk[r] = ni | (ki << 16);
      b_go[r] = (OffT)(t.bn[ni] + t.bk[ki]);
      if (ni < nlim && ki < klim) b_ok |= 1u << r;
    }
    kc_log2 = g.kc_log2;
    part_stride = g.part_stride;
    nkt = 1ull << ((p.nk > LK ? p.nk - LK : 0) - kc_log2);   // k tiles per chunk
    int lnt = p.nn > LN ? p.nn - LN : 0;
    int lmt = p.nm > LM ? p.nm - LM : 0;
    ntiles = 1ull << (p.nb + lmt + lnt);
    remap = g.xcd_remap;
    tile = g.tile0 + blockIdx.x;
  }

  __device__ __forceinline__ void set_tile(const StepArgs& p, const Strides& S, uint64_t t) {
    uint64_t bidx, mt, nt;
    const uint64_t chunk = t / ntiles;   // split k: the chunk is the slowest index
    t -= chunk * ntiles;
    tile_coords(p, LM, LN, t, ntiles, remap, bidx, mt, nt);
    baseA = scatter_range(mt << LM, S.Am(), LM, p.nm) + scatter(bidx, S.Ab(), p.nb);
    baseB = scatter_range(nt << LN, S.Bn(), LN, p.nn) + scatter(bidx, S.Bb(), p.nb);
    baseC = scatter_range(mt << LM, S.Cm(), LM, p.nm) + scatter_range(nt << LN, S.Cn(), LN, p.nn) +
            scatter(bidx, S.Cb(), p.nb) + (int64_t)chunk * part_stride;
    // the chunk's k tiles share their high k bits; the walk below covers the
    // low ones in Gray order from this base
    const int lk_lo = LK + (p.nk > LK ? p.nk - LK : 0) - kc_log2;
    kA = scatter_range(chunk << lk_lo, S.Ak(), lk_lo, p.nk);
    kB = scatter_range(chunk << lk_lo, S.Bk(), lk_lo, p.nk);
    gray = 0;
  }

  __device__ __forceinline__ void advance(const Strides& S, uint64_t kt) {
    int j = __builtin_ctzll(kt);
    uint64_t bit = 1ull << j;
    int64_t da = (int64_t)1 << S.Ak()[LK + j], db = (int64_t)1 << S.Bk()[LK + j];
    if (gray & bit) { kA -= da; kB -= db; } else { kA += da; kB += db; }
    gray ^= bit;
  }

  __device__ __forceinline__ void gload(const StepArgs& p, float2* ra, float2* rb) {
#pragma unroll
    for (int r = 0; r < AE; ++r)
      ra[r] = (a_ok >> r) & 1u ? p.A[baseA + kA + a_go[r]] : make_float2(0.f, 0.f);
#pragma unroll
    for (int r = 0; r < BE; ++r)
      rb[r] = (b_ok >> r) & 1u ? p.B[baseB + kB + b_go[r]] : make_float2(0.f, 0.f);
  }

  // lane holds real column (lane & 31) of each 32x32 block, rows
  // 8*(r/4) + 4*(lane/32) + r%4 for accumulator r
  template <int WVN, int WM, int WN>
  __device__ __forceinline__ void epilogue(const StepArgs& p, const GemmTables<MT, NT, KT>& t,
                                           int64_t cbase, floatx16 (&acc)[WM][WN]) const {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wave_m = wave / WVN, wave_n = wave % WVN;
    const int half = lane >> 5, par = lane & 1;
    const int mlim = 1 << (p.nm < LM ? p.nm : LM), nlim = 1 << (p.nn < LN ? p.nn : LN);
    float* C = reinterpret_cast<float*>(p.C + cbase);
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      int col = wave_n * WN * 16 + j * 16 + ((lane & 31) >> 1);
      if (col >= nlim) continue;
      int64_t offn = t.cn[col];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          int row = wave_m * WM * 32 + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          if (row >= mlim) continue;
          float* cf = C + 2 * (offn + t.cm[row]) + par;
          float v = acc[i][j][r];
          if (p.accumulate) v += *cf;
          *cf = v;
        }
      }
    }
  }
};

// One output tile per workgroup, shared by both precisions.  The tile's first
// MFMA takes a zero accumulator (Ops::compute<true>).  Ops supplies the LDS
// staging (lstore), the MFMA block of one k tile (compute), the number of
// accumulator blocks per 32-row block (kAcc) and the epilogue.  (A persistent
// loop over tiles keeps the epilogue's offsets live across tiles and costs an
// occupancy step, so each workgroup runs one tile.)
template <int WVN, int WM, int WN, int MT, int NT, int KT, class OffT, class Ops>
__device__ __forceinline__ void gemm_tiles(const StepArgs& p, const Strides& S,
                                           GemmCommon<MT, NT, KT, OffT>& c,
                                           const GemmTables<MT, NT, KT>& tab, Ops& ops) {
  using GC = GemmCommon<MT, NT, KT, OffT>;
  const uint64_t tile = c.tile;
  if (tile >= c.ntiles << c.kc_log2) return;
  float2 ra[GC::AE], rb[GC::BE];
  floatx16 acc[WM][Ops::kAcc];
  c.set_tile(p, S, tile);
  c.gload(p, ra, rb);
  ops.lstore(0, ra, rb);
  __syncthreads();
  // k tile 0 (defines acc), then the double-buffered rest
  if (c.nkt > 1) {
    c.advance(S, 1);
    c.gload(p, ra, rb);
  }
  ops.template compute<true>(0, acc);
  if (c.nkt > 1) ops.lstore(1, ra, rb);
  __syncthreads();
  for (uint64_t kt = 1; kt < c.nkt; ++kt) {
    const int buf = kt & 1;
    const bool last = kt + 1 == c.nkt;
    if (!last) {
      c.advance(S, kt + 1);
      c.gload(p, ra, rb);
    }
    ops.template compute<false>(buf, acc);
    if (!last) ops.lstore(buf ^ 1, ra, rb);
    __syncthreads();
  }
  ops.epilogue(p, tab, acc);
}

// ---------------------------------------------------------------------------
// complex64 on FP32 MFMA
template <int WVM, int WVN, int WM, int WN, int MT, int NT, int KT, class GC>
struct OpsC64 {
  static constexpr int kAcc = WN;
  float (*sA)[2][KT][MT];
  float2 (*sB)[KT][NT];
  const GC* c;
  float sa, sb;
  int lane, wave_m, wave_n;
  __device__ __forceinline__ void epilogue(const StepArgs& p, const GemmTables<MT, NT, KT>& t,
                                           floatx16 (&acc)[WM][WN]) {
    c->template epilogue<WVN, WM, WN>(p, t, c->baseC, acc);
  }
  __device__ __forceinline__ void lstore(int buf, const float2* ra, const float2* rb) {
#pragma unroll
    for (int r = 0; r < GC::AE; ++r) {
      const int m = c->a_mk[r] & 0xFFFF, k = c->a_mk[r] >> 16;
      sA[buf][0][k][m] = ra[r].x;
      sA[buf][1][k][m] = sa * ra[r].y;
    }
#pragma unroll
    for (int r = 0; r < GC::BE; ++r)
      sB[buf][c->b_nk[r] >> 16][c->b_nk[r] & 0xFFFF] = make_float2(rb[r].x, sb * rb[r].y);
  }
  // one k column of the tile; ZERO: start from a zero accumulator
  template <bool ZERO>
  __device__ __forceinline__ void kstep(int buf, int kk, floatx16 (&acc)[WM][WN]) {
    const int half = lane >> 5, par = lane & 1;
    float av[WM], bv[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i) av[i] = sA[buf][half][kk][wave_m * WM * 32 + i * 32 + (lane & 31)];
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      float2 bc = sB[buf][kk][wave_n * WN * 16 + j * 16 + ((lane & 31) >> 1)];
      bv[j] = half == 0 ? (par ? bc.y : bc.x) : (par ? bc.x : -bc.y);
    }
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const floatx16 zero = {};
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], ZERO ? zero : acc[i][j], 0,
                                                         0, 0);
      }
  }
  template <bool FIRST>
  __device__ __forceinline__ void compute(int buf, floatx16 (&acc)[WM][WN]) {
    int k0 = 0;
    if constexpr (FIRST) {
      kstep<true>(buf, 0, acc);
      k0 = 1;
    }
#pragma unroll 4
    for (int kk = k0; kk < KT; ++kk) kstep<false>(buf, kk, acc);
  }
};

template <int WVM, int WVN, int WM, int WN, int LK, class OffT>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(LK == 4 && WVM * WM <= 4 && WVM * WM * WVN * WN <= 16 ? 3 : 1)))
k_gemm_c64(GemmArgs g) {
  constexpr int MT = WVM * WM * 32, NT = WVN * WN * 16, KT = 1 << LK;
  using GC = GemmCommon<MT, NT, KT, OffT>;
  static_assert(GC::AE >= 1 && GC::BE >= 1, "tile too small for 256 threads");
  __shared__ float sA[2][2][KT][MT];
  __shared__ float2 sB[2][KT][NT];
  __shared__ GemmTables<MT, NT, KT> tab;
  __shared__ Strides S;
  const StepArgs& p = g.s;
  load_strides(p, S);
  __syncthreads();
  build_tables<MT, NT, KT>(p, S, tab);
  __syncthreads();
  GC c;
  c.init(g, tab);
  OpsC64<WVM, WVN, WM, WN, MT, NT, KT, GC> ops;
  ops.sA = sA;
  ops.sB = sB;
  ops.c = &c;
  ops.sa = p.conjA ? -1.f : 1.f;
  ops.sb = p.conjB ? -1.f : 1.f;
  ops.lane = threadIdx.x & 63;
  ops.wave_m = (threadIdx.x >> 6) / WVN;
  ops.wave_n = (threadIdx.x >> 6) % WVN;
  gemm_tiles<WVN, WM, WN>(p, S, c, tab, ops);
}

// ---------------------------------------------------------------------------
// complex64 with three real products per complex product (Gauss):
//   T1 = Re A Re B,  T2 = Im A Im B,  T3 = (Re A + Im A)(Re B + Im B),
//   Re C = T1 - T2,  Im C = T3 - T1 - T2,
// 6 real flops per complex multiply-add instead of the embedding's 8.  Same
// LDS staging as OpsC64 (A as Re / Im planes, B as complex entries); one
// v_mfma_f32_32x32x2f32 covers two complex k for a 32 x 32 complex block
// (lanes 0-31 the even k, lanes 32-63 the odd one), so a wave's WN 16-column
// blocks become WN / 2 blocks of 32 complex columns with three accumulators
// each.
template <int WVM, int WVN, int WM, int WN, int MT, int NT, int KT, class GC>
struct OpsC64G {
  static_assert(WN % 2 == 0 && KT % 2 == 0, "32-column blocks, k pairs");
  static constexpr int NB = WN / 2;
  static constexpr int kAcc = 3 * NB;
  float (*sA)[2][KT][MT];
  float2 (*sB)[KT][NT];
  const GC* c;
  float sa, sb;
  int lane, wave_m, wave_n;
  __device__ __forceinline__ void lstore(int buf, const float2* ra, const float2* rb) {
#pragma unroll
    for (int r = 0; r < GC::AE; ++r) {
      const int m = c->a_mk[r] & 0xFFFF, k = c->a_mk[r] >> 16;
      sA[buf][0][k][m] = ra[r].x;
      sA[buf][1][k][m] = sa * ra[r].y;
    }
#pragma unroll
    for (int r = 0; r < GC::BE; ++r)
      sB[buf][c->b_nk[r] >> 16][c->b_nk[r] & 0xFFFF] = make_float2(rb[r].x, sb * rb[r].y);
  }
  // one k pair of the tile; ZERO: start from zero accumulators
  template <bool ZERO>
  __device__ __forceinline__ void kstep(int buf, int k2, floatx16 (&acc)[WM][kAcc]) {
    const int k = 2 * k2 + (lane >> 5), l31 = lane & 31;
    float ar[WM], ai[WM], br[NB], bi[NB];
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      ar[i] = sA[buf][0][k][wave_m * WM * 32 + i * 32 + l31];
      ai[i] = sA[buf][1][k][wave_m * WM * 32 + i * 32 + l31];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const float2 bc = sB[buf][k][wave_n * WN * 16 + j * 32 + l31];
      br[j] = bc.x;
      bi[j] = bc.y;
    }
    const floatx16 zero = {};
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      const float as = ar[i] + ai[i];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        acc[i][3 * j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i], br[j],
                                                             ZERO ? zero : acc[i][3 * j], 0, 0, 0);
        acc[i][3 * j + 1] = __builtin_amdgcn_mfma_f32_32x32x2f32(
            ai[i], bi[j], ZERO ? zero : acc[i][3 * j + 1], 0, 0, 0);
        acc[i][3 * j + 2] = __builtin_amdgcn_mfma_f32_32x32x2f32(
            as, br[j] + bi[j], ZERO ? zero : acc[i][3 * j + 2], 0, 0, 0);
      }
    }
  }
  template <bool FIRST>
  __device__ __forceinline__ void compute(int buf, floatx16 (&acc)[WM][kAcc]) {
    int k0 = 0;
    if constexpr (FIRST) {
      kstep<true>(buf, 0, acc);
      k0 = 1;
    }
#pragma unroll 2
    for (int k2 = k0; k2 < KT / 2; ++k2) kstep<false>(buf, k2, acc);
  }
  // lane holds complex column 32 j + (lane & 31) of block j, rows
  // 8 (r / 4) + 4 (lane / 32) + r % 4 of entry r of its three accumulators
  __device__ __forceinline__ void epilogue(const StepArgs& p, const GemmTables<MT, NT, KT>& t,
                                           floatx16 (&acc)[WM][kAcc]) {
    constexpr int LM = ilog2<MT>::value, LN = ilog2<NT>::value;
    const int half = lane >> 5, l31 = lane & 31;
    const int mlim = 1 << (p.nm < LM ? p.nm : LM), nlim = 1 << (p.nn < LN ? p.nn : LN);
    float2* C = p.C + c->baseC;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int col = wave_n * WN * 16 + j * 32 + l31;
      if (col >= nlim) continue;
      const int64_t offn = t.cn[col];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = wave_m * WM * 32 + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          if (row >= mlim) continue;
          const float t1 = acc[i][3 * j][r], t2 = acc[i][3 * j + 1][r], t3 = acc[i][3 * j + 2][r];
          float2 v = make_float2(t1 - t2, t3 - t1 - t2);
          float2* cp = C + offn + t.cm[row];
          if (p.accumulate) {
            const float2 o = *cp;
            v = make_float2(o.x + v.x, o.y + v.y);
          }
          *cp = v;
        }
      }
    }
  }
};

template <int WVM, int WVN, int WM, int WN, int LK, class OffT>
__global__ void __launch_bounds__(256) k_gemm_c64g(GemmArgs g) {
  constexpr int MT = WVM * WM * 32, NT = WVN * WN * 16, KT = 1 << LK;
  using GC = GemmCommon<MT, NT, KT, OffT>;
  static_assert(GC::AE >= 1 && GC::BE >= 1, "tile too small for 256 threads");
  __shared__ float sA[2][2][KT][MT];
  __shared__ float2 sB[2][KT][NT];
  __shared__ GemmTables<MT, NT, KT> tab;
  __shared__ Strides S;
  const StepArgs& p = g.s;
  load_strides(p, S);
  __syncthreads();
  build_tables<MT, NT, KT>(p, S, tab);
  __syncthreads();
  GC c;
  c.init(g, tab);
  OpsC64G<WVM, WVN, WM, WN, MT, NT, KT, GC> ops;
  ops.sA = sA;
  ops.sB = sB;
  ops.c = &c;
  ops.sa = p.conjA ? -1.f : 1.f;
  ops.sb = p.conjB ? -1.f : 1.f;
  ops.lane = threadIdx.x & 63;
  ops.wave_m = (threadIdx.x >> 6) / WVN;
  ops.wave_n = (threadIdx.x >> 6) % WVN;
  gemm_tiles<WVN, WM, WN>(p, S, c, tab, ops);
}

// ---------------------------------------------------------------------------
// split-BF16 (3 products) on BF16 MFMA with float32 accumulation.  LDS holds
// the tile already split: A as [m][kr] and the real-embedded B as
// [real column][kr] (kr = 2 kc + part), hi and lo planes.  Rows are 64 bytes;
// the 16-byte chunk of a row is XOR-swizzled with bits 2-3 of the row so the
// 16 lanes of one ds_read_b128 phase hit 16 distinct bank groups.  The split
// uses the hardware round-to-nearest-even conversion (v_cvt_pk_bf16_f32).
__device__ __forceinline__ int swz(int row, int kr) {
  return row * 32 + ((((kr >> 3) ^ (row >> 2)) & 3) << 3) + (kr & 7);
}

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));

// (x, y) -> packed bf16 hi pair and lo pair
__device__ __forceinline__ void split_pair(float x, float y, uint32_t& hi, uint32_t& lo) {
  f2v v = {x, y};
  b2v h = __builtin_convertvector(v, b2v);
  f2v hf = __builtin_convertvector(h, f2v);
  b2v l = __builtin_convertvector(v - hf, b2v);
  hi = __builtin_bit_cast(uint32_t, h);
  lo = __builtin_bit_cast(uint32_t, l);
}

template <int WVM, int WVN, int WM, int WN, int MT, int NT, int KT, class GC>
struct OpsSB16 {
  static constexpr int kAcc = WN;
  uint16_t (*sA)[2][MT * 32];
  uint16_t (*sB)[2][2 * NT * 32];
  const GC* c;
  uint32_t ca, cb;   // sign masks for the imaginary half (conjugation)
  int lane, wave_m, wave_n;
  __device__ __forceinline__ void epilogue(const StepArgs& p, const GemmTables<MT, NT, KT>& t,
                                           floatx16 (&acc)[WM][WN]) {
    c->template epilogue<WVN, WM, WN>(p, t, c->baseC, acc);
  }
  __device__ __forceinline__ void lstore(int buf, const float2* ra, const float2* rb) {
#pragma unroll
    for (int r = 0; r < GC::AE; ++r) {
      uint32_t hi, lo;
      split_pair(ra[r].x, ra[r].y, hi, lo);
      int o = swz(c->a_mk[r] & 0xFFFF, 2 * (c->a_mk[r] >> 16));
      *reinterpret_cast<uint32_t*>(&sA[buf][0][o]) = hi ^ ca;
      *reinterpret_cast<uint32_t*>(&sA[buf][1][o]) = lo ^ ca;
    }
#pragma unroll
    for (int r = 0; r < GC::BE; ++r) {
      uint32_t hi, lo;
      split_pair(rb[r].x, rb[r].y, hi, lo);   // (Br, Bi) halves, conj applied below
      hi ^= cb;
      lo ^= cb;
      int o = swz(2 * (c->b_nk[r] & 0xFFFF), 2 * (c->b_nk[r] >> 16));
      // real column 2n: (Br, -Bi); real column 2n+1: (Bi, Br)
      *reinterpret_cast<uint32_t*>(&sB[buf][0][o]) = hi ^ 0x80000000u;
      *reinterpret_cast<uint32_t*>(&sB[buf][1][o]) = lo ^ 0x80000000u;
      *reinterpret_cast<uint32_t*>(&sB[buf][0][o + 32]) = (hi >> 16) | (hi << 16);
      *reinterpret_cast<uint32_t*>(&sB[buf][1][o + 32]) = (lo >> 16) | (lo << 16);
    }
  }
  template <bool FIRST>
  __device__ __forceinline__ void compute(int buf, floatx16 (&acc)[WM][WN]) {
    const int half = lane >> 5;
    const floatx16 zero = {};
#pragma unroll
    for (int s2 = 0; s2 < KT / 8; ++s2) {
      const int kof = 16 * s2 + 8 * half;
      bf16x8_t ah[WM], al[WM], bh[WN], bl[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        int row = wave_m * WM * 32 + i * 32 + (lane & 31);
        ah[i] = *reinterpret_cast<const bf16x8_t*>(&sA[buf][0][swz(row, kof)]);
        al[i] = *reinterpret_cast<const bf16x8_t*>(&sA[buf][1][swz(row, kof)]);
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        int col = wave_n * WN * 32 + j * 32 + (lane & 31);
        bh[j] = *reinterpret_cast<const bf16x8_t*>(&sB[buf][0][swz(col, kof)]);
        bl[j] = *reinterpret_cast<const bf16x8_t*>(&sB[buf][1][swz(col, kof)]);
      }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              ah[i], bh[j], FIRST && s2 == 0 ? zero : acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
  }
};

template <int WVM, int WVN, int WM, int WN, class OffT>
__global__ void __launch_bounds__(256) k_gemm_sb16(GemmArgs g) {
  constexpr int KT = 16;
  constexpr int MT = WVM * WM * 32, NT = WVN * WN * 16;
  using GC = GemmCommon<MT, NT, KT, OffT>;
  static_assert(2 * KT == 32, "row layout assumes 32 bf16 per row");
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][2][MT * 32];
  __shared__ __attribute__((aligned(16))) uint16_t sB[2][2][2 * NT * 32];
  __shared__ GemmTables<MT, NT, KT> tab;
  __shared__ Strides S;
  const StepArgs& p = g.s;
  load_strides(p, S);
  __syncthreads();
  build_tables<MT, NT, KT>(p, S, tab);
  __syncthreads();
  GC c;
  c.init(g, tab);
  OpsSB16<WVM, WVN, WM, WN, MT, NT, KT, GC> ops;
  ops.sA = sA;
  ops.sB = sB;
  ops.c = &c;
  ops.ca = p.conjA ? 0x80000000u : 0u;
  ops.cb = p.conjB ? 0x80000000u : 0u;
  ops.lane = threadIdx.x & 63;
  ops.wave_m = (threadIdx.x >> 6) / WVN;
  ops.wave_n = (threadIdx.x >> 6) % WVN;
  gemm_tiles<WVN, WM, WN>(p, S, c, tab, ops);
}

// Sum of the split-k partial tiles of a GEMM step: partial c holds the
// chunk's result at the result's own offsets plus c * n_out (the result is a
// dense layout of n_out entries), added in chunk order in float64.
__global__ void __launch_bounds__(256) k_gemm_splitk_reduce(float2* C, const float2* part,
                                                            int64_t n_out, int32_t nchunk,
                                                            int32_t accumulate) {
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < n_out;
       o += (int64_t)gridDim.x * 256) {
    double re = 0.0, im = 0.0;
    for (int32_t c = 0; c < nchunk; ++c) {
      const float2 v = part[(int64_t)c * n_out + o];
      re += v.x;
      im += v.y;
    }
    if (accumulate) {
      const float2 v = C[o];
      re += v.x;
      im += v.y;
    }
    C[o] = make_float2((float)re, (float)im);
  }
}

}  // namespace tnk
