// Fused chains of stream steps.
//
// Along a contraction path the largest tensors usually absorb one small
// tensor after another (a gate, a small slice-dependent piece): each such
// step reads and writes the whole large tensor although it touches only a few
// of its bits.  A chain runs several of these steps in one pass.  The bits
// the chain sums over (plus a few low-stride bits, for coalescing) form the
// tile; the remaining ("passive") bits enumerate tiles.  A workgroup loads
// one tile of the chain input into LDS, applies every step of the chain there
// -- each step maps the tile through its small operand, summing its k bits
// and creating its n bits -- and stores the tile of the chain output.  Bits
// live in fixed LDS slots; a tile buffer holds 2^TB complex values and the
// steps ping-pong between two buffers.
//
// Each output value is computed exactly as the per-step stream kernel does
// (zero start, complex FMAs in increasing k order), so a chain is bitwise
// identical to running its steps one by one.
//
// One LDS buffer holds the tile: a thread owns one row of a step (all tile
// bits but the summed ones), reads the row's 2^nk values into registers and
// writes its 2^nn results back into the same row (the new bits take the slots
// the summed bits freed, plus free ones), so rows never touch each other and
// the step runs in place.  All argument arrays are 32-bit and read at uniform
// indices, so they stay in scalar registers.
#pragma once

#include "kernels_common.h"

namespace tnk {

constexpr int kChainSteps = 8;
constexpr int kChainTile = 12;
constexpr int kChainPas = 40;
constexpr int kChainBF = 4096;  // staged small operands, all steps (floats)
constexpr int kChainV = 512;    // complex entries staged for vector-unit steps

struct ChainStepArgs {
  const float2* B;
  int32_t nk, nn, nrow, nbb;                  // summed / new / row bits, batch bits of B
  int32_t mfma;                               // run on the matrix cores
  int32_t boff0;                              // first staged float of this step
  int32_t voff0;                              // first entry offset in the table (vector steps)
  int32_t kslot[8], nslot[8], kB[8], nB[8];   // LDS slots and B strides of k and n bits
  int32_t rslot[kChainTile];                  // LDS slots of the row bits
  int32_t bB[kChainTile], bpas[kChainTile];   // batch bits: B stride, tile-number bit
};

struct ChainArgs {
  const float2* X;   // chain input (large operand of the first step)
  float2* Y;         // chain output (result of the last step)
  int32_t nsteps, tin, tout, npas;
  int32_t b_per_tile;   // some small operand depends on passive (batch) bits
  int32_t b_total;      // staged small-operand floats
  int32_t split;        // matrix-core steps in split-BF16 (three BF16 products)
  int32_t in_slot[kChainTile], in_log2[kChainTile];    // input tile bits, input-stride order
  int32_t out_slot[kChainTile], out_log2[kChainTile];  // output tile bits, output-stride order
  int32_t pas_in[kChainPas], pas_out[kChainPas];       // passive bits: X / Y strides
  // with t = blockIdx.x + m gridDim.x: X / Y offset change from tile m to
  // m + 1 is din / dout[ctz(m + 1)]
  int64_t din[kChainPas], dout[kChainPas];
  ChainStepArgs st[kChainSteps];
};

// The arguments are read in place from the kernel-argument segment (constant
// address space): every index into them is uniform, so they come in through
// scalar loads and no private copy of the structure is made.
#define TNK_KARG __attribute__((address_space(4)))
typedef const TNK_KARG int32_t karg_i32;
typedef const TNK_KARG ChainStepArgs karg_step;
typedef const TNK_KARG ChainArgs karg_chain;

// sum_j bit_j(idx) << s[j] over bits [lo, hi)
__device__ __forceinline__ int64_t chain_off(uint64_t idx, karg_i32* s, int lo, int hi) {
  int64_t off = 0;
#pragma unroll 1
  for (int j = lo; j < hi; ++j) off += (int64_t)((idx >> j) & 1ull) << s[j];
  return off;
}

__device__ __forceinline__ int32_t chain_slot(uint32_t idx, karg_i32* s, int lo, int hi) {
  int32_t off = 0;
#pragma unroll 1
  for (int j = lo; j < hi; ++j) off |= (int32_t)((idx >> j) & 1u) << s[j];
  return off;
}

// LDS positions are XOR-swizzled: bits 5..11 of a slot index are folded into
// bits 0..4 (the bank of an 8-byte element), so lanes whose positions differ
// only in high slots do not all hit one bank.  The map is XOR-linear and only
// changes bits 0..4, hence a bijection of every 2^TB buffer, and it commutes
// with assembling a position from disjoint bit groups.
__device__ __forceinline__ int32_t chain_swz(int32_t x) {
  return x ^ (((x >> 5) ^ (x >> 9)) & 31);
}

// Per-workgroup tables, built once before the tile loop: everything that
// does not depend on the tile.
#define TNK_GLOBAL __attribute__((address_space(1)))
typedef float chain_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 chain_ld(const TNK_GLOBAL chain_f2* p, int64_t i) {
  const chain_f2 v = p[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void chain_st(TNK_GLOBAL chain_f2* p, int64_t i, float2 v) {
  p[i] = chain_f2{v.x, v.y};
}

// Offsets of tile element (e << 8) + tid: the part of the high bits e is
// linear in those bits, so it is kept as one term per bit (HBM offsets add,
// swizzled LDS byte offsets XOR) and formed on the scalar unit per element.
struct ChainElemOffsets {
  int32_t o[4];   // log2 strides of element bits 8.. (bits beyond the tile are never set)
  int32_t l[4];
  __device__ __forceinline__ ChainElemOffsets(const karg_i32* log2s, const karg_i32* slots, int n) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      o[b] = 8 + b < n ? log2s[8 + b] : 0;
      l[b] = 8 + b < n ? 8 * chain_swz(1 << slots[8 + b]) : 0;
    }
  }
  // Makes the terms opaque to the compiler at this point, so offsets are
  // formed where they are used instead of being hoisted (and kept live)
  // out of the tile loop.
  __device__ __forceinline__ void refresh() {
    asm volatile("" : "+s"(o[0]), "+s"(o[1]), "+s"(o[2]), "+s"(o[3]));
    asm volatile("" : "+s"(l[0]), "+s"(l[1]), "+s"(l[2]), "+s"(l[3]));
  }
  __device__ __forceinline__ int64_t hbm(int e) const {
    int64_t r = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if ((e >> b) & 1) r += (int64_t)1 << o[b];
    return r;
  }
  __device__ __forceinline__ int32_t lds(int e) const {
    int32_t r = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if ((e >> b) & 1) r ^= l[b];
    return r;
  }
};


// small operand of a step staged as [n][k]
template <int NK, int NN>
__device__ __forceinline__ void chain_rows(karg_step& S, float2* buf, const float2* sB) {
  constexpr int K = 1 << NK, N = 1 << NN;
  int32_t koff[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int32_t o = 0;
#pragma unroll
    for (int j = 0; j < NK; ++j) o |= ((k >> j) & 1) << S.kslot[j];
    koff[k] = o;
  }
  int32_t ns[NN > 0 ? NN : 1];
#pragma unroll
  for (int j = 0; j < NN; ++j) ns[j] = S.nslot[j];
  const int nrow = S.nrow;
  const uint32_t rows = 1u << nrow;
  int32_t rlo = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < nrow) rlo |= ((threadIdx.x >> j) & 1) << S.rslot[j];
  for (uint32_t r0 = 0; r0 < rows; r0 += 256) {
    if (r0 + threadIdx.x >= rows) break;
    // rows of 256-row group r0 / 256: its bits sit at row slots 8..nrow-1
    int32_t rh = 0;
    for (int j = 8; j < nrow; ++j) rh |= (int32_t)((r0 >> j) & 1u) << S.rslot[j];
    const int32_t base = rlo | rh;
    float2 a[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = buf[chain_swz(base | koff[k])];
    // one output column at a time: its K small-operand values are LDS
    // broadcasts (every lane reads the same address)
#pragma unroll 1
    for (int n = 0; n < N; ++n) {
      int32_t no = 0;
#pragma unroll
      for (int j = 0; j < NN; ++j) no |= ((n >> j) & 1) << ns[j];
      const float2* bn = sB + n * K;
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < K; ++k) cfma(acc, a[k], bn[k]);
      buf[chain_swz(base | no)] = acc;
    }
  }
}

// The same step on the FP32 matrix cores (v_mfma_f32_16x16x4f32) for
// 4 <= 2^nk <= 64 summed and 8 <= 2^nn <= 32 new values, 2^(nk+nn) <= 512
// (the plan's rule): the complex product is the real one of A' (rows x 2K,
// re/im interleaved) and B' = [[Br, Bi], [-Bi, Br]] (2K x 2N).  A wave takes
// 16 rows at a time.  In k step s, lane group g = lane / 16 supplies complex
// k = g K/4 + s/2, real part s % 2, so a lane reads its row's K/4 values
// once; B' is staged in LDS in the order the lanes read it (one float per
// lane and instruction, consecutive across lanes), and held in registers
// for the whole step when it is small.  Output lane layout: rows
// 4 (lane / 16) + r, real column lane % 16 of the 16-column block (which
// column that is: chain_col).  The row's values are all read before any is written, and 16-row blocks of
// different waves are disjoint, so the step runs in place.  Sums run in the
// matrix core's order, not the stream kernel's.
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Byte offset (times 8, swizzled) of the high row part of 16-row block rb:
// the bits of rb sit at row slots rslot[4..nrow-1], and since the swizzle is
// XOR-linear the offset is the XOR of one term per set bit of rb.  Block
// numbers are wave-uniform, so this runs on the scalar unit.
struct ChainBlockRows {
  int32_t H[6];
  __device__ __forceinline__ explicit ChainBlockRows(karg_step& S) {
#pragma unroll
    for (int t = 0; t < 6; ++t) H[t] = t + 4 < S.nrow ? 8 * chain_swz(1 << S.rslot[4 + t]) : 0;
  }
  __device__ __forceinline__ int32_t operator()(uint32_t rb) const {
    int32_t h = 0;
#pragma unroll
    for (int t = 0; t < 6; ++t)
      if ((rb >> t) & 1u) h ^= H[t];
    return h;
  }
};

// Real output column of lane li in 16-column block cb.  With two or more
// blocks, blocks 2c and 2c + 1 hold the real and imaginary parts of complex
// columns 16 c .. 16 c + 15, so a lane ends with both parts of one value and
// writes it as one 8-byte store; a single block holds 8 complex columns with
// real and imaginary parts in alternate lanes.
__device__ __forceinline__ void chain_col(int cb, int li, int CB, int& n, int& q) {
  if (CB >= 2) {
    n = 16 * (cb >> 1) + li;
    q = cb & 1;
  } else {
    n = li >> 1;
    q = li & 1;
  }
}

template <int NK, int NN>
__device__ __forceinline__ void chain_rows_mfma(karg_step& S, float2* buf, const float* sBf) {
  constexpr int K = 1 << NK, N = 1 << NN;
  constexpr int KG = K / 4;          // complex k per lane group
  constexpr int KS = K / 2;          // k steps of 4 real values
  constexpr int CB = N / 8;          // 16-column blocks of the real output
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const ChainBlockRows brow(S);
  const int g = lane >> 4, li = lane & 15;
  // B' was staged as [cb][k step][lane] (see the staging in k_chain)
  const float* bw = sBf + lane;
  int32_t ks[NK];
#pragma unroll
  for (int t = 0; t < NK; ++t) ks[t] = S.kslot[t];
  int32_t koff[KG];
#pragma unroll
  for (int j = 0; j < KG; ++j) {
    const int k = g * KG + j;
    int32_t o = 0;
#pragma unroll
    for (int t = 0; t < NK; ++t) o |= ((k >> t) & 1) << ks[t];
    koff[j] = o;
  }
  constexpr int CP = CB >= 2 ? CB / 2 : 1;   // stores per output row
  int32_t noff[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) {
    int n, qq;
    chain_col(2 * c, li, CB, n, qq);
    int32_t o = 0;
#pragma unroll
    for (int t = 0; t < NN; ++t) o |= ((n >> t) & 1) << S.nslot[t];
    noff[c] = o;
  }
  // in-block row offsets: the lane's input row li, its output rows 4 g + r
  int32_t rs[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) rs[t] = S.rslot[t];
  int32_t in_lo = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) in_lo |= ((li >> t) & 1) << rs[t];
  int32_t out_lo[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int32_t o = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) o |= (((4 * g + r) >> t) & 1) << rs[t];
    out_lo[r] = o;
  }
  const uint32_t blocks = 1u << (S.nrow - 4);
  // Byte offsets in LDS.  A position is the OR of disjoint bit groups and
  // the swizzle is XOR-linear, so swz(hi | c) = swz(hi) ^ swz(c): the lane's
  // parts are swizzled once per step, the block's part once per block, and
  // an address is one XOR (times 8 bytes; bit 2 carries the real / imaginary
  // half of an output value, which the block part never has).
  char* lb = reinterpret_cast<char*>(buf);
  const int q = CB >= 2 ? 0 : li & 1;
  int32_t ra[KG], wr[4], wn[CP];
#pragma unroll
  for (int j = 0; j < KG; ++j) ra[j] = 8 * chain_swz(in_lo | koff[j]);
#pragma unroll
  for (int r = 0; r < 4; ++r) wr[r] = 8 * chain_swz(out_lo[r]) + 4 * q;
#pragma unroll
  for (int c = 0; c < CP; ++c) wn[c] = 8 * chain_swz(noff[c]);
  // B' is held in registers for the whole step when it is small, else read
  // per block
  constexpr bool BREG = KS * CB <= 16;
  float bv[BREG ? KS * CB : 1];
  if (BREG) {
#pragma unroll
    for (int i = 0; i < KS * CB; ++i) bv[i] = bw[i * 64];
  }
  // The next block's values are read while this block's products run (two
  // register sets used in turn, when they fit); blocks have disjoint rows, so
  // reading the next block before this one is written is safe.
  constexpr bool DB = KG <= 4;
  auto load = [&](uint32_t rb, int32_t& hh, float2 (&x)[KG]) {
    hh = brow(rb);
#pragma unroll
    for (int j = 0; j < KG; ++j) x[j] = *reinterpret_cast<const float2*>(lb + (hh ^ ra[j]));
  };
  auto block = [&](int32_t hh, const float2 (&x)[KG]) {
    floatx4 acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s2 = 0; s2 < KS; ++s2) {
      const float av = (s2 & 1) ? x[s2 >> 1].y : x[s2 >> 1].x;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
            av, BREG ? bv[BREG ? cb * KS + s2 : 0] : bw[(cb * KS + s2) * 64], acc[cb], 0, 0, 0);
    }
    if (CB >= 2) {
#pragma unroll
      for (int c = 0; c < CP; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float* o = reinterpret_cast<float*>(lb + (hh ^ wn[c] ^ wr[r]));
          o[0] = acc[2 * c][r];
          o[1] = acc[2 * c + 1][r];
        }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) *reinterpret_cast<float*>(lb + (hh ^ wn[0] ^ wr[r])) = acc[0][r];
    }
  };
  if (DB) {
    int32_t h0 = 0, h1 = 0;
    float2 a0[KG], a1[KG];
    if ((uint32_t)wave < blocks) load(wave, h0, a0);
    for (uint32_t rb = wave; rb < blocks; rb += 8) {
      if (rb + 4 < blocks) load(rb + 4, h1, a1);
      block(h0, a0);
      if (rb + 4 >= blocks) break;
      if (rb + 8 < blocks) load(rb + 8, h0, a0);
      block(h1, a1);
    }
  } else {
    for (uint32_t rb = wave; rb < blocks; rb += 4) {
      int32_t h0;
      float2 a0[KG];
      load(rb, h0, a0);
      block(h0, a0);
    }
  }
}

// Split-BF16 variant (v_mfma_f32_16x16x16_bf16): each real value x is
// hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest even), and
// the product is hi*hi + hi*lo + lo*hi with float32 accumulation.  A k step
// covers 16 real k: lane group g supplies real k 4g .. 4g+3, i.e. complex
// k = 8 s + 2 g and 8 s + 2 g + 1 (zero beyond K when K = 4).  B' hi and lo
// are staged as 4 BF16 per lane, in the lanes' read order.
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 b4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void chain_split4(f4v v, shortx4& hi, shortx4& lo) {
  const b4v h = __builtin_convertvector(v, b4v);
  const f4v hf = __builtin_convertvector(h, f4v);
  const b4v l = __builtin_convertvector(v - hf, b4v);
  hi = __builtin_bit_cast(shortx4, h);
  lo = __builtin_bit_cast(shortx4, l);
}

template <int NK, int NN>
__device__ __forceinline__ void chain_rows_mfma_sb(karg_step& S, float2* buf, const float* sBf) {
  constexpr int K = 1 << NK, N = 1 << NN;
  constexpr int KS = K >= 8 ? K / 8 : 1;   // k steps of 16 real values
  constexpr int CB = N / 8;                // 16-column blocks of the real output
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const ChainBlockRows brow(S);
  const int g = lane >> 4, li = lane & 15;
  const shortx4* bh = reinterpret_cast<const shortx4*>(sBf) + lane;
  const shortx4* bl = bh + CB * KS * 64;
  int32_t ks[NK];
#pragma unroll
  for (int t = 0; t < NK; ++t) ks[t] = S.kslot[t];
  // complex k of the lane: 8 s + 2 g + e, e = 0, 1
  int32_t koff[KS][2];
  bool kok[KS][2];
#pragma unroll
  for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int k = 8 * s2 + 2 * g + e;
      int32_t o = 0;
#pragma unroll
      for (int t = 0; t < NK; ++t) o |= ((k >> t) & 1) << ks[t];
      koff[s2][e] = o;
      kok[s2][e] = k < K;
    }
  constexpr int CP = CB >= 2 ? CB / 2 : 1;
  int32_t noff[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) {
    int n, qq;
    chain_col(2 * c, li, CB, n, qq);
    int32_t o = 0;
#pragma unroll
    for (int t = 0; t < NN; ++t) o |= ((n >> t) & 1) << S.nslot[t];
    noff[c] = o;
  }
  int32_t rs[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) rs[t] = S.rslot[t];
  int32_t in_lo = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) in_lo |= ((li >> t) & 1) << rs[t];
  int32_t wr[4], wn[CP];
  const int q = CB >= 2 ? 0 : li & 1;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int32_t o = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) o |= (((4 * g + r) >> t) & 1) << rs[t];
    wr[r] = 8 * chain_swz(o) + 4 * q;
  }
#pragma unroll
  for (int c = 0; c < CP; ++c) wn[c] = 8 * chain_swz(noff[c]);
  int32_t ra[KS][2];
#pragma unroll
  for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
    for (int e = 0; e < 2; ++e) ra[s2][e] = 8 * chain_swz(in_lo | koff[s2][e]);
  char* lb = reinterpret_cast<char*>(buf);
  const uint32_t blocks = 1u << (S.nrow - 4);
  constexpr bool BREG = KS * CB <= 4;   // B' hi and lo in registers for the step
  shortx4 rh[BREG ? KS * CB : 1], rl[BREG ? KS * CB : 1];
  if (BREG) {
#pragma unroll
    for (int i = 0; i < KS * CB; ++i) {
      rh[i] = bh[i * 64];
      rl[i] = bl[i * 64];
    }
  }
  // as in the FP32 variant: the next block's values are read early (two
  // register sets used in turn, when they fit)
  constexpr bool DB = KS <= 2;
  auto load = [&](uint32_t rb, int32_t& hh, float2 (&x)[KS][2]) {
    hh = brow(rb);
#pragma unroll
    for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
      for (int e = 0; e < 2; ++e)
        x[s2][e] = kok[s2][e] ? *reinterpret_cast<const float2*>(lb + (hh ^ ra[s2][e]))
                              : make_float2(0.f, 0.f);
  };
  auto block = [&](int32_t hh, const float2 (&x)[KS][2]) {
    shortx4 ah[KS], al[KS];
#pragma unroll
    for (int s2 = 0; s2 < KS; ++s2) {
      const f4v v = {x[s2][0].x, x[s2][0].y, x[s2][1].x, x[s2][1].y};
      chain_split4(v, ah[s2], al[s2]);
    }
    floatx4 acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int i = cb * KS + s2;
        const shortx4 vh = BREG ? rh[BREG ? i : 0] : bh[i * 64];
        const shortx4 vl = BREG ? rl[BREG ? i : 0] : bl[i * 64];
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[s2], vh, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[s2], vl, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[s2], vh, acc[cb], 0, 0, 0);
      }
    if (CB >= 2) {
#pragma unroll
      for (int c = 0; c < CP; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float* o = reinterpret_cast<float*>(lb + (hh ^ wn[c] ^ wr[r]));
          o[0] = acc[2 * c][r];
          o[1] = acc[2 * c + 1][r];
        }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) *reinterpret_cast<float*>(lb + (hh ^ wn[0] ^ wr[r])) = acc[0][r];
    }
  };
  if (DB) {
    int32_t h0 = 0, h1 = 0;
    float2 a0[KS][2], a1[KS][2];
    if ((uint32_t)wave < blocks) load(wave, h0, a0);
    for (uint32_t rb = wave; rb < blocks; rb += 8) {
      if (rb + 4 < blocks) load(rb + 4, h1, a1);
      block(h0, a0);
      if (rb + 4 >= blocks) break;
      if (rb + 8 < blocks) load(rb + 8, h0, a0);
      block(h1, a1);
    }
  } else {
    for (uint32_t rb = wave; rb < blocks; rb += 4) {
      int32_t h0;
      float2 a0[KS][2];
      load(rb, h0, a0);
      block(h0, a0);
    }
  }
}

// Builds of the chain kernel (CLS):
//  0  every step shape, no prefetch;
//  1  no split-BF16 matrix-core step with 2^nk >= 32 (the only shapes that
//     need far more registers than the rest): room to prefetch the next tile;
//  2  small shapes only (chain_small_step): few enough registers for 4 waves
//     per SIMD (matrix steps up to 2^4 x 2^4, vector steps up to 2^3 x 2^4
//     and 2^4 x 2^2), used when the chain's staged operands also leave room for 4
//     workgroups per CU.
// The launcher picks the build from the chain's steps and staging size.
__host__ __device__ constexpr bool chain_small_step(int nk, int nn, bool mfma) {
  return mfma ? (nk <= 4 && nn <= 4) : (nk <= 3 && nn <= 4) || (nk == 4 && nn <= 2);
}

template <int CLS>
__device__ __forceinline__ void chain_step(karg_step& S, float2* buf, const float* sBf, bool split) {
  constexpr bool LIGHT = CLS != 0, SMALL = CLS == 2;
#define TNK_CHAIN_MFMA(A, B)                      \
  if (S.nk == A && S.nn == B) {                   \
    if (split)                                    \
      chain_rows_mfma_sb<A, B>(S, buf, sBf);      \
    else                                          \
      chain_rows_mfma<A, B>(S, buf, sBf);         \
    return;                                       \
  }
  if (S.mfma) {
    TNK_CHAIN_MFMA(2, 3) TNK_CHAIN_MFMA(2, 4) TNK_CHAIN_MFMA(3, 3) TNK_CHAIN_MFMA(3, 4)
    TNK_CHAIN_MFMA(4, 3) TNK_CHAIN_MFMA(4, 4)
    if constexpr (!SMALL) {
      TNK_CHAIN_MFMA(2, 5) TNK_CHAIN_MFMA(3, 5) TNK_CHAIN_MFMA(4, 5)
      if (!split || !LIGHT) {
        TNK_CHAIN_MFMA(5, 3) TNK_CHAIN_MFMA(5, 4)
        TNK_CHAIN_MFMA(6, 3)
      }
    }
  }
#undef TNK_CHAIN_MFMA
  const float2* sB = reinterpret_cast<const float2*>(sBf);
  // the per-step stream kernel covers nk, nn in 0..4; so does the chain
#define TNK_CHAIN_CASE(A, B)                \
  if (S.nk == A && S.nn == B) {             \
    chain_rows<A, B>(S, buf, sB);           \
    return;                                 \
  }
#define TNK_CHAIN_ROW(A) \
  TNK_CHAIN_CASE(A, 0) TNK_CHAIN_CASE(A, 1) TNK_CHAIN_CASE(A, 2) TNK_CHAIN_CASE(A, 3) TNK_CHAIN_CASE(A, 4)
  TNK_CHAIN_ROW(0) TNK_CHAIN_ROW(1) TNK_CHAIN_ROW(2) TNK_CHAIN_ROW(3)
  TNK_CHAIN_CASE(4, 0) TNK_CHAIN_CASE(4, 1) TNK_CHAIN_CASE(4, 2)
  if constexpr (!SMALL) {
    TNK_CHAIN_CASE(4, 3) TNK_CHAIN_CASE(4, 4)
  }
#undef TNK_CHAIN_ROW
#undef TNK_CHAIN_CASE
}

// Split-BF16 staging: entry i (lane i % 64, k step (i / 64) % KS, column
// block i / (64 KS)) holds the lane's 4 real k of B' as BF16 hi, and the
// same index past CB KS 64 entries as BF16 lo.
__device__ __forceinline__ void chain_stage_mfma_sb(karg_step& S, const float2* B, float* dst) {
  const int nk = S.nk, nn = S.nn, K = 1 << nk;
  const int KS = K >= 8 ? K / 8 : 1, CB = (1 << nn) / 8;
  const int cnt = CB * KS * 64;
  shortx4* dh = reinterpret_cast<shortx4*>(dst);
  shortx4* dl = dh + cnt;
  for (int i = threadIdx.x; i < cnt; i += 256) {
    const int lane = i & 63, s2 = (i >> 6) % KS, cb = (i >> 6) / KS;
    const int g = lane >> 4, li = lane & 15;
    int n, q;
    chain_col(cb, li, CB, n, q);
    float v[4];
    for (int j = 0; j < 4; ++j) {
      const int kr = 16 * s2 + 4 * g + j, k = kr >> 1, p = kr & 1;
      float x = 0.f;
      if (k < K) {
        const float2 b = B[chain_off(k, S.kB, 0, nk) + chain_off(n, S.nB, 0, nn)];
        x = p ? (q ? b.x : -b.y) : (q ? b.y : b.x);
      }
      v[j] = x;
    }
    shortx4 h, l;
    chain_split4(f4v{v[0], v[1], v[2], v[3]}, h, l);
    dh[i] = h;
    dl[i] = l;
  }
}

// Stage the small operand of a matrix-core step as B' in the lanes' read
// order: float i is lane i % 64, k step (i / 64) % KS, column block
// i / (64 KS); lane (g, li) holds the real column of chain_col (complex n,
// part q) and real k row s of lane group g (complex k = g K/4 + s/2, part p).
__device__ __forceinline__ void chain_stage_mfma(karg_step& S, const float2* B, float* dst) {
  const int nk = S.nk, nn = S.nn, K = 1 << nk;
  const int KG = K / 4, KS = K / 2, CB = (1 << nn) / 8;
  const int cnt = 4 << (nk + nn);
  for (int i = threadIdx.x; i < cnt; i += 256) {
    const int lane = i & 63, s2 = (i >> 6) % KS, cb = (i >> 6) / KS;
    const int g = lane >> 4, li = lane & 15;
    int n, q;
    chain_col(cb, li, CB, n, q);
    const int k = g * KG + (s2 >> 1), p = s2 & 1;
    const float2 b = B[chain_off(k, S.kB, 0, nk) + chain_off(n, S.nB, 0, nn)];
    dst[i] = p ? (q ? b.x : -b.y) : (q ? b.y : b.x);
  }
}

// The staged small operands live in dynamic LDS sized per launch (the
// floats ChainArgs::b_total), so chains with small operands leave room for
// more workgroups per CU.
extern __shared__ __attribute__((aligned(16))) float chain_staged[];

// CLS (see chain_step): build 1 loads the next tile's input into registers
// while this tile's steps run, so its latency overlaps the arithmetic;
// build 2 runs at 4 waves per SIMD instead.
template <int TB, int CLS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CLS == 2 ? 4 : 3)))
k_chain(ChainArgs) {
  constexpr bool PF = CLS == 1;
  constexpr int E = TB > 8 ? 1 << (TB - 8) : 1;   // tile elements per thread, at most
  constexpr int EB = E < 8 ? E : 8;                // loads in flight per batch
  __shared__ float2 buf[1 << TB];
  float* sBf = chain_staged;
  karg_chain& g = *(karg_chain*)__builtin_amdgcn_kernarg_segment_ptr();
  const int tid = threadIdx.x;
  const int nsteps = g.nsteps, npas = g.npas, tin = g.tin, tout = g.tout;
  // tile numbers: t = blockIdx.x + m * gridDim.x with gridDim.x a power of two,
  // so the low tile bits are this workgroup's and only the high ones (m)
  // vary.  Going from m to m + 1 flips bits 0..c of m, c = ctz(m + 1): the
  // tile's offsets change by din[c] / dout[c].
  const int lg = 31 - __builtin_clz(gridDim.x);
  const int64_t bx_lo = chain_off(blockIdx.x, g.pas_in, 0, lg < npas ? lg : npas);
  const int64_t by_lo = chain_off(blockIdx.x, g.pas_out, 0, lg < npas ? lg : npas);
  const int lo_in = tin < 8 ? tin : 8, lo_out = tout < 8 ? tout : 8;
  const int64_t xin_lo = chain_off(tid, g.in_log2, 0, lo_in);
  const int32_t lin8 = 8 * chain_swz(chain_slot(tid, g.in_slot, 0, lo_in));
  const int64_t yout_lo = chain_off(tid, g.out_log2, 0, lo_out);
  const int32_t lout8 = 8 * chain_swz(chain_slot(tid, g.out_slot, 0, lo_out));
  char* lb = reinterpret_cast<char*>(buf);
  const uint32_t n_in = 1u << tin, n_out = 1u << tout;
  // elements per thread (uniform) and whether this thread has element 0
  const int ne_in = tin > 8 ? 1 << (tin - 8) : 1, ne_out = tout > 8 ? 1 << (tout - 8) : 1;
  const bool in_ok = (uint32_t)tid < n_in, out_ok = (uint32_t)tid < n_out;
  ChainElemOffsets ei(g.in_log2, g.in_slot, tin), eo(g.out_log2, g.out_slot, tout);
  // tensor base addresses, kept in scalar registers (refreshed per tile so
  // they are not reloaded from the argument segment at every use)
  uint64_t xa = (uint64_t)g.X, ya = (uint64_t)g.Y;
  // a tile of 256 or more elements has every thread busy: the guards are
  // then uniform (whole elements), else only element 0 of some threads
  const bool lane_in = in_ok || tin >= 8, lane_out = out_ok || tout >= 8;
  const uint64_t n_tiles = 1ull << npas;
  __syncthreads();
  float2 pf[PF ? E : 1];
  if (PF && blockIdx.x < n_tiles) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (e < ne_in && lane_in) pf[e] = chain_ld((const TNK_GLOBAL chain_f2*)xa, bx_lo + xin_lo + ei.hbm(e));
  }
  int64_t bx = bx_lo, by = by_lo;
  uint64_t m = 0;
  // Small operands that depend on batch bits of the tile number are staged
  // again only when such a bit changes: bits below lg are this workgroup's
  // and never change; bit lg + b flips from tile m to m + 1 iff b <= ctz(m+1).
  int bmin = 64;
  if (g.b_per_tile)
    for (int q = 0; q < nsteps; ++q)
      for (int j = 0; j < g.st[q].nbb; ++j) {
        const int b = g.st[q].bpas[j] - lg;
        if (b >= 0 && b < bmin) bmin = b;
      }
  bool restage = true;
  for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x, ++m) {
    ei.refresh();
    eo.refresh();
    asm volatile("" : "+s"(xa), "+s"(ya));
    const TNK_GLOBAL chain_f2* Xp = (const TNK_GLOBAL chain_f2*)xa;
    TNK_GLOBAL chain_f2* Yp = (TNK_GLOBAL chain_f2*)ya;
    const bool more = t + gridDim.x < n_tiles;
    const int cm = more ? (int)__builtin_ctzll(m + 1) : 0;
    const int64_t dbx = more ? g.din[cm] : 0, dby = more ? g.dout[cm] : 0;
    // small operands: [n][k] complex (vector steps) or B' (matrix steps)
    if (restage) {
      for (int q = 0; q < nsteps; ++q) {
        karg_step& S = g.st[q];
        int64_t bb = 0;
#pragma unroll 1
        for (int j = 0; j < S.nbb; ++j) bb += (int64_t)((t >> S.bpas[j]) & 1ull) << S.bB[j];
        const float2* B = S.B + bb;
        if (S.mfma && g.split) {
          chain_stage_mfma_sb(S, B, sBf + S.boff0);
        } else if (S.mfma) {
          chain_stage_mfma(S, B, sBf + S.boff0);
        } else {
          const int nk = S.nk, nn = S.nn, cnt = 1 << (nk + nn);
          float2* dst = reinterpret_cast<float2*>(sBf + S.boff0);
          for (int i = tid; i < cnt; i += 256) {
            const int n = i >> nk, k = i & ((1 << nk) - 1);
            dst[i] = B[chain_off(k, S.kB, 0, nk) + chain_off(n, S.nB, 0, nn)];
          }
        }
      }
      restage = false;
    }
    restage = more && cm >= bmin;
    if (PF) {
      // the prefetched tile into LDS, then the next tile's loads
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (e < ne_in && lane_in) *reinterpret_cast<float2*>(lb + (lin8 ^ ei.lds(e))) = pf[e];
      __syncthreads();
      if (more) {
        const int64_t bxn = bx + dbx;
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (e < ne_in && lane_in) pf[e] = chain_ld(Xp, bxn + xin_lo + ei.hbm(e));
      }
    } else {
      // load the input tile, eight loads per thread in flight at a time
#pragma unroll
      for (int e0 = 0; e0 < E; e0 += EB) {
        float2 v[EB];
#pragma unroll
        for (int e = 0; e < EB; ++e)
          if (e0 + e < ne_in && lane_in) v[e] = chain_ld(Xp, bx + xin_lo + ei.hbm(e0 + e));
#pragma unroll
        for (int e = 0; e < EB; ++e)
          if (e0 + e < ne_in && lane_in)
            *reinterpret_cast<float2*>(lb + (lin8 ^ ei.lds(e0 + e))) = v[e];
      }
      __syncthreads();
    }
    for (int q = 0; q < nsteps; ++q) {
      karg_step& S = g.st[q];
      chain_step<CLS>(S, buf, sBf + S.boff0, g.split != 0);
      __syncthreads();
    }
    // store the output tile
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += EB) {
      float2 v[EB];
#pragma unroll
      for (int e = 0; e < EB; ++e)
        if (e0 + e < ne_out && lane_out)
          v[e] = *reinterpret_cast<const float2*>(lb + (lout8 ^ eo.lds(e0 + e)));
#pragma unroll
      for (int e = 0; e < EB; ++e)
        if (e0 + e < ne_out && lane_out) chain_st(Yp, by + yout_lo + eo.hbm(e0 + e), v[e]);
    }
    __syncthreads();
    bx += dbx;
    by += dby;
  }
}

}  // namespace tnk
