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
constexpr int kChainB = 1024;   // staged small-operand elements, all steps

struct ChainStepArgs {
  const float2* B;
  int32_t nk, nn, nrow, nbb;                  // summed / new / row bits, batch bits of B
  int32_t kslot[4], nslot[4], kB[4], nB[4];   // LDS slots and B strides of k and n bits
  int32_t rslot[kChainTile];                  // LDS slots of the row bits
  int32_t bB[kChainTile], bpas[kChainTile];   // batch bits: B stride, tile-number bit
};

struct ChainArgs {
  const float2* X;   // chain input (large operand of the first step)
  float2* Y;         // chain output (result of the last step)
  int32_t nsteps, tin, tout, npas;
  int32_t b_per_tile;   // some small operand depends on passive (batch) bits
  int32_t b_total;      // staged small-operand elements (sum of 2^(nk+nn))
  int32_t in_slot[kChainTile], in_log2[kChainTile];    // input tile bits, input-stride order
  int32_t out_slot[kChainTile], out_log2[kChainTile];  // output tile bits, output-stride order
  int32_t pas_in[kChainPas], pas_out[kChainPas];       // passive bits: X / Y strides
  ChainStepArgs st[kChainSteps];
};

// sum_j bit_j(idx) << s[j] over bits [lo, hi)
__device__ __forceinline__ int64_t chain_off(uint64_t idx, const int32_t* s, int lo, int hi) {
  int64_t off = 0;
#pragma unroll 1
  for (int j = lo; j < hi; ++j) off += (int64_t)((idx >> j) & 1ull) << s[j];
  return off;
}

__device__ __forceinline__ int32_t chain_slot(uint32_t idx, const int32_t* s, int lo, int hi) {
  int32_t off = 0;
#pragma unroll 1
  for (int j = lo; j < hi; ++j) off |= (int32_t)((idx >> j) & 1u) << s[j];
  return off;
}

// small operand of a step staged as [n][k]
template <int NK, int NN>
__device__ __forceinline__ void chain_rows(const ChainStepArgs& S, float2* buf, const float2* sB) {
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
  const int lo = nrow < 8 ? nrow : 8;
  const uint32_t rows = 1u << nrow;
  const int32_t rlo = chain_slot(threadIdx.x, S.rslot, 0, lo);
  for (uint32_t r0 = 0; r0 < rows; r0 += 256) {
    if (r0 + threadIdx.x >= rows) break;
    const int32_t base = rlo | chain_slot(r0, S.rslot, 8, nrow);
    float2 a[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = buf[base | koff[k]];
#pragma unroll 1
    for (int n = 0; n < N; ++n) {
      int32_t no = 0;
#pragma unroll
      for (int j = 0; j < NN; ++j) no |= ((n >> j) & 1) << ns[j];
      const float2* bn = sB + n * K;
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < K; ++k) cfma(acc, a[k], bn[k]);
      buf[base | no] = acc;
    }
  }
}

__device__ __forceinline__ void chain_step(const ChainStepArgs& S, float2* buf, const float2* sB) {
  // the per-step stream kernel covers nk, nn in 0..4; so does the chain
#define TNK_CHAIN_CASE(A, B)          \
  if (S.nk == A && S.nn == B) {       \
    chain_rows<A, B>(S, buf, sB);     \
    return;                           \
  }
#define TNK_CHAIN_ROW(A) \
  TNK_CHAIN_CASE(A, 0) TNK_CHAIN_CASE(A, 1) TNK_CHAIN_CASE(A, 2) TNK_CHAIN_CASE(A, 3) TNK_CHAIN_CASE(A, 4)
  TNK_CHAIN_ROW(0) TNK_CHAIN_ROW(1) TNK_CHAIN_ROW(2) TNK_CHAIN_ROW(3) TNK_CHAIN_ROW(4)
#undef TNK_CHAIN_ROW
#undef TNK_CHAIN_CASE
}

template <int TB>
__global__ void __launch_bounds__(256) k_chain(ChainArgs g) {
  __shared__ float2 buf[1 << TB];
  __shared__ float2 sB[kChainB];
  const int tid = threadIdx.x;
  const uint64_t n_tiles = 1ull << g.npas;
  // per-thread parts of the load / store offsets (tile bits 0..7 = thread id)
  const int lo_in = g.tin < 8 ? g.tin : 8, lo_out = g.tout < 8 ? g.tout : 8;
  const int64_t xin_lo = chain_off(tid, g.in_log2, 0, lo_in);
  const int32_t lin_lo = chain_slot(tid, g.in_slot, 0, lo_in);
  const int64_t yout_lo = chain_off(tid, g.out_log2, 0, lo_out);
  const int32_t lout_lo = chain_slot(tid, g.out_slot, 0, lo_out);
  const uint32_t n_in = 1u << g.tin, n_out = 1u << g.tout;
  bool staged = false;
  for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t bx = chain_off(t, g.pas_in, 0, g.npas);
    const int64_t by = chain_off(t, g.pas_out, 0, g.npas);
    // small operands, [n][k] per step
    if (!staged || g.b_per_tile) {
      int off = 0;
      for (int q = 0; q < g.nsteps; ++q) {
        const ChainStepArgs& S = g.st[q];
        const int nk = S.nk, nn = S.nn, cnt = 1 << (nk + nn);
        int64_t bb = 0;
#pragma unroll 1
        for (int j = 0; j < S.nbb; ++j) bb += (int64_t)((t >> S.bpas[j]) & 1ull) << S.bB[j];
        for (int i = tid; i < cnt; i += 256) {
          const int n = i >> nk, k = i & ((1 << nk) - 1);
          sB[off + i] = S.B[bb + chain_off(k, S.kB, 0, nk) + chain_off(n, S.nB, 0, nn)];
        }
        off += cnt;
      }
      staged = true;
    }
    // load the input tile
    for (uint32_t r0 = 0; r0 < n_in; r0 += 256) {
      if (r0 + tid >= n_in) break;
      const int64_t go = bx + xin_lo + chain_off(r0, g.in_log2, 8, g.tin);
      buf[lin_lo | chain_slot(r0, g.in_slot, 8, g.tin)] = g.X[go];
    }
    __syncthreads();
    int off = 0;
    for (int q = 0; q < g.nsteps; ++q) {
      const ChainStepArgs& S = g.st[q];
      chain_step(S, buf, sB + off);
      off += 1 << (S.nk + S.nn);
      __syncthreads();
    }
    // store the output tile
    for (uint32_t r0 = 0; r0 < n_out; r0 += 256) {
      if (r0 + tid >= n_out) break;
      const int64_t go = by + yout_lo + chain_off(r0, g.out_log2, 8, g.tout);
      g.Y[go] = buf[lout_lo | chain_slot(r0, g.out_slot, 8, g.tout)];
    }
    __syncthreads();
  }
}

}  // namespace tnk
