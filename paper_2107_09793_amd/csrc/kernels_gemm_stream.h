// Skinny GEMM steps as a stream over row bands (complex64 on FP32 MFMA).
//
// Shapes with few columns and summed values against many rows (a column tile
// of at most 128 complex columns times all k within 2^13 complex entries,
// 2^5 - 2^40 rows), which one-tile-per-workgroup kernels run far below the
// matrix-core and memory rates: every tile would restage B, rebuild its
// offset tables and drain its pipeline.  Here a workgroup of 8 waves (2 per
// SIMD, one workgroup per CU) stages the B block of its column tile -- every
// k -- in LDS once, and each wave then walks its own 32-row bands: per band
// it streams A through a wave-private LDS buffer in k tiles (the next tile's
// loads in flight while the matrix cores work on the current one) and writes
// the 32-row result band once.  No workgroup barrier follows the staging of
// B, so the waves drift apart and one wave's loads and stores overlap the
// other's matrix-core work on the same SIMD.
//
// Every A entry is read once per column tile.  Workgroups 8j .. 8j+7 (one per
// XCD) share a column tile and consecutive groups of 8 cycle over the column
// tiles, so the column tiles of one band run on the same XCD (one L2) at about
// the same time.
//
// Arithmetic per MFMA is the real embedding of the tile kernels: one
// v_mfma_f32_32x32x2f32 covers one complex k for 32 rows and 16 complex
// columns (lanes 0-31: Re A and the first row of B's 2x2 block, lanes 32-63:
// Im A and the second row).
#pragma once

#include "kernels_gemm.h"

namespace tnk {

constexpr int kStreamWaves = 8;            // waves per workgroup (2 per SIMD)
constexpr int kStreamBEntries = 1 << 13;   // complex entries of a staged B block
constexpr int kStreamMaxK = 1 << 9;

struct StreamGemmArgs {
  StepArgs s;
  // enumeration of a band's k tile (5 row bits, then the k tile's bits):
  // bit j set = row bit, in the order of tile_mask (ascending A stride)
  uint32_t a_mask;
  int32_t lnt;       // log2 column tiles
  uint64_t nbands;   // 32-row bands: 2^(nm - 5)
};

// LDS position of A entry (k, row) of a band's k tile: the 32 rows of one k
// are consecutive floats, XOR-swizzled by k so that staging writes of
// interleaved (row, k) enumerations spread over the banks; reads of one k by
// 32 lanes stay a permutation of 32 consecutive floats.
__device__ __forceinline__ int sa_pos(int k, int row) { return k * 32 + (row ^ ((k << 2) & 31)); }

template <int WN, int LKT>
__global__ void __launch_bounds__(64 * kStreamWaves) k_gemm_stream_c64(StreamGemmArgs g) {
  constexpr int NT = WN * 16, LN = ilog2<NT>::value, KT = 1 << LKT;
  constexpr int NTHR = 64 * kStreamWaves;
  constexpr int AE = 32 * KT / 64;   // A entries per lane per k tile
  __shared__ __attribute__((aligned(16))) float2 sB[kStreamBEntries];   // [k][column]
  __shared__ float sA[kStreamWaves][2][KT * 32];                        // per wave: Re, Im
  __shared__ int64_t t_ak[kStreamMaxK];
  __shared__ int64_t t_cn[NT];
  __shared__ int64_t t_am[32], t_cm[32];
  __shared__ Strides S;
  const StepArgs& p = g.s;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  {
    const int32_t* src = reinterpret_cast<const int32_t*>(p.sA_b);
    int32_t* dst = reinterpret_cast<int32_t*>(S.v);
    for (int i = tid; i < 9 * kMaxBits / 4; i += NTHR) dst[i] = src[i];
  }
  __syncthreads();
  const int nk = p.nk, K = 1 << nk;
  const int ntl = 1 << g.lnt;
  const int ctile = (int)(blockIdx.x >> 3) & (ntl - 1);
  const uint64_t group = (blockIdx.x & 7u) | ((uint64_t)(blockIdx.x >> (3 + g.lnt)) << 3);
  const uint64_t ngroups = gridDim.x >> g.lnt;
  const int64_t bbase = scatter_range((uint64_t)ctile << LN, S.Bn(), LN, p.nn);
  const int64_t cbase_n = scatter_range((uint64_t)ctile << LN, S.Cn(), LN, p.nn);
  for (int i = tid; i < K; i += NTHR) t_ak[i] = scatter(i, S.Ak(), nk);
  for (int i = tid; i < NT; i += NTHR) t_cn[i] = scatter(i, S.Cn(), LN);
  if (tid < 32) {
    t_am[tid] = scatter(tid, S.Am(), 5);
    t_cm[tid] = scatter(tid, S.Cm(), 5);
  }
  const float sb = p.conjB ? -1.f : 1.f;
  for (int e = tid; e < K * NT; e += NTHR) {
    const int n = e & (NT - 1), k = e >> LN;
    const float2 v = p.B[bbase + scatter(n, S.Bn(), LN) + scatter(k, S.Bk(), nk)];
    sB[e] = make_float2(v.x, sb * v.y);
  }
  __syncthreads();

  // per-lane entries of a band's k tile: in-band offset and LDS position
  uint32_t a_go[AE];
  int a_pos[AE];
#pragma unroll
  for (int r = 0; r < AE; ++r) {
    int mi, ki;
    split_bits(lane + 64 * r, g.a_mask, 5 + LKT, mi, ki);
    a_go[r] = (uint32_t)(t_am[mi] + t_ak[ki]);
    a_pos[r] = sa_pos(ki, mi);
  }
  const uint64_t bstride = ngroups * kStreamWaves;
  uint64_t band = group * kStreamWaves + wave;
  if (band >= g.nbands) return;   // no barrier follows
  const int nkt = K >> LKT;
  float* sa = &sA[wave][0][0];
  const float asign = p.conjA ? -1.f : 1.f;
  const int half = lane >> 5, par = lane & 1, l31 = lane & 31;
  const uint32_t bsign = (half & (par ^ 1)) ? 0x80000000u : 0u;
  float2 ra[AE];
  int64_t abase = scatter_range(band << 5, S.Am(), 5, p.nm);
#pragma unroll
  for (int r = 0; r < AE; ++r) ra[r] = p.A[abase + a_go[r]];
#pragma unroll
  for (int r = 0; r < AE; ++r) {
    sa[a_pos[r]] = ra[r].x;
    sa[KT * 32 + a_pos[r]] = asign * ra[r].y;
  }
  __builtin_amdgcn_wave_barrier();
  floatx16 acc[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) acc[j] = floatx16{};
  int kt = 0;
  for (;;) {
    // the next k tile (of this band or of the wave's next band) is loaded
    // while the matrix cores work on this one
    int kt2 = kt + 1;
    uint64_t band2 = band;
    int64_t abase2 = abase;
    if (kt2 == nkt) {
      kt2 = 0;
      band2 = band + bstride;
      if (band2 < g.nbands) abase2 = scatter_range(band2 << 5, S.Am(), 5, p.nm);
    }
    const bool more = band2 < g.nbands;
    if (more) {
      const int64_t b2 = abase2 + t_ak[kt2 << LKT];
#pragma unroll
      for (int r = 0; r < AE; ++r) ra[r] = p.A[b2 + a_go[r]];
    }
    // operands of k column kk: A entry (row l31, Re or Im by half) and the
    // lane's real-embedded B entry, the float (l31 ^ half) of complex row kk
    // of the block, negated for the lanes of -Im B (half 1, real column).
    // Each k column's operands are read from LDS while the matrix cores run
    // the previous column's products.
    const float* bk = reinterpret_cast<const float*>(sB) + (kt << LKT) * 2 * NT + (l31 ^ half);
    const float* ak = sa + half * KT * 32;
    float ax, bx[WN], ay, by[WN];
    auto operands = [&](int kk, float& a, float (&b)[WN]) {
      a = ak[sa_pos(kk, l31)];
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j] = bk[kk * 2 * NT + j * 32];
    };
    auto products = [&](float a, const float (&b)[WN]) {
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const float bv = __uint_as_float(__float_as_uint(b[j]) ^ bsign);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc[j], 0, 0, 0);
      }
    };
    operands(0, ax, bx);
#pragma unroll 1
    for (int kk = 0; kk < KT; kk += 2) {
      operands(kk + 1, ay, by);
      products(ax, bx);
      if (kk + 2 < KT) operands(kk + 2, ax, bx);
      products(ay, by);
    }
    if (kt == nkt - 1) {
      // the band's result: lane holds real column l31 of each 32 x 32 block,
      // rows 8 (r / 4) + 4 half + r % 4 of accumulator entry r
      const int64_t cb = scatter_range(band << 5, S.Cm(), 5, p.nm) + cbase_n;
      float* C = reinterpret_cast<float*>(p.C);
      if (p.accumulate) {
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          const int64_t on = cb + t_cn[j * 16 + (l31 >> 1)];
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            float* cf = C + 2 * (on + t_cm[8 * (r >> 2) + 4 * half + (r & 3)]) + par;
            *cf += acc[j][r];
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          const int64_t on = cb + t_cn[j * 16 + (l31 >> 1)];
#pragma unroll
          for (int r = 0; r < 16; ++r)
            C[2 * (on + t_cm[8 * (r >> 2) + 4 * half + (r & 3)]) + par] = acc[j][r];
        }
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[j] = floatx16{};
    }
    if (!more) break;
    // one wave's LDS operations run in order: the reads above have their
    // values before the buffer is overwritten, and the writes land before
    // the next tile's reads (the wave barriers keep the compiler from
    // moving them across)
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < AE; ++r) {
      sa[a_pos[r]] = ra[r].x;
      sa[KT * 32 + a_pos[r]] = asign * ra[r].y;
    }
    __builtin_amdgcn_wave_barrier();
    kt = kt2;
    band = band2;
    abase = abase2;
  }
}

}  // namespace tnk
