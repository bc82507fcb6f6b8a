// Skinny GEMM steps as a stream over row bands (complex64 on FP32 MFMA and
// split-BF16 on BF16 MFMA).
//
// Shapes with few columns and summed values against many rows (a column tile
// of at most 128 complex columns times all k within the 64 KiB B buffer,
// 2^10 - 2^40 rows), which one-tile-per-workgroup kernels run far below the
// matrix-core and memory rates: every tile would restage B, rebuild its
// offset tables and drain its pipeline.  Here a workgroup of 8 waves (2 per
// SIMD, one workgroup per CU) stages the B block of its column tile -- every
// k -- in LDS once, and each wave then walks its own 32-row bands: per band
// it streams A through a wave-private LDS buffer in k tiles (the next tiles'
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
// Arithmetic is the real embedding of the tile kernels, with the product's
// 32 x 32 real blocks (16 complex columns) in the same accumulator layout in
// both precisions:
// * complex64: one v_mfma_f32_32x32x2f32 per complex k (lanes 0-31: Re A
//   and the first row of B's 2x2 block, lanes 32-63: Im A and the second);
// * split-BF16: x = hi + lo, hi = bf16(x), lo = bf16(x - hi) (round to
//   nearest even); three v_mfma_f32_32x32x16_bf16 (hi hi, hi lo, lo hi) per 8
//   complex k, A rows and the embedded B columns as interleaved (Re, Im)
//   pairs.
#pragma once

#include "kernels_gemm.h"

namespace tnk {

constexpr int kStreamWaves = 8;             // waves per workgroup (2 per SIMD)
constexpr int kStreamBBytes = 64 * 1024;    // staged B block
constexpr int kStreamMaxK = 1 << 9;

struct StreamGemmArgs {
  StepArgs s;
  // enumeration of a band's k tile (5 row bits, then the k tile's bits):
  // bit j set = row bit, in the order of tile_mask (ascending A stride)
  uint32_t a_mask;
  int32_t lnt;       // log2 column tiles
  int32_t lgroups;   // log2 band groups per column tile (grid = 2^(lgroups + lnt))
  uint64_t nbands;   // 32-row bands: 2^(nm - 5)
};

// Result stores of the real-embedded layout (both precisions): lane holds
// real column l31 of each 32 x 32 block j (Re, par 0, or Im, par 1, of
// complex column 16 j + l31 / 2), rows 8 (q / 4) + 4 half + q % 4 of
// accumulator entry q.  C += result when accumulating.
template <int WN>
__device__ __forceinline__ void store_embedded(float2* C2, int64_t cbase, const int64_t* t_cn,
                                               const int64_t* t_cm, int lane, int accumulate,
                                               floatx16 (&acc)[WN]) {
  const int half = lane >> 5, par = lane & 1, l31 = lane & 31;
  float* C = reinterpret_cast<float*>(C2);
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int64_t on = cbase + t_cn[j * 16 + (l31 >> 1)];
    auto at = [&](int q) -> float& {
      return C[2 * (on + t_cm[8 * (q >> 2) + 4 * half + (q & 3)]) + par];
    };
    if (accumulate) {
#pragma unroll
      for (int q0 = 0; q0 < 16; q0 += 4) {
        float old[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) old[q] = at(q0 + q);
#pragma unroll
        for (int q = 0; q < 4; ++q) at(q0 + q) = old[q] + acc[j][q0 + q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) at(q) = acc[j][q];
    }
  }
}

// ---------------------------------------------------------------------------
// complex64 operands.  A k tile in LDS: the Re plane (KT x 32 floats, the 32
// rows of one k consecutive and XOR-swizzled by k so that staging writes of
// interleaved (row, k) enumerations spread over the banks), 32 floats of
// padding so that the Im plane read by lanes 32-63 sits on the other half of
// the banks, then the Im plane.  B: complex [k][column].
template <int KT>
struct StreamC64 {
  static constexpr int kIm = KT * 32 + 32;
  static constexpr int kWaveBytes = (kIm + KT * 32) * 4;
  template <int WN>
  static constexpr int kAcc = WN;   // one 32 x 32 real block per 16 columns
  template <int WN>
  __device__ static void store(float2* C, int64_t cbase, const int64_t* t_cn, const int64_t* t_cm,
                               int lane, int accumulate, floatx16 (&acc)[WN]) {
    store_embedded<WN>(C, cbase, t_cn, t_cm, lane, accumulate, acc);
  }

  __device__ static int a_pos(int ki, int mi) { return ki * 32 + (mi ^ ((ki << 2) & 31)); }
  __device__ static void put_a(char* sa, int pos, float2 v) {
    float* f = reinterpret_cast<float*>(sa);
    f[pos] = v.x;
    f[kIm + pos] = v.y;
  }
  template <int NT>
  __device__ static void put_b(char* sb, int k, int n, float2 v, int) {
    reinterpret_cast<float2*>(sb)[k * NT + n] = v;
  }
  // The k tile's products.  Operands of k column kk: the A entry (row l31,
  // Re or Im by half) and the lane's real-embedded B entry, the float
  // (l31 ^ half) of complex row kk, negated for the lanes of -Im B (half 1,
  // real column); each column's operands are read while the previous
  // column's products run.
  template <int WN, int NT>
  __device__ static void tile(const char* sa, const char* sb, int kt, int lane, int,
                              floatx16 (&acc)[WN]) {
    const int half = lane >> 5, par = lane & 1, l31 = lane & 31;
    const uint32_t bsign = (half & (par ^ 1)) ? 0x80000000u : 0u;
    const float* bk = reinterpret_cast<const float*>(sb) + kt * KT * 2 * NT + (l31 ^ half);
    const float* ak = reinterpret_cast<const float*>(sa) + half * kIm;
    float ax, bx[WN], ay, by[WN];
    auto operands = [&](int kk, float& a, float (&b)[WN]) {
      a = ak[a_pos(kk, l31)];
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
  }
};

// ---------------------------------------------------------------------------
// split-BF16 operands.  A k tile in LDS: the hi plane, then the lo plane,
// each 32 rows of 2 KT bf16 (the (Re, Im) pairs of the row's KT complex k);
// the 16-byte chunks of a row are XOR-swizzled by row so that the 16 lanes of
// one ds_read_b128 phase hit distinct banks.  B: the embedded operand as it
// is read, [hi | lo][k / 4][real column][4 packed pairs]: real column 2n
// holds (Re B, -Im B), column 2n + 1 holds (Im B, Re B), so a lane's 8 bf16
// (4 complex k of its column) are one 16-byte read.
template <int KT>
struct StreamSB16 {
  static constexpr int kRowBytes = 4 * KT;
  static constexpr int kChunks = kRowBytes / 16;
  static constexpr int kPlane = 32 * kRowBytes;
  static constexpr int kWaveBytes = 2 * kPlane;
  static constexpr int kSwzShift = KT == 32 ? 1 : 2;   // rows sharing banks: 256 B / row bytes
  static_assert(KT == 16 || KT == 32, "split-BF16 stream tiles walk k by 16 or 32");
  template <int WN>
  static constexpr int kAcc = WN;
  template <int WN>
  __device__ static void store(float2* C, int64_t cbase, const int64_t* t_cn, const int64_t* t_cm,
                               int lane, int accumulate, floatx16 (&acc)[WN]) {
    store_embedded<WN>(C, cbase, t_cn, t_cm, lane, accumulate, acc);
  }

  __device__ static int chunk(int row, int q) { return q ^ ((row >> kSwzShift) & (kChunks - 1)); }
  __device__ static int a_pos(int ki, int mi) {
    return mi * kRowBytes + chunk(mi, ki >> 2) * 16 + (ki & 3) * 4;
  }
  __device__ static void put_a(char* sa, int pos, float2 v) {
    uint32_t hi, lo;
    split_pair(v.x, v.y, hi, lo);
    *reinterpret_cast<uint32_t*>(sa + pos) = hi;
    *reinterpret_cast<uint32_t*>(sa + kPlane + pos) = lo;
  }
  template <int NT>
  __device__ static void put_b(char* sb, int k, int n, float2 v, int K) {
    uint32_t hi, lo;
    split_pair(v.x, v.y, hi, lo);   // low half Re B, high half Im B
    const int plane = K * NT * 8;   // bytes of one plane
    char* b0 = sb + ((k >> 2) * 2 * NT + 2 * n) * 16 + (k & 3) * 4;
    *reinterpret_cast<uint32_t*>(b0) = hi ^ 0x80000000u;
    *reinterpret_cast<uint32_t*>(b0 + 16) = (hi >> 16) | (hi << 16);
    *reinterpret_cast<uint32_t*>(b0 + plane) = lo ^ 0x80000000u;
    *reinterpret_cast<uint32_t*>(b0 + plane + 16) = (lo >> 16) | (lo << 16);
  }
  template <int WN, int NT>
  __device__ static void tile(const char* sa, const char* sb, int kt, int lane, int K,
                              floatx16 (&acc)[WN]) {
    const int half = lane >> 5, l31 = lane & 31;
    const int plane = K * NT * 8;
    const char* arow = sa + l31 * kRowBytes;
#pragma unroll 2
    for (int s = 0; s < KT / 8; ++s) {
      const int q = 2 * s + half;   // this lane's 4 complex k: chunk q of the row
      const bf16x8_t ah = *reinterpret_cast<const bf16x8_t*>(arow + chunk(l31, q) * 16);
      const bf16x8_t al = *reinterpret_cast<const bf16x8_t*>(arow + kPlane + chunk(l31, q) * 16);
      const char* bq = sb + ((kt * (KT / 4) + q) * 2 * NT + l31) * 16;
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const bf16x8_t bh = *reinterpret_cast<const bf16x8_t*>(bq + j * 32 * 16);
        const bf16x8_t bl = *reinterpret_cast<const bf16x8_t*>(bq + plane + j * 32 * 16);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[j], 0, 0, 0);
      }
    }
  }
};

// ---------------------------------------------------------------------------
// complex64 with three real products per complex product (Gauss):
// T1 = Re A Re B, T2 = Im A Im B, T3 = (Re A + Im A)(Re B + Im B) summed over
// k, then Re C = T1 - T2 and Im C = T3 - T1 - T2: three v_mfma_f32_32x32x2f32
// per two complex k and 32 complex columns, where the real embedding takes
// four.  The MFMA columns are complex columns (blocks of 32), so WN (16-column
// units) is even and block b holds accumulators 3 b .. 3 b + 2.  A k tile in
// LDS: the Re and Im planes, each [k / 2][row][k % 2] (the two k of one MFMA
// side by side, so the two half-waves read the even and the odd banks); the
// sum Re A + Im A is formed on reading.  B: the planes Re B, Im B and
// Re B + Im B, each [k / 2][column][k % 2].
template <int KT>
struct StreamC64G {
  static constexpr int kPlane = KT * 32;   // floats of one A plane
  static constexpr int kWaveBytes = 2 * kPlane * 4;
  template <int WN>
  static constexpr int kAcc = 3 * (WN / 2);

  __device__ static int a_pos(int ki, int mi) { return ((ki >> 1) * 32 + mi) * 2 + (ki & 1); }
  __device__ static void put_a(char* sa, int pos, float2 v) {
    float* f = reinterpret_cast<float*>(sa);
    f[pos] = v.x;
    f[kPlane + pos] = v.y;
  }
  template <int NT>
  __device__ static void put_b(char* sb, int k, int n, float2 v, int K) {
    float* f = reinterpret_cast<float*>(sb);
    const int plane = K * NT;
    const int pos = ((k >> 1) * NT + n) * 2 + (k & 1);
    f[pos] = v.x;
    f[plane + pos] = v.y;
    f[2 * plane + pos] = v.x + v.y;
  }
  template <int WN, int NT>
  __device__ static void tile(const char* sa, const char* sb, int kt, int lane, int K,
                              floatx16 (&acc)[kAcc<WN>]) {
    constexpr int NB = WN / 2;
    const int half = lane >> 5, l31 = lane & 31;
    const int plane = K * NT;
    const float* ar = reinterpret_cast<const float*>(sa) + l31 * 2 + half;
    const float* bp = reinterpret_cast<const float*>(sb) + (kt * (KT / 2) * NT + l31) * 2 + half;
    // operands of k pair k2: Re A, Im A, and per block Re B, Im B, Re B + Im B;
    // each pair's operands are read while the previous pair's products run
    float ax[2], bx[3 * NB], ay[2], by[3 * NB];
    auto operands = [&](int k2, float (&a)[2], float (&b)[3 * NB]) {
      a[0] = ar[k2 * 64];
      a[1] = ar[kPlane + k2 * 64];
#pragma unroll
      for (int bl = 0; bl < NB; ++bl) {
        const float* bb = bp + (k2 * NT + bl * 32) * 2;
        b[3 * bl] = bb[0];
        b[3 * bl + 1] = bb[plane];
        b[3 * bl + 2] = bb[2 * plane];
      }
    };
    auto products = [&](const float (&a)[2], const float (&b)[3 * NB]) {
      const float a_s = a[0] + a[1];
#pragma unroll
      for (int bl = 0; bl < NB; ++bl) {
        acc[3 * bl] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], b[3 * bl], acc[3 * bl], 0, 0, 0);
        acc[3 * bl + 1] =
            __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], b[3 * bl + 1], acc[3 * bl + 1], 0, 0, 0);
        acc[3 * bl + 2] =
            __builtin_amdgcn_mfma_f32_32x32x2f32(a_s, b[3 * bl + 2], acc[3 * bl + 2], 0, 0, 0);
      }
    };
    operands(0, ax, bx);
#pragma unroll 1
    for (int k2 = 0; k2 < KT / 2; k2 += 2) {
      operands(k2 + 1, ay, by);
      products(ax, bx);
      if (k2 + 2 < KT / 2) operands(k2 + 2, ax, bx);
      products(ay, by);
    }
  }
  // lane holds complex column 32 b + l31 of block b, rows 8 (q / 4) + 4 half
  // + q % 4 of entry q of its three accumulators
  template <int WN>
  __device__ static void store(float2* C, int64_t cbase, const int64_t* t_cn, const int64_t* t_cm,
                               int lane, int accumulate, floatx16 (&acc)[kAcc<WN>]) {
    constexpr int NB = WN / 2;
    const int half = lane >> 5, l31 = lane & 31;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int64_t on = cbase + t_cn[b * 32 + l31];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const float t1 = acc[3 * b][q], t2 = acc[3 * b + 1][q], t3 = acc[3 * b + 2][q];
        float2 v = make_float2(t1 - t2, t3 - t1 - t2);
        float2* cp = C + on + t_cm[8 * (q >> 2) + 4 * half + (q & 3)];
        if (accumulate) {
          const float2 o = *cp;
          v = make_float2(o.x + v.x, o.y + v.y);
        }
        *cp = v;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// The stream kernel.  P: operand policy (StreamC64, StreamC64G, StreamSB16); WN: 16-column
// blocks per column tile; LKT: log2 complex k per k tile; DEPTH: k tiles in
// flight per wave besides the one in LDS (1 or 2).
template <template <int> class P, int WN, int LKT, int DEPTH>
__global__ void __launch_bounds__(64 * kStreamWaves) k_gemm_stream(StreamGemmArgs g) {
  constexpr int NT = WN * 16, LN = ilog2<NT>::value, KT = 1 << LKT;
  constexpr int NTHR = 64 * kStreamWaves;
  constexpr int AE = 32 * KT / 64;   // A entries per lane per k tile
  using Pol = P<KT>;
  __shared__ __attribute__((aligned(16))) char sB[kStreamBBytes];
  __shared__ __attribute__((aligned(16))) char sA[kStreamWaves][Pol::kWaveBytes];
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
  const int64_t bbase = scatter_range((uint64_t)ctile << LN, S.Bn(), LN, p.nn);
  const int64_t cbase_n = scatter_range((uint64_t)ctile << LN, S.Cn(), LN, p.nn);
  for (int i = tid; i < K; i += NTHR) t_ak[i] = scatter(i, S.Ak(), nk);
  for (int i = tid; i < NT; i += NTHR) t_cn[i] = scatter(i, S.Cn(), LN);
  if (tid < 32) {
    t_am[tid] = scatter(tid, S.Am(), 5);
    t_cm[tid] = scatter(tid, S.Cm(), 5);
  }
  const float sbs = p.conjB ? -1.f : 1.f;
  for (int e = tid; e < K * NT; e += NTHR) {
    const int n = e & (NT - 1), k = e >> LN;
    const float2 v = p.B[bbase + scatter(n, S.Bn(), LN) + scatter(k, S.Bk(), nk)];
    Pol::template put_b<NT>(sB, k, n, make_float2(v.x, sbs * v.y), K);
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
    a_pos[r] = Pol::a_pos(ki, mi);
  }
  // The wave's bands are band0 + i 2^lb (the groups' waves interleave), i in
  // Gray-code order: consecutive bands differ in one bit of i, so the next
  // band's base offsets are the current ones plus or minus one stride.  A
  // unit is one k tile of one band; the wave runs nkt units per band.
  const int lb = g.lgroups + 3;
  const uint64_t band0 = (group << 3) + wave;
  if (band0 >= g.nbands) return;   // no barrier follows
  const uint64_t nbw = g.nbands > (1ull << lb) ? g.nbands >> lb : 1;   // bands of this wave
  const int nkt = K >> LKT;
  const uint64_t nunits = nbw * (uint64_t)nkt;
  char* sa = &sA[wave][0];
  const float asign = p.conjA ? -1.f : 1.f;

  struct Walk {   // position in the wave's units and the base offset there
    int kt;
    uint64_t bi, gray;
    int64_t base;
  };
  auto advance = [&](Walk& w, const int8_t* strides) {
    if (++w.kt == nkt) {
      w.kt = 0;
      if (++w.bi < nbw) {
        const int j = __builtin_ctzll(w.bi);
        const uint64_t bit = 1ull << j;
        const int64_t d = (int64_t)1 << strides[5 + lb + j];   // row bit that changes
        w.base += (w.gray & bit) ? -d : d;
        w.gray ^= bit;
      }
    }
  };
  Walk wl{0, 0, 0, scatter_range(band0 << 5, S.Am(), 5, p.nm)};             // next load
  Walk wc{0, 0, 0, scatter_range(band0 << 5, S.Cm(), 5, p.nm) + cbase_n};   // computed
  uint64_t ul = 0, uc = 0;   // units loaded, units computed
  float2 rx[AE], ry[AE];
  auto load = [&](float2 (&r)[AE]) {
    const int64_t b = wl.base + t_ak[wl.kt << LKT];
#pragma unroll
    for (int i = 0; i < AE; ++i) r[i] = p.A[b + a_go[i]];
    advance(wl, S.Am());
    ++ul;
  };
  // One wave's LDS operations run in order: the reads of the previous tile
  // have their values before the buffer is overwritten, and the writes land
  // before the next tile's reads (the wave barriers keep the compiler from
  // moving them across).
  auto stage = [&](const float2 (&r)[AE]) {
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < AE; ++i) Pol::put_a(sa, a_pos[i], make_float2(r[i].x, asign * r[i].y));
    __builtin_amdgcn_wave_barrier();
  };
  load(rx);
  stage(rx);
  if (ul < nunits) load(rx);
  if (DEPTH == 2 && ul < nunits) load(ry);

  constexpr int NACC = Pol::template kAcc<WN>;
  floatx16 acc[NACC];
#pragma unroll
  for (int j = 0; j < NACC; ++j) acc[j] = floatx16{};
  // One unit: the matrix-core work on the staged tile, then the next tile
  // (held in slot r) into LDS and slot r refilled with the unit DEPTH + 1
  // ahead, then -- at the end of a band -- the result stores.  Staging before
  // the stores matters: vector memory operations retire in order, so a wait
  // for loads issued before the stores would wait for the stores as well.
  auto unit = [&](float2 (&r)[AE]) -> bool {
    Pol::template tile<WN, NT>(sa, sB, wc.kt, lane, K, acc);
    const bool more = uc + 1 < nunits;
    if (more) stage(r);
    if (ul < nunits) load(r);
    if (wc.kt == nkt - 1) {
      Pol::template store<WN>(p.C, wc.base, t_cn, t_cm, lane, p.accumulate, acc);
#pragma unroll
      for (int q = 0; q < NACC; ++q) acc[q] = floatx16{};
    }
    advance(wc, S.Cm());
    ++uc;
    return more;
  };
  if constexpr (DEPTH == 2) {
    for (;;) {
      if (!unit(rx)) break;
      if (!unit(ry)) break;
    }
  } else {
    while (unit(rx)) {
    }
  }
}

}  // namespace tnk
