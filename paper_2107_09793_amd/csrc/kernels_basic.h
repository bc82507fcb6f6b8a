// Vector-ALU contraction kernels, the bit permutation and the float64 slice
// sum.  All kernels use 256-thread workgroups (four 64-wide wavefronts).
#pragma once

#include "kernels_common.h"

namespace tnk {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Plain contraction: one thread per output element; the k sum walks k in
// Gray-code order so each step changes exactly one bit of k (one add to each
// operand offset).  Fixed order -> reproducible.
__global__ void __launch_bounds__(kBlock) k_simple(StepArgs p) {
  const uint64_t n_out = 1ull << (p.nb + p.nm + p.nn);
  const uint64_t K = 1ull << p.nk;
  for (uint64_t o = (uint64_t)blockIdx.x * kBlock + threadIdx.x; o < n_out;
       o += (uint64_t)gridDim.x * kBlock) {
    uint64_t n = o & ((1ull << p.nn) - 1);
    uint64_t m = (o >> p.nn) & ((1ull << p.nm) - 1);
    uint64_t b = o >> (p.nn + p.nm);
    int64_t oa = scatter(m, p.sA_m, p.nm) + scatter(b, p.sA_b, p.nb);
    int64_t ob = scatter(n, p.sB_n, p.nn) + scatter(b, p.sB_b, p.nb);
    int64_t oc = scatter(n, p.sC_n, p.nn) + scatter(m, p.sC_m, p.nm) + scatter(b, p.sC_b, p.nb);
    float2 acc = make_float2(0.f, 0.f);
    uint64_t g = 0;
    for (uint64_t i = 0; i < K; ++i) {
      if (i) {
        int j = __builtin_ctzll(i);
        uint64_t bit = 1ull << j;
        int64_t da = (int64_t)1 << p.sA_k[j], db = (int64_t)1 << p.sB_k[j];
        if (g & bit) { oa -= da; ob -= db; } else { oa += da; ob += db; }
        g ^= bit;
      }
      cfma(acc, maybe_conj(p.A[oa], p.conjA), maybe_conj(p.B[ob], p.conjB));
    }
    if (p.accumulate) {
      float2 c = p.C[oc];
      acc.x += c.x;
      acc.y += c.y;
    }
    p.C[oc] = acc;
  }
}

// ---------------------------------------------------------------------------
// Split-k, pass 1: workgroup (chunk, output) sums 2^chunk_log2 consecutive k
// values; threads stride by 256 and the workgroup reduces in a fixed tree.
__global__ void __launch_bounds__(kBlock) k_splitk_partial(StepArgs p) {
  __shared__ float2 red[kBlock];
  const uint64_t chunk = blockIdx.x;
  const uint64_t nchunk = gridDim.x;
  const uint64_t o = (uint64_t)blockIdx.y + ((uint64_t)blockIdx.z << 16);
  uint64_t n = o & ((1ull << p.nn) - 1);
  uint64_t m = (o >> p.nn) & ((1ull << p.nm) - 1);
  uint64_t b = o >> (p.nn + p.nm);
  const int cl = p.chunk_log2;
  int64_t oa = scatter(m, p.sA_m, p.nm) + scatter(b, p.sA_b, p.nb);
  int64_t ob = scatter(n, p.sB_n, p.nn) + scatter(b, p.sB_b, p.nb);
  oa += scatter_range(chunk << cl, p.sA_k, cl, p.nk) + scatter_range(threadIdx.x, p.sA_k, 0, 8);
  ob += scatter_range(chunk << cl, p.sB_k, cl, p.nk) + scatter_range(threadIdx.x, p.sB_k, 0, 8);
  float2 acc = make_float2(0.f, 0.f);
  const uint64_t iters = 1ull << (cl - 8);
  for (uint64_t i = 0; i < iters; ++i) {
    int64_t da = scatter_range(i << 8, p.sA_k, 8, cl);
    int64_t db = scatter_range(i << 8, p.sB_k, 8, cl);
    cfma(acc, maybe_conj(p.A[oa + da], p.conjA), maybe_conj(p.B[ob + db], p.conjB));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x].x += red[threadIdx.x + s].x;
      red[threadIdx.x].y += red[threadIdx.x + s].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) p.scratch[o * nchunk + chunk] = red[0];
}

// Split-k, pass 2: one thread per output sums its chunks in order, in float64.
__global__ void __launch_bounds__(kBlock) k_splitk_reduce(StepArgs p, int64_t nchunk) {
  const uint64_t n_out = 1ull << (p.nb + p.nm + p.nn);
  uint64_t o = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (o >= n_out) return;
  uint64_t n = o & ((1ull << p.nn) - 1);
  uint64_t m = (o >> p.nn) & ((1ull << p.nm) - 1);
  uint64_t b = o >> (p.nn + p.nm);
  int64_t oc = scatter(n, p.sC_n, p.nn) + scatter(m, p.sC_m, p.nm) + scatter(b, p.sC_b, p.nb);
  double re = 0.0, im = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) {
    float2 v = p.scratch[o * nchunk + c];
    re += v.x;
    im += v.y;
  }
  if (p.accumulate) {
    float2 c = p.C[oc];
    re += c.x;
    im += c.y;
  }
  p.C[oc] = make_float2((float)re, (float)im);
}

// ---------------------------------------------------------------------------
// Stream: few summed and few column bits (nk <= 4, nn <= 4).  One thread per
// row (b, m) keeps its 2^nk operand values in registers and produces its
// 2^nn outputs; the small operand is read through the cache.
template <int NK, int NN>
__global__ void __launch_bounds__(kBlock) k_stream(StepArgs p) {
  const uint64_t rows = 1ull << (p.nb + p.nm);
  for (uint64_t r = (uint64_t)blockIdx.x * kBlock + threadIdx.x; r < rows;
       r += (uint64_t)gridDim.x * kBlock) {
    uint64_t m = r & ((1ull << p.nm) - 1);
    uint64_t b = r >> p.nm;
    int64_t oa = scatter(m, p.sA_m, p.nm) + scatter(b, p.sA_b, p.nb);
    int64_t ob = scatter(b, p.sB_b, p.nb);
    int64_t oc = scatter(m, p.sC_m, p.nm) + scatter(b, p.sC_b, p.nb);
    float2 a[1 << NK];
#pragma unroll
    for (int k = 0; k < (1 << NK); ++k)
      a[k] = maybe_conj(p.A[oa + scatter(k, p.sA_k, NK)], p.conjA);
#pragma unroll
    for (int n = 0; n < (1 << NN); ++n) {
      int64_t obn = ob + scatter(n, p.sB_n, NN);
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < (1 << NK); ++k)
        cfma(acc, a[k], maybe_conj(p.B[obn + scatter(k, p.sB_k, NK)], p.conjB));
      int64_t ocn = oc + scatter(n, p.sC_n, NN);
      if (p.accumulate) {
        float2 c = p.C[ocn];
        acc.x += c.x;
        acc.y += c.y;
      }
      p.C[ocn] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Bit permutation (plain version: one element per thread).
struct PermArgs {
  const float2* in;
  float2* out;
  int32_t nbits;
  int8_t sin[kMaxBits], sout[kMaxBits];
};

__global__ void __launch_bounds__(kBlock) k_permute_plain(PermArgs p) {
  const uint64_t n = 1ull << p.nbits;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock)
    p.out[scatter(i, p.sout, p.nbits)] = p.in[scatter(i, p.sin, p.nbits)];
}

// ---------------------------------------------------------------------------
// float64 fill (output initialisation; a kernel, not a memset, so the call
// sequence can be captured in a graph).
__global__ void __launch_bounds__(kBlock) k_fill_c128(double2* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    out[i] = make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------------------
// Slice sum (Eq. sliced_sum): the root holds the partial results of the
// resident slices as bits; each output element adds them in float64 in a
// fixed order.  mode 0: out[o] += sum over the selected resident slices;
// mode 1: out[row * n_out + o] = slice value.
constexpr int kMaxSel = 240;
struct SumArgs {
  const float2* root;
  double2* out;
  int32_t open_bits, res_bits;
  int32_t mode;
  int32_t n_sel;          // -1: every resident slice; else entries of sel_r / sel_row
  int64_t row_base;       // mode 1, all slices: row of resident slice r is row_base + rowbit(r)
  int8_t s_open[kMaxBits], s_res[kMaxBits];
  int8_t res_slicebit[kMaxBits];
  int32_t sel_r[kMaxSel];
  int32_t sel_row[kMaxSel];
};

__global__ void __launch_bounds__(kBlock) k_slice_sum(SumArgs p) {
  const uint64_t n_out = 1ull << p.open_bits;
  uint64_t o = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (o >= n_out) return;
  int64_t oo = scatter(o, p.s_open, p.open_bits);
  if (p.mode == 0) {
    double2 acc = p.out[o];
    if (p.n_sel < 0) {
      uint64_t R = 1ull << p.res_bits;
      for (uint64_t r = 0; r < R; ++r) {
        float2 v = p.root[oo + scatter(r, p.s_res, p.res_bits)];
        acc.x += (double)v.x;
        acc.y += (double)v.y;
      }
    } else {
      for (int i = 0; i < p.n_sel; ++i) {
        float2 v = p.root[oo + scatter((uint64_t)p.sel_r[i], p.s_res, p.res_bits)];
        acc.x += (double)v.x;
        acc.y += (double)v.y;
      }
    }
    p.out[o] = acc;
  } else {
    if (p.n_sel < 0) {
      uint64_t R = 1ull << p.res_bits;
      for (uint64_t r = 0; r < R; ++r) {
        float2 v = p.root[oo + scatter(r, p.s_res, p.res_bits)];
        int64_t row = p.row_base;
        for (int j = 0; j < p.res_bits; ++j) row += (int64_t)((r >> j) & 1) << p.res_slicebit[j];
        p.out[row * (int64_t)n_out + o] = make_double2(v.x, v.y);
      }
    } else {
      for (int i = 0; i < p.n_sel; ++i) {
        float2 v = p.root[oo + scatter((uint64_t)p.sel_r[i], p.s_res, p.res_bits)];
        p.out[(int64_t)p.sel_row[i] * (int64_t)n_out + o] = make_double2(v.x, v.y);
      }
    }
  }
}

}  // namespace tnk
