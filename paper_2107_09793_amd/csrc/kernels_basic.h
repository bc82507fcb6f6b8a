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
// row r = (m, b) keeps its 2^nk operand values in registers and produces its
// 2^nn outputs; the small operand is read through the cache.  Row offsets are
// split into the lane's low 8 bits (computed once) and the workgroup's high
// bits (uniform); every stride table is read at compile-time indices.
struct StreamArgs {
  const float2* A;
  const float2* B;
  float2* C;
  int32_t nrow;           // row bits: m bits then batch bits
  int32_t nbB;            // batch bits (the top nbB row bits), B's batch strides below
  int32_t conjA, conjB, accumulate;
  int8_t rowA[kMaxBits], rowC[kMaxBits];   // strides of row bit j in A and C
  int8_t bB[kMaxBits];                     // stride in B of batch bit j
  int8_t kA[4], kB[4], nB[4], nC[4];
};

template <int N>
__device__ __forceinline__ int64_t scatter_c(uint64_t idx, const int8_t* s, int lo, int hi) {
  int64_t off = 0;
#pragma unroll
  for (int j = 0; j < N; ++j)
    if (j >= lo && j < hi) off += (int64_t)((idx >> j) & 1ull) << s[j];
  return off;
}

template <int NK, int NN>
__global__ void __launch_bounds__(kBlock) k_stream(StreamArgs p) {
  constexpr int KN = (1 << NK) * (1 << NN);
  __shared__ float2 sB[KN];
  const int nrow = p.nrow;
  const uint64_t rows = 1ull << nrow;
  const int low = nrow < 8 ? nrow : 8;
  const int64_t la = scatter_c<8>(threadIdx.x, p.rowA, 0, low);
  const int64_t lc = scatter_c<8>(threadIdx.x, p.rowC, 0, low);
  int64_t kofA[1 << NK];
#pragma unroll
  for (int k = 0; k < (1 << NK); ++k) kofA[k] = scatter_c<NK>(k, p.kA, 0, NK);
  const int brow0 = nrow - p.nbB;   // first batch bit among the row bits
  // B lives in LDS when all rows of a workgroup pass share one batch value
  const bool shared_b = p.nbB == 0 || brow0 >= 8;
  int64_t staged = -1;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < rows;
       base += (uint64_t)gridDim.x * kBlock) {
    const int64_t ha = scatter_c<kMaxBits>(base, p.rowA, 8, nrow);   // uniform
    const int64_t hc = scatter_c<kMaxBits>(base, p.rowC, 8, nrow);
    if (shared_b) {
      const int64_t ob = p.nbB ? scatter_c<kMaxBits>(base >> brow0, p.bB, 0, p.nbB) : 0;
      if (ob != staged) {
        __syncthreads();
        for (int i = threadIdx.x; i < KN; i += kBlock) {
          const int k = i / (1 << NN), n = i % (1 << NN);
          sB[i] = maybe_conj(p.B[ob + scatter_c<NK>(k, p.kB, 0, NK) + scatter_c<NN>(n, p.nB, 0, NN)],
                             p.conjB);
        }
        __syncthreads();
        staged = ob;
      }
    }
    const uint64_t r = base + threadIdx.x;
    if (r >= rows) continue;
    const int64_t oa = la + ha, oc = lc + hc;
    float2 a[1 << NK];
#pragma unroll
    for (int k = 0; k < (1 << NK); ++k) a[k] = maybe_conj(p.A[oa + kofA[k]], p.conjA);
    const int64_t ob = shared_b ? 0 : scatter_c<kMaxBits>(r >> brow0, p.bB, 0, p.nbB);
#pragma unroll
    for (int n = 0; n < (1 << NN); ++n) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < (1 << NK); ++k) {
        float2 b = shared_b ? sB[k * (1 << NN) + n]
                            : maybe_conj(p.B[ob + scatter_c<NK>(k, p.kB, 0, NK) +
                                             scatter_c<NN>(n, p.nB, 0, NN)], p.conjB);
        cfma(acc, a[k], b);
      }
      const int64_t ocn = oc + scatter_c<NN>(n, p.nC, 0, NN);
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

// ---------------------------------------------------------------------------
// Adjoint of the slice sum: every resident slice of the root receives the
// output gradient of its output element.
struct RootGradArgs {
  const double2* grad_out;
  float2* dst;
  int32_t open_bits, res_bits, accumulate;
  int8_t s_open[kMaxBits], s_res[kMaxBits];
};

__global__ void __launch_bounds__(kBlock) k_root_grad(RootGradArgs p) {
  const uint64_t n = 1ull << (p.open_bits + p.res_bits);
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock) {
    uint64_t o = i & ((1ull << p.open_bits) - 1), r = i >> p.open_bits;
    int64_t off = scatter(o, p.s_open, p.open_bits) + scatter(r, p.s_res, p.res_bits);
    double2 g = p.grad_out[o];
    float2 v = make_float2((float)g.x, (float)g.y);
    if (p.accumulate) {
      float2 c = p.dst[off];
      v.x += c.x;
      v.y += c.y;
    }
    p.dst[off] = v;
  }
}

}  // namespace tnk
