// Vector-ALU contraction kernels, the bit permutation and the float64 slice
// sum.  All kernels use 256-thread workgroups (four 64-wide wavefronts).
#pragma once

#include "kernels_common.h"

namespace tnk {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Plain contraction: one thread per output element, k summed in increasing
// order (the same multiply-add sequence as the stream kernel and the
// persistent executor, so the three agree bit for bit).
__global__ void __launch_bounds__(kBlock) k_simple(StepArgs p) {
  const uint64_t n_out = 1ull << (p.nb + p.nm + p.nn);
  for (uint64_t o = (uint64_t)blockIdx.x * kBlock + threadIdx.x; o < n_out;
       o += (uint64_t)gridDim.x * kBlock) {
    uint64_t n = o & ((1ull << p.nn) - 1);
    uint64_t m = (o >> p.nn) & ((1ull << p.nm) - 1);
    uint64_t b = o >> (p.nn + p.nm);
    int64_t oa = scatter(m, p.sA_m, p.nm) + scatter(b, p.sA_b, p.nb);
    int64_t ob = scatter(n, p.sB_n, p.nn) + scatter(b, p.sB_b, p.nb);
    int64_t oc = scatter(n, p.sC_n, p.nn) + scatter(m, p.sC_m, p.nm) + scatter(b, p.sC_b, p.nb);
    float2 acc = dot_k(p.A, oa, p.sA_k, p.conjA, p.B, ob, p.sB_k, p.conjB, p.nk);
    if (p.accumulate) {
      float2 c = p.C[oc];
      acc.x += c.x;
      acc.y += c.y;
    }
    p.C[oc] = acc;
  }
}

// ---------------------------------------------------------------------------
// A batch of tiny steps (consecutive in the schedule, each at most 2^13
// multiply-adds and 2^11 outputs) in one launch of one workgroup.  The steps
// come by level (a step's operands are produced by steps of lower levels or
// before the batch, and no step writes what another step of its level reads
// or writes); the outputs of all steps of one level are spread over
// the workgroup's 1024 threads, each formed as k_simple forms it, and a
// workgroup barrier separates the levels (a level's results are visible to
// every wave of the workgroup once it is passed).  No workgroup waits on
// another, and the descriptors travel in the kernel arguments.
constexpr int kTinyMax = 20;
constexpr int kTinyClassBits = 14;
// threads of the batch's workgroup: a step's outputs (at most 2^11) take one
// or two passes, and a level's several steps spread over 16 waves
constexpr int kTinyBlock = 1024;
struct TinyStep {
  const float2* A;
  const float2* B;
  float2* C;
  int8_t nb, nm, nn, nk, level;
  int8_t conjA, conjB, accumulate;   // as in StepArgs
  int8_t sA_b[kTinyClassBits], sB_b[kTinyClassBits], sC_b[kTinyClassBits];
  int8_t sA_m[kTinyClassBits], sC_m[kTinyClassBits];
  int8_t sB_n[kTinyClassBits], sC_n[kTinyClassBits];
  int8_t sA_k[kTinyClassBits], sB_k[kTinyClassBits];
};
struct TinyArgs {
  int32_t n;
  TinyStep st[kTinyMax];
};
static_assert(sizeof(TinyArgs) <= 4000, "kernel arguments");

static_assert(sizeof(TinyArgs) % 4 == 0, "descriptor copy in 32-bit words");

__global__ void __launch_bounds__(kTinyBlock) k_tiny_run(TinyArgs args) {
  // the descriptors go to LDS once: every output of every level looks up its
  // step's sizes and strides, and from the kernel arguments (indexed per
  // thread) each lookup would be a dependent memory round trip
  __shared__ TinyArgs a;
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&args);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&a);
    for (int i = threadIdx.x; i < (int)(sizeof(TinyArgs) / 4); i += kTinyBlock) dst[i] = src[i];
  }
  __syncthreads();
  int s = 0;
  while (s < a.n) {
    const int lv = a.st[s].level;
    int e = s + 1;
    while (e < a.n && a.st[e].level == lv) ++e;
    uint32_t total = 0;
    for (int j = s; j < e; ++j) total += 1u << (a.st[j].nb + a.st[j].nm + a.st[j].nn);
    for (uint32_t f = threadIdx.x; f < total; f += kTinyBlock) {
      int j = s;
      uint32_t o = f;
      while (o >= (1u << (a.st[j].nb + a.st[j].nm + a.st[j].nn))) {
        o -= 1u << (a.st[j].nb + a.st[j].nm + a.st[j].nn);
        ++j;
      }
      const TinyStep& T = a.st[j];
      const int nb = T.nb, nm = T.nm, nn = T.nn, nk = T.nk;
      const uint32_t n = o & ((1u << nn) - 1);
      const uint32_t m = (o >> nn) & ((1u << nm) - 1);
      const uint32_t b = o >> (nn + nm);
      const int64_t oa = scatter(m, T.sA_m, nm) + scatter(b, T.sA_b, nb);
      const int64_t ob = scatter(n, T.sB_n, nn) + scatter(b, T.sB_b, nb);
      const int64_t oc = scatter(n, T.sC_n, nn) + scatter(m, T.sC_m, nm) + scatter(b, T.sC_b, nb);
      float2 acc = dot_k(T.A, oa, T.sA_k, T.conjA, T.B, ob, T.sB_k, T.conjB, nk);
      if (T.accumulate) {
        const float2 c = T.C[oc];
        acc.x += c.x;
        acc.y += c.y;
      }
      T.C[oc] = acc;
    }
    __syncthreads();
    s = e;
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

// Offset of bits [lo, hi) of idx, as a plain loop: with a uniform idx the
// compiler keeps it in scalar registers.
__device__ __forceinline__ int64_t scatter_loop(uint64_t idx, const int8_t* s, int lo, int hi) {
  int64_t off = 0;
#pragma unroll 1
  for (int j = lo; j < hi; ++j) off += (int64_t)((idx >> j) & 1ull) << s[j];
  return off;
}

template <int N>
__device__ __forceinline__ int64_t scatter_c(uint64_t idx, const int8_t* s, int lo, int hi) {
  int64_t off = 0;
#pragma unroll
  for (int j = 0; j < N; ++j)
    if (j >= lo && j < hi) off += (int64_t)((idx >> j) & 1ull) << s[j];
  return off;
}

// SHB: every row of a workgroup pass shares one batch value, so the small
// operand is staged in LDS once per pass and read by broadcast; otherwise it
// is read through the cache per row.
template <int NK, int NN, bool SHB>
__global__ void __launch_bounds__(kBlock) k_stream(StreamArgs p) {
  constexpr int KN = (1 << NK) * (1 << NN);
  __shared__ float2 sB[SHB ? KN : 1];
  const int nrow = p.nrow;
  const uint64_t rows = 1ull << nrow;
  const int low = nrow < 8 ? nrow : 8;
  const int64_t la = scatter_c<8>(threadIdx.x, p.rowA, 0, low);
  const int64_t lc = scatter_c<8>(threadIdx.x, p.rowC, 0, low);
  const int brow0 = nrow - p.nbB;   // first batch bit among the row bits
  int64_t staged = -1;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < rows;
       base += (uint64_t)gridDim.x * kBlock) {
    const int64_t ha = scatter_loop(base, p.rowA, 8, nrow);   // uniform
    const int64_t hc = scatter_loop(base, p.rowC, 8, nrow);
    if (SHB) {
      const int64_t ob = p.nbB ? scatter_loop(base >> brow0, p.bB, 0, p.nbB) : 0;
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
    const float2* Ar = p.A + (la + ha);
    float2* Cr = p.C + (lc + hc);
    float2 a[1 << NK];
#pragma unroll
    for (int k = 0; k < (1 << NK); ++k)
      a[k] = maybe_conj(Ar[scatter_c<NK>(k, p.kA, 0, NK)], p.conjA);
    const float2* Br = SHB ? nullptr : p.B + scatter_loop(r >> brow0, p.bB, 0, p.nbB);
#pragma unroll
    for (int n = 0; n < (1 << NN); ++n) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < (1 << NK); ++k) {
        float2 b;
        if (SHB) {
          b = sB[k * (1 << NN) + n];
        } else {
          b = maybe_conj(Br[scatter_c<NK>(k, p.kB, 0, NK) + scatter_c<NN>(n, p.nB, 0, NN)],
                         p.conjB);
        }
        cfma(acc, a[k], b);
      }
      float2* cp = Cr + scatter_c<NN>(n, p.nC, 0, NN);
      if (p.accumulate) {
        float2 c = *cp;
        acc.x += c.x;
        acc.y += c.y;
      }
      *cp = acc;
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
// Bit permutation through an LDS tile (the transpose of the TTGT
// decomposition, Sec. 3.1, for tensors whose dims are all 2).  The tile holds
// the 2^TB elements spanned by TB index bits: the bits of the lowest input
// strides (contiguous reads), the bits of the lowest output strides
// (contiguous writes) and, if fewer, further bits.  A workgroup reads its tile
// in input order into LDS, then writes it in output order.  LDS positions are
// XOR-swizzled (low half ^= high half) so the strided LDS reads of the write
// phase spread over banks.  All offsets are XOR/OR-linear in the index bits,
// so each thread splits them into a per-thread part (its 8 low bits) and a
// per-element part, the latter summed from the strides of the element
// number's set bits (compile-time) rather than held per element.  The 2^12
// tile is the kernel's only LDS (the tile-index strides come from the kernel
// arguments): 32 KiB, so five workgroups share a CU, and the registers fit
// the five (20 waves per CU in flight).
struct PermTileArgs {
  const float2* in;
  float2* out;
  int32_t tbits;            // bits in the tile (= the kernel's TB)
  int32_t rbits;            // bits enumerating tiles
  int32_t half;             // swizzle width
  int8_t rin[16];           // input log2 stride of tile position p (read order = LDS order)
  int8_t wout[16], wpos[16];  // write order: output log2 stride and LDS position
  int8_t tin[kMaxBits], tout[kMaxBits];  // tile-index bits: input / output log2 strides
};

__device__ __forceinline__ uint32_t perm_swz(uint32_t x, int half) {
  return x ^ ((x >> half) & ((1u << half) - 1u));
}

template <int TB>
__global__ void __launch_bounds__(kBlock) k_permute_tile(PermTileArgs p) {
  static_assert(TB >= 8 && TB <= 16, "tile of 256 threads x E elements");
  constexpr int E = 1 << (TB - 8);
  __shared__ float2 tile[1 << TB];
  const int tid = threadIdx.x;
  // per-thread parts (tile bits 0..7 = thread id bits)
  int64_t in_lo = 0, out_lo = 0;
  uint32_t wl_lo = 0;
#pragma unroll 1
  for (int b = 0; b < 8; ++b) {
    const int64_t bit = (tid >> b) & 1;
    in_lo += bit << p.rin[b];
    out_lo += bit << p.wout[b];
    wl_lo |= (uint32_t)bit << p.wpos[b];
  }
  const uint32_t rl_lo = perm_swz((uint32_t)tid, p.half);
  wl_lo = perm_swz(wl_lo, p.half);
  // per-element parts (tile bits 8.. = element counter e): element e's
  // offsets are sums of the strides of its set bits
  int64_t in_b[TB - 8], out_b[TB - 8];
  uint32_t w_b[TB - 8];
#pragma unroll
  for (int b = 8; b < TB; ++b) {
    in_b[b - 8] = (int64_t)1 << p.rin[b];
    out_b[b - 8] = (int64_t)1 << p.wout[b];
    w_b[b - 8] = 1u << p.wpos[b];
  }
  const int half = p.half;
  const uint64_t n_tiles = 1ull << p.rbits;
  for (uint64_t g = blockIdx.x; g < n_tiles; g += gridDim.x) {
    int64_t bin = 0, bout = 0;
#pragma unroll 1
    for (int b = 0; b < p.rbits; ++b) {
      const int64_t bit = (g >> b) & 1ull;
      bin += bit << p.tin[b];
      bout += bit << p.tout[b];
    }
    float2 v[E];
    const int64_t ib = bin + in_lo, ob = bout + out_lo;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int64_t a = 0;
#pragma unroll
      for (int b = 0; b < TB - 8; ++b)
        if ((e >> b) & 1) a += in_b[b];
      v[e] = p.in[ib + a];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) tile[rl_lo ^ perm_swz((uint32_t)e << 8, half)] = v[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      uint32_t w = 0;
#pragma unroll
      for (int b = 0; b < TB - 8; ++b)
        if ((e >> b) & 1) w |= w_b[b];
      v[e] = tile[wl_lo ^ perm_swz(w, half)];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int64_t c = 0;
#pragma unroll
      for (int b = 0; b < TB - 8; ++b)
        if ((e >> b) & 1) c += out_b[b];
      p.out[ob + c] = v[e];
    }
    __syncthreads();
  }
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
  // grid-stride: outputs beyond 2^32 / 256 workgroups (e.g. a whole state of
  // 4^16 entries) are covered by later passes of the same threads
  for (uint64_t o = (uint64_t)blockIdx.x * kBlock + threadIdx.x; o < n_out;
       o += (uint64_t)gridDim.x * kBlock) {
    const int64_t oo = scatter(o, p.s_open, p.open_bits);
    if (p.mode == 0) {
      double2 acc = p.out[o];
      if (p.n_sel < 0) {
        const uint64_t R = 1ull << p.res_bits;
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
        const uint64_t R = 1ull << p.res_bits;
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
}

// ---------------------------------------------------------------------------
// Adjoint of the slice sum: every resident slice of the root that the sum
// took receives the output gradient of its output element (times the number
// of times the slice was listed); n_sel < 0: every resident slice, once.
struct RootGradArgs {
  const double2* grad_out;
  float2* dst;
  int32_t open_bits, res_bits, accumulate;
  int32_t n_sel;
  int8_t s_open[kMaxBits], s_res[kMaxBits];
  int32_t sel_r[kMaxSel];
  float sel_w[kMaxSel];
};

__global__ void __launch_bounds__(kBlock) k_root_grad(RootGradArgs p) {
  const uint64_t rsel = p.n_sel < 0 ? 1ull << p.res_bits : (uint64_t)p.n_sel;
  const uint64_t n = rsel << p.open_bits;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock) {
    const uint64_t o = i & ((1ull << p.open_bits) - 1), j = i >> p.open_bits;
    const uint64_t r = p.n_sel < 0 ? j : (uint64_t)p.sel_r[j];
    const float w = p.n_sel < 0 ? 1.f : p.sel_w[j];
    int64_t off = scatter(o, p.s_open, p.open_bits) + scatter(r, p.s_res, p.res_bits);
    double2 g = p.grad_out[o];
    float2 v = make_float2(w * (float)g.x, w * (float)g.y);
    if (p.accumulate) {
      float2 c = p.dst[off];
      v.x += c.x;
      v.y += c.y;
    }
    p.dst[off] = v;
  }
}

// complex64 zero fill (gradient buffers that accumulate; a kernel, not a
// memset, so the call sequence can be captured in a graph).
__global__ void __launch_bounds__(kBlock) k_fill_c64(float2* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    out[i] = make_float2(0.f, 0.f);
}

}  // namespace tnk
