// C ABI (include/tn.h) and the host-side launcher.
//
// tn_contract walks the plan's schedule: steps that depend on no outer
// sliced index run once, the others once per outer iteration, each as one or
// two kernel launches on the caller's stream; after each iteration the
// resident slice results are added in float64 (Eq. sliced_sum).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tn.h"
#include "kernels_basic.h"
#include "kernels_chain.h"
#include "kernels_gemm.h"
#include "kernels_gemm_stream.h"
#include "kernels_persist.h"
#include "plan.h"

struct tn_plan_s {
  tn::Plan p;
};

static_assert(sizeof(tnk::SmallStep) == tn::kSmallStepBytes, "descriptor size");
static_assert(tnk::kSmallBits == tn::kSmallClassBits, "descriptor bits");
static_assert(tnk::kCtrStride == tn::kCtrStride, "counter spacing");
static_assert(tnk::kTinyMax == tn::kTinyMaxSteps && tnk::kTinyClassBits == tn::kTinyClassBits,
              "batches of tiny steps");

namespace {

thread_local std::string g_err;

tn_status fail(tn_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define TN_HIP_CHECK(expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(TN_E_HIP, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
  } while (0)

inline unsigned grid_for(uint64_t work, uint64_t cap = 1u << 20) {
  uint64_t g = (work + tnk::kBlock - 1) / tnk::kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

void copy_bits(int8_t* dst, const std::vector<int8_t>& src) {
  for (size_t i = 0; i < src.size(); ++i) dst[i] = src[i];
}

tnk::StepArgs make_args(const tn::StepDesc& S) {
  tnk::StepArgs a;
  memset(&a, 0, sizeof a);
  a.nb = (int32_t)S.bA.size();
  a.nm = (int32_t)S.mA.size();
  a.nn = (int32_t)S.nB.size();
  a.nk = (int32_t)S.kA.size();
  copy_bits(a.sA_b, S.bA);
  copy_bits(a.sB_b, S.bB);
  copy_bits(a.sC_b, S.bC);
  copy_bits(a.sA_m, S.mA);
  copy_bits(a.sC_m, S.mC);
  copy_bits(a.sB_n, S.nB);
  copy_bits(a.sC_n, S.nC);
  copy_bits(a.sA_k, S.kA);
  copy_bits(a.sB_k, S.kB);
  return a;
}

template <int NK, int NN>
void launch_stream_nn(const tnk::StreamArgs& a, uint64_t rows, hipStream_t st) {
  const bool shb = a.nbB == 0 || a.nrow - a.nbB >= 8;
  if (shb)
    hipLaunchKernelGGL((tnk::k_stream<NK, NN, true>), dim3(grid_for(rows, 1u << 16)),
                       dim3(tnk::kBlock), 0, st, a);
  else
    hipLaunchKernelGGL((tnk::k_stream<NK, NN, false>), dim3(grid_for(rows, 1u << 16)),
                       dim3(tnk::kBlock), 0, st, a);
}

template <int NK>
void launch_stream_k(const tnk::StreamArgs& a, int nn, uint64_t rows, hipStream_t st) {
  switch (nn) {
    case 0: launch_stream_nn<NK, 0>(a, rows, st); break;
    case 1: launch_stream_nn<NK, 1>(a, rows, st); break;
    case 2: launch_stream_nn<NK, 2>(a, rows, st); break;
    case 3: launch_stream_nn<NK, 3>(a, rows, st); break;
    default: launch_stream_nn<NK, 4>(a, rows, st); break;
  }
}

// Stream launch: row bits are the row (m) bits followed by the batch bits.
void launch_stream(const tnk::StepArgs& s, hipStream_t st) {
  tnk::StreamArgs a;
  memset(&a, 0, sizeof a);
  a.A = s.A;
  a.B = s.B;
  a.C = s.C;
  a.nrow = s.nm + s.nb;
  a.nbB = s.nb;
  a.conjA = s.conjA;
  a.conjB = s.conjB;
  a.accumulate = s.accumulate;
  for (int j = 0; j < s.nm; ++j) {
    a.rowA[j] = s.sA_m[j];
    a.rowC[j] = s.sC_m[j];
  }
  for (int j = 0; j < s.nb; ++j) {
    a.rowA[s.nm + j] = s.sA_b[j];
    a.rowC[s.nm + j] = s.sC_b[j];
    a.bB[j] = s.sB_b[j];
  }
  for (int j = 0; j < s.nk; ++j) {
    a.kA[j] = s.sA_k[j];
    a.kB[j] = s.sB_k[j];
  }
  for (int j = 0; j < s.nn; ++j) {
    a.nB[j] = s.sB_n[j];
    a.nC[j] = s.sC_n[j];
  }
  const uint64_t rows = 1ull << a.nrow;
  switch (s.nk) {
    case 0: launch_stream_k<0>(a, s.nn, rows, st); break;
    case 1: launch_stream_k<1>(a, s.nn, rows, st); break;
    case 2: launch_stream_k<2>(a, s.nn, rows, st); break;
    case 3: launch_stream_k<3>(a, s.nn, rows, st); break;
    default: launch_stream_k<4>(a, s.nn, rows, st); break;
  }
}

// Enumeration mask of a tile: merge the class-1 bits (rows of A / columns of
// B) and the k bits, each in class order, by ascending stride; bits beyond a
// class's size go last.  Bit j of the result is set where the merged order
// takes a class-1 bit.
uint32_t tile_mask(int L1, const int8_t* s1, int n1, int L2, const int8_t* s2, int n2) {
  uint32_t mask = 0;
  int i = 0, j = 0;
  for (int pos = 0; pos < L1 + L2; ++pos) {
    int k1 = i < L1 ? (i < n1 ? s1[i] : 1000 + i) : 1 << 30;
    int k2 = j < L2 ? (j < n2 ? s2[j] : 1000 + j) : 1 << 30;
    if (k1 <= k2) {
      mask |= 1u << pos;
      ++i;
    } else {
      ++j;
    }
  }
  return mask;
}

// Largest in-tile offset of a tile whose class-1 / k bits are the lowest L1 /
// L2 bits of their classes.
int64_t max_tile_offset(int L1, const int8_t* s1, int n1, int L2, const int8_t* s2, int n2) {
  int64_t m = 0;
  for (int j = 0; j < L1 && j < n1; ++j) m += (int64_t)1 << s1[j];
  for (int j = 0; j < L2 && j < n2; ++j) m += (int64_t)1 << s2[j];
  return m;
}

// One workgroup of 256 threads per tile.  A dispatch holds fewer than 2^32
// work-items, so steps with more than 2^23 tiles run as several launches,
// each over the next range of logical tiles.
constexpr uint64_t kMaxTilesPerLaunch = 1ull << 23;
template <auto Kernel>
void launch_tiles(uint64_t ntiles, const tnk::GemmArgs& g0, hipStream_t st) {
  tnk::GemmArgs g = g0;
  for (uint64_t t0 = 0; t0 < ntiles; t0 += kMaxTilesPerLaunch) {
    g.tile0 = t0;
    const uint64_t n = std::min(ntiles - t0, kMaxTilesPerLaunch);
    hipLaunchKernelGGL(Kernel, dim3((unsigned)n), dim3(256), 0, st, g);
  }
}

template <int WVM, int WVN, int WM, int WN, int LK>
tn_status launch_gemm_cfg(const tnk::StepArgs& a, int32_t precision, hipStream_t st,
                          int32_t chunks, float2* scratch, bool embed) {
  constexpr int MT = WVM * WM * 32, NT = WVN * WN * 16;
  constexpr int LM = tnk::ilog2<MT>::value, LN = tnk::ilog2<NT>::value;
  // split-BF16 tiles always walk k by 16
  const int lk = precision == tn::PREC_SPLIT_BF16 ? 4 : LK;
  tnk::GemmArgs g;
  memset(&g, 0, sizeof g);
  g.s = a;
  g.a_mask = tile_mask(LM, a.sA_m, a.nm, lk, a.sA_k, a.nk);
  g.b_mask = tile_mask(LN, a.sB_n, a.nn, lk, a.sB_k, a.nk);
  int lmt = a.nm > LM ? a.nm - LM : 0, lnt = a.nn > LN ? a.nn - LN : 0;
  uint64_t ntiles = 1ull << (a.nb + lmt + lnt);
  // split k: chunks of the k tiles write partial tiles into the scratch
  // area, which k_gemm_splitk_reduce adds up into C
  int kc = 0;
  while ((1 << (kc + 1)) <= chunks && kc + 1 <= a.nk - lk) ++kc;
  const int64_t n_out = (int64_t)1 << (a.nb + a.nm + a.nn);
  if (kc > 0) {
    if (!scratch) return fail(TN_E_INVALID, "split-k GEMM step without scratch");
    g.kc_log2 = kc;
    g.part_stride = n_out;
    g.s.C = scratch;
    g.s.accumulate = 0;
  }
  g.xcd_remap = (kc == 0 && ntiles >= 64) ? 1 : 0;
  const uint64_t nwg = ntiles << kc;
  const bool small = max_tile_offset(LM, a.sA_m, a.nm, lk, a.sA_k, a.nk) < (1ll << 31) &&
                     max_tile_offset(LN, a.sB_n, a.nn, lk, a.sB_k, a.nk) < (1ll << 31);
  if (precision == tn::PREC_SPLIT_BF16) {
    if (small) launch_tiles<tnk::k_gemm_sb16<WVM, WVN, WM, WN, int32_t>>(nwg, g, st);
    else launch_tiles<tnk::k_gemm_sb16<WVM, WVN, WM, WN, int64_t>>(nwg, g, st);
  } else if constexpr (WN % 2 == 0) {
    // complex64: three real products per complex product, unless the real
    // embedding is asked for (TN_FLAG_GEMM_EMBED)
    if (!embed) {
      if (small) launch_tiles<tnk::k_gemm_c64g<WVM, WVN, WM, WN, LK, int32_t>>(nwg, g, st);
      else launch_tiles<tnk::k_gemm_c64g<WVM, WVN, WM, WN, LK, int64_t>>(nwg, g, st);
    } else {
      if (small) launch_tiles<tnk::k_gemm_c64<WVM, WVN, WM, WN, LK, int32_t>>(nwg, g, st);
      else launch_tiles<tnk::k_gemm_c64<WVM, WVN, WM, WN, LK, int64_t>>(nwg, g, st);
    }
  } else {
    if (small) launch_tiles<tnk::k_gemm_c64<WVM, WVN, WM, WN, LK, int32_t>>(nwg, g, st);
    else launch_tiles<tnk::k_gemm_c64<WVM, WVN, WM, WN, LK, int64_t>>(nwg, g, st);
  }
  if (kc > 0)
    hipLaunchKernelGGL(tnk::k_gemm_splitk_reduce, dim3(grid_for((uint64_t)n_out)), dim3(256), 0,
                       st, a.C, scratch, n_out, (int32_t)(1 << kc), a.accumulate);
  return TN_OK;
}

// Stream kernel over 32-row bands (shape checked by stream_gemm_shape).  The
// k bits go in ascending order of A's strides (k is summed, so any order
// serves), so that a band's k tile is A's lowest-stride k bits.  About one
// workgroup per CU; a power of two (at least 8) of workgroups per column tile.
template <template <int> class P, int WN, int LKT, int DEPTH>
void launch_stream_cfg(const tnk::StreamGemmArgs& g, unsigned grid, hipStream_t st) {
  hipLaunchKernelGGL((tnk::k_gemm_stream<P, WN, LKT, DEPTH>), dim3(grid),
                     dim3(64 * tnk::kStreamWaves), 0, st, g);
}

bool launch_gemm_stream(const tnk::StepArgs& a, int32_t precision, bool gauss, hipStream_t st) {
  // in-band offsets of A are held in 32 bits
  int64_t band_off = 0;
  for (int j = 0; j < 5; ++j) band_off += (int64_t)1 << a.sA_m[j];
  for (int j = 0; j < a.nk; ++j) band_off += (int64_t)1 << a.sA_k[j];
  if (band_off >= (1ll << 32)) return false;
  tnk::StreamGemmArgs g;
  memset(&g, 0, sizeof g);
  g.s = a;
  int ord[tnk::kMaxBits];
  for (int j = 0; j < a.nk; ++j) ord[j] = j;
  std::sort(ord, ord + a.nk, [&](int x, int y) { return a.sA_k[x] < a.sA_k[y]; });
  for (int j = 0; j < a.nk; ++j) {
    g.s.sA_k[j] = a.sA_k[ord[j]];
    g.s.sB_k[j] = a.sB_k[ord[j]];
  }
  int ln, lkt;
  tn::stream_gemm_tile(a.nn, a.nk, precision, &ln, &lkt);
  if (gauss) {
    ln = std::min(std::min(a.nn, 6), 12 - a.nk);
    lkt = 5;
  }
  g.a_mask = tile_mask(5, g.s.sA_m, a.nm, lkt, g.s.sA_k, a.nk);
  g.lnt = a.nn - ln;
  g.nbands = 1ull << (a.nm - 5);
  // 2^lgroups band groups of 8 waves per column tile (at least 8, one per
  // XCD), about one workgroup per CU in all, never more than the bands need
  int lg = 3;
  while (lg < 8 - g.lnt && (1ull << (lg + 1 + 3)) <= g.nbands) ++lg;
  g.lgroups = lg;
  const unsigned grid = 1u << (lg + g.lnt);
  if (gauss) {
    if (ln == 5) launch_stream_cfg<tnk::StreamC64G, 2, 5, 2>(g, grid, st);
    else launch_stream_cfg<tnk::StreamC64G, 4, 5, 2>(g, grid, st);
    return true;
  }
  if (precision == tn::PREC_SPLIT_BF16) {
    switch (ln) {
      case 4: launch_stream_cfg<tnk::StreamSB16, 1, 5, 2>(g, grid, st); break;
      case 5: launch_stream_cfg<tnk::StreamSB16, 2, 5, 2>(g, grid, st); break;
      default: launch_stream_cfg<tnk::StreamSB16, 4, 5, 2>(g, grid, st); break;
    }
    return true;
  }
  switch (ln) {
    case 4: launch_stream_cfg<tnk::StreamC64, 1, 5, 2>(g, grid, st); break;
    case 5: launch_stream_cfg<tnk::StreamC64, 2, 5, 2>(g, grid, st); break;
    case 6: launch_stream_cfg<tnk::StreamC64, 4, 5, 2>(g, grid, st); break;
    default: launch_stream_cfg<tnk::StreamC64, 8, 4, 1>(g, grid, st); break;
  }
  return true;
}

tn_status launch_gemm(const tnk::StepArgs& a, int32_t precision, int32_t tile, hipStream_t st,
                      int32_t chunks, float2* scratch, bool embed) {
  if (tile == tn::kGemmStreamGauss) {
    if (tn::stream_gauss_shape(a.nb, a.nm, a.nn, a.nk, chunks, precision) &&
        launch_gemm_stream(a, precision, true, st))
      return TN_OK;
    tile = tn::kGemmStream;
  }
  if (tile == tn::kGemmStream) {
    if (tn::stream_gemm_shape(a.nb, a.nm, a.nn, a.nk, chunks, precision) &&
        launch_gemm_stream(a, precision, false, st))
      return TN_OK;
    tile = tn::rule_tile(a.nn);
  }
  switch (tile) {
    case 0: return launch_gemm_cfg<2, 2, 2, 2, 4>(a, precision, st, chunks, scratch, embed);   // 128 x 64
    case 1: return launch_gemm_cfg<4, 1, 1, 2, 4>(a, precision, st, chunks, scratch, embed);   // 128 x 32
    case 2: return launch_gemm_cfg<4, 1, 2, 1, 4>(a, precision, st, chunks, scratch, embed);   // 256 x 16
    case 3: return launch_gemm_cfg<2, 2, 2, 4, 4>(a, precision, st, chunks, scratch, embed);   // 128 x 128
    case 4: return launch_gemm_cfg<2, 2, 4, 2, 4>(a, precision, st, chunks, scratch, embed);   // 256 x 64
    case 5: return launch_gemm_cfg<2, 2, 2, 2, 5>(a, precision, st, chunks, scratch, embed);   // 128 x 64, k tile 32
    case 6: return launch_gemm_cfg<4, 1, 1, 2, 3>(a, precision, st, chunks, scratch, embed);   // 128 x 32, k tile 8
    case 7: return launch_gemm_cfg<4, 1, 1, 1, 4>(a, precision, st, chunks, scratch, embed);   // 128 x 16
    default: return fail(TN_E_INVALID, "unknown GEMM tile configuration");
  }
}

// Launch one contraction (forward or adjoint) with the given kernel family.
tn_status launch_step(int32_t kind, int32_t chunks, int32_t tile, const tnk::StepArgs& a0,
                      float2* scratch, int32_t precision, hipStream_t st, bool embed) {
  tnk::StepArgs a = a0;
  const uint64_t n_out = 1ull << (a.nb + a.nm + a.nn);
  if (kind == tn::KIND_SPLITK) {
    int cl = a.nk;
    int64_t nch = chunks;
    while ((1ll << (a.nk - cl)) < nch) --cl;
    a.chunk_log2 = cl;
    a.scratch = scratch;
    dim3 grid((unsigned)nch, (unsigned)(n_out < 65536 ? n_out : 65536),
              (unsigned)((n_out + 65535) / 65536));
    hipLaunchKernelGGL(tnk::k_splitk_partial, grid, dim3(tnk::kBlock), 0, st, a);
    hipLaunchKernelGGL(tnk::k_splitk_reduce, dim3(grid_for(n_out, 1u << 30)), dim3(tnk::kBlock),
                       0, st, a, nch);
  } else if (kind == tn::KIND_STREAM && a.nk <= 4 && a.nn <= 4) {
    launch_stream(a, st);
  } else if (kind == tn::KIND_GEMM) {
    tn_status s = launch_gemm(a, precision, tile, st, chunks, scratch, embed);
    if (s != TN_OK) return s;
  } else {
    hipLaunchKernelGGL(tnk::k_simple, dim3(grid_for(n_out)), dim3(tnk::kBlock), 0, st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return TN_OK;
}

// Kernel family and split-k chunks for an arbitrary (adjoint) shape.
int32_t kind_for(const tnk::StepArgs& a, uint32_t flags, int32_t* chunks) {
  int64_t scratch;
  return tn::choose_kind(a.nb, a.nm, a.nn, a.nk, flags, chunks, &scratch);
}

struct Ctx {
  const tn::Plan& p;
  const void* const* leaves;
  char* ws;
  float2* scratch;
  hipStream_t st;
};

// Element offset of leaf t's sub-block for outer iteration outer_val (its
// outer sliced bits fixed to that iteration's values).
int64_t leaf_outer_off(const tn::Plan& p, int t, uint64_t outer_val) {
  const tn::LeafDesc& L = p.leaves[t];
  int64_t off = 0;
  for (size_t i = 0; i < L.outer_bits.size(); ++i) {
    int bit = L.outer_bits[i];
    for (int j = 0; j < p.outer_bits; ++j)
      if (p.outer_bit_ids[j] == bit && ((outer_val >> j) & 1)) off += (int64_t)1 << L.outer_log2s[i];
  }
  return off;
}

const float2* node_ptr(const Ctx& c, int node, uint64_t outer_val) {
  const tn::Plan& p = c.p;
  if (node < p.n_tensors)
    return static_cast<const float2*>(c.leaves[node]) + leaf_outer_off(p, node, outer_val);
  return reinterpret_cast<const float2*>(c.ws + p.steps[node - p.n_tensors].c_off);
}

struct Probe {
  int32_t step = -1;
  hipEvent_t start = nullptr, stop = nullptr;
  bool done = false;
};

tn_status run_step(const Ctx& c, int k, uint64_t outer_val, Probe* probe = nullptr) {
  const tn::Plan& p = c.p;
  const tn::StepDesc& S = p.steps[k];
  tnk::StepArgs a = make_args(S);
  a.A = node_ptr(c, S.a, outer_val);
  a.B = node_ptr(c, S.b, outer_val);
  a.C = reinterpret_cast<float2*>(c.ws + S.c_off);
  bool timed = probe && !probe->done && probe->step == k;
  if (timed) TN_HIP_CHECK(hipEventRecord(probe->start, c.st));
  tn_status s = launch_step(S.kind, S.splitk_chunks, S.tile, a, c.scratch, p.precision, c.st,
                            (p.flags & 1024u) != 0);
  if (timed && s == TN_OK) {
    TN_HIP_CHECK(hipEventRecord(probe->stop, c.st));
    probe->done = true;
  }
  return s;
}

// A batch of tiny steps: one launch of one workgroup (k_tiny_run), the steps
// in the plan's level order.  A probe of one of its steps times the batch.
tn_status launch_tiny(const Ctx& c, const tn::Segment& g, uint64_t outer_val, Probe* probe) {
  const tn::Plan& p = c.p;
  tnk::TinyArgs a;
  memset(&a, 0, sizeof a);
  a.n = g.end - g.begin;
  bool timed = false;
  for (int q = g.begin; q < g.end; ++q) {
    const int k = p.sched[q];
    const tn::StepDesc& S = p.steps[k];
    tnk::TinyStep& T = a.st[q - g.begin];
    T.A = node_ptr(c, S.a, outer_val);
    T.B = node_ptr(c, S.b, outer_val);
    T.C = reinterpret_cast<float2*>(c.ws + S.c_off);
    T.nb = (int8_t)S.bA.size();
    T.nm = (int8_t)S.mA.size();
    T.nn = (int8_t)S.nB.size();
    T.nk = (int8_t)S.kA.size();
    T.level = p.tiny_level[q];
    copy_bits(T.sA_b, S.bA);
    copy_bits(T.sB_b, S.bB);
    copy_bits(T.sC_b, S.bC);
    copy_bits(T.sA_m, S.mA);
    copy_bits(T.sC_m, S.mC);
    copy_bits(T.sB_n, S.nB);
    copy_bits(T.sC_n, S.nC);
    copy_bits(T.sA_k, S.kA);
    copy_bits(T.sB_k, S.kB);
    timed |= probe && !probe->done && probe->step == k;
  }
  if (timed) TN_HIP_CHECK(hipEventRecord(probe->start, c.st));
  hipLaunchKernelGGL(tnk::k_tiny_run, dim3(1), dim3(tnk::kTinyBlock), 0, c.st, a);
  TN_HIP_CHECK(hipGetLastError());
  if (timed) {
    TN_HIP_CHECK(hipEventRecord(probe->stop, c.st));
    probe->done = true;
  }
  return TN_OK;
}

// Tiny products issued one after another outside the plan's batches (the
// adjoint's forward values, recomputations and adjoint products) gathered
// into k_tiny_run launches.  A product's level is one above that of every
// earlier product of the batch it conflicts with -- it reads memory that one
// writes, or writes memory that one reads or writes -- so running the levels
// in order, all products of a level at once, gives the issue order's results
// whatever the buffers share.  Any other launch on the stream flushes first.
class TinyBatcher {
 public:
  TinyBatcher(hipStream_t st, bool enabled) : st_(st), enabled_(enabled) {}
  // true when the product qualifies (the plan's tiny-step limits)
  bool fits(const tnk::StepArgs& a, int32_t kind, int32_t chunks) const {
    return enabled_ && kind != tn::KIND_SPLITK && chunks <= 1 && a.nb + a.nm + a.nn <= tn::kTinyOutBits &&
           a.nb + a.nm + a.nn + a.nk <= tn::kTinyCmacBits && a.nb <= tnk::kTinyClassBits &&
           a.nm <= tnk::kTinyClassBits && a.nn <= tnk::kTinyClassBits &&
           a.nk <= tnk::kTinyClassBits;
  }
  tn_status add(const tnk::StepArgs& a) {
    if (n_ == tnk::kTinyMax) {
      tn_status s = flush();
      if (s != TN_OK) return s;
    }
    Item& it = items_[n_];
    it.a = a;
    it.rA = range(a.A, {a.sA_b, a.sA_m, a.sA_k}, {a.nb, a.nm, a.nk});
    it.rB = range(a.B, {a.sB_b, a.sB_n, a.sB_k}, {a.nb, a.nn, a.nk});
    it.rC = range(a.C, {a.sC_b, a.sC_m, a.sC_n}, {a.nb, a.nm, a.nn});
    int lv = 0;
    for (int i = 0; i < n_; ++i) {
      const Item& e = items_[i];
      const bool conflict = meet(e.rC, it.rA) || meet(e.rC, it.rB) || meet(e.rC, it.rC) ||
                            meet(it.rC, e.rA) || meet(it.rC, e.rB);
      if (conflict) lv = std::max(lv, e.level + 1);
    }
    it.level = lv;
    ++n_;
    return TN_OK;
  }
  tn_status flush() {
    if (n_ == 0) return TN_OK;
    int order[tnk::kTinyMax];
    for (int i = 0; i < n_; ++i) order[i] = i;
    std::stable_sort(order, order + n_,
                     [&](int x, int y) { return items_[x].level < items_[y].level; });
    tnk::TinyArgs t;
    memset(&t, 0, sizeof t);
    t.n = n_;
    for (int j = 0; j < n_; ++j) {
      const Item& e = items_[order[j]];
      tnk::TinyStep& T = t.st[j];
      T.A = e.a.A;
      T.B = e.a.B;
      T.C = e.a.C;
      T.nb = (int8_t)e.a.nb;
      T.nm = (int8_t)e.a.nm;
      T.nn = (int8_t)e.a.nn;
      T.nk = (int8_t)e.a.nk;
      T.level = (int8_t)e.level;
      T.conjA = (int8_t)(e.a.conjA != 0);
      T.conjB = (int8_t)(e.a.conjB != 0);
      T.accumulate = (int8_t)(e.a.accumulate != 0);
      memcpy(T.sA_b, e.a.sA_b, tnk::kTinyClassBits);
      memcpy(T.sB_b, e.a.sB_b, tnk::kTinyClassBits);
      memcpy(T.sC_b, e.a.sC_b, tnk::kTinyClassBits);
      memcpy(T.sA_m, e.a.sA_m, tnk::kTinyClassBits);
      memcpy(T.sC_m, e.a.sC_m, tnk::kTinyClassBits);
      memcpy(T.sB_n, e.a.sB_n, tnk::kTinyClassBits);
      memcpy(T.sC_n, e.a.sC_n, tnk::kTinyClassBits);
      memcpy(T.sA_k, e.a.sA_k, tnk::kTinyClassBits);
      memcpy(T.sB_k, e.a.sB_k, tnk::kTinyClassBits);
    }
    n_ = 0;
    ++launches_;
    hipLaunchKernelGGL(tnk::k_tiny_run, dim3(1), dim3(tnk::kTinyBlock), 0, st_, t);
    TN_HIP_CHECK(hipGetLastError());
    return TN_OK;
  }
  int64_t launches() const { return launches_; }

 private:
  struct Range {
    uintptr_t lo, hi;   // bytes [lo, hi)
  };
  struct Item {
    tnk::StepArgs a;
    Range rA, rB, rC;
    int level;
  };
  // bytes an operand can touch: its base up to the largest offset its bits
  // reach (every bit set), plus one entry
  static Range range(const void* base, std::initializer_list<const int8_t*> s,
                     std::initializer_list<int> nbits) {
    uint64_t top = 0;
    auto b = nbits.begin();
    for (const int8_t* v : s) {
      for (int j = 0; j < *b; ++j) top += 1ull << v[j];
      ++b;
    }
    const uintptr_t lo = reinterpret_cast<uintptr_t>(base);
    return {lo, lo + (top + 1) * sizeof(float2)};
  }
  static bool meet(const Range& x, const Range& y) { return x.lo < y.hi && y.lo < x.hi; }
  hipStream_t st_;
  bool enabled_;
  Item items_[tnk::kTinyMax];
  int n_ = 0;
  int64_t launches_ = 0;
};

// One fused chain (all its steps, one launch).
// Operand addresses of a launch: node id -> device pointer.
using NodeSrc = std::function<const float2*(int)>;

tn_status run_chain_with(const Ctx& c, const tn::ChainGroup& g, const NodeSrc& src, float2* Y,
                         Probe* probe);

tn_status run_chain(const Ctx& c, const tn::ChainGroup& g, uint64_t outer_val,
                    Probe* probe = nullptr) {
  return run_chain_with(
      c, g, [&](int x) { return node_ptr(c, x, outer_val); },
      reinterpret_cast<float2*>(c.ws + c.p.steps[g.last].c_off), probe);
}

tn_status run_chain_with(const Ctx& c, const tn::ChainGroup& g, const NodeSrc& src, float2* Y,
                         Probe* probe) {
  const tn::Plan& p = c.p;
  static_assert(sizeof(tnk::ChainArgs) % 4 == 0, "argument copy in 32-bit words");
  static_assert(tnk::kChainSteps == tn::kChainMaxSteps && tnk::kChainTile == tn::kChainTileBits &&
                    tnk::kChainPas == tn::kChainPassive && tnk::kChainBF == tn::kChainBFloats &&
                    tnk::kChainV == tn::kChainVElems,
                "chain limits agree");
  tnk::ChainArgs a;
  memset(&a, 0, sizeof a);
  const tn::StepDesc& F = p.steps[g.first];
  a.X = src(F.a);
  a.Y = Y;
  a.nsteps = (int32_t)g.st.size();
  a.tin = (int32_t)g.in_slot.size();
  a.tout = (int32_t)g.out_slot.size();
  a.npas = (int32_t)g.pas_in.size();
  for (size_t i = 0; i < g.in_slot.size(); ++i) {
    a.in_slot[i] = g.in_slot[i];
    a.in_log2[i] = g.in_log2[i];
  }
  for (size_t i = 0; i < g.out_slot.size(); ++i) {
    a.out_slot[i] = g.out_slot[i];
    a.out_log2[i] = g.out_log2[i];
  }
  for (size_t i = 0; i < g.pas_in.size(); ++i) {
    a.pas_in[i] = g.pas_in[i];
    a.pas_out[i] = g.pas_out[i];
  }
  int fl = 0, ve = 0;   // staged floats, vector-step table entries
  for (size_t q = 0; q < g.st.size(); ++q) {
    const tn::ChainStepDesc& d = g.st[q];
    tnk::ChainStepArgs& t = a.st[q];
    if (d.kslot.size() > 6 || d.nslot.size() > 6 || d.rslot.size() > (size_t)tnk::kChainTile ||
        d.bB.size() > (size_t)tnk::kChainTile)
      return fail(TN_E_INVALID, "chain step exceeds its descriptor");
    t.B = src(p.steps[d.step].b);
    t.nk = (int8_t)d.kslot.size();
    t.nn = (int8_t)d.nslot.size();
    t.nrow = (int8_t)d.nrow;
    t.nbb = (int8_t)d.bB.size();
    for (size_t j = 0; j < d.kslot.size(); ++j) {
      t.kslot[j] = d.kslot[j];
      t.kB[j] = d.kB[j];
    }
    for (size_t j = 0; j < d.nslot.size(); ++j) {
      t.nslot[j] = d.nslot[j];
      t.nB[j] = d.nB[j];
    }
    for (size_t j = 0; j < d.rslot.size(); ++j) t.rslot[j] = d.rslot[j];
    for (size_t j = 0; j < d.bB.size(); ++j) {
      t.bB[j] = d.bB[j];
      t.bpas[j] = d.bpas[j];
    }
    if (!d.bB.empty()) a.b_per_tile = 1;
    t.boff0 = fl;
    t.voff0 = ve;
    t.mfma = tn::chain_step_mfma(t.nk, t.nn, t.nrow, p.flags);
    if ((t.nk > 4 || t.nn > 4) && !t.mfma)
      return fail(TN_E_INVALID, "chain step shape needs the matrix-core path");
    if (t.mfma ? t.nrow > 10 : t.nrow > 14)   // row-part table: 64 entries per step
      return fail(TN_E_INVALID, "chain step has more rows than its table");
    fl += tn::chain_staged_floats(t.nk, t.nn, t.mfma);
    if (!t.mfma) ve += 1 << (t.nk + t.nn);
  }
  a.b_total = fl;
  a.split = p.precision == tn::PREC_SPLIT_BF16;
  if (fl > tnk::kChainBF || ve > tnk::kChainV || g.tile_bits > tnk::kChainTile)
    return fail(TN_E_INVALID, "chain exceeds its on-chip limits");
  const uint64_t n_tiles = 1ull << a.npas;
  const unsigned grid = (unsigned)std::min<uint64_t>(n_tiles, 1u << 16);
  {
    int lg = 0;
    while ((1u << (lg + 1)) <= grid) ++lg;
    int64_t si = 0, so = 0;
    for (int c = 0; c < tnk::kChainPas; ++c) {
      a.din[c] = a.dout[c] = 0;
      if (lg + c < a.npas) {
        a.din[c] = ((int64_t)1 << a.pas_in[lg + c]) - si;
        a.dout[c] = ((int64_t)1 << a.pas_out[lg + c]) - so;
        si += (int64_t)1 << a.pas_in[lg + c];
        so += (int64_t)1 << a.pas_out[lg + c];
      }
    }
  }
  bool timed = false;
  static_assert(sizeof(a.st[0].kslot) / sizeof(a.st[0].kslot[0]) >= 6 &&
                    sizeof(a.st[0].nslot) / sizeof(a.st[0].nslot[0]) >= 6,
                "chain step arrays hold the largest summed / new bit counts");
  if (probe && !probe->done)
    for (int k = g.first; k <= g.last; ++k) timed |= probe->step == k;
  if (timed) TN_HIP_CHECK(hipEventRecord(probe->start, c.st));
  // kernel build: small shapes with staged operands that leave room for 4
  // workgroups per CU (LDS: 32 KiB tile + staging <= 40 KiB), else the
  // prefetching build unless a split-BF16 step needs the full one
  bool heavy = false, small = true;
  for (int q = 0; q < a.nsteps; ++q) {
    heavy |= tn::chain_needs_heavy(a.st[q].nk, a.st[q].mfma != 0, a.split != 0);
    small &= tnk::chain_small_step(a.st[q].nk, a.st[q].nn, a.st[q].mfma != 0);
  }
  const size_t dyn = std::max<size_t>(16, (size_t)a.b_total * sizeof(float));
  small &= (sizeof(float2) << 12) + dyn <= 40u * 1024u;
  if (g.tile_bits <= 10)
    hipLaunchKernelGGL((tnk::k_chain<10, 0>), dim3(grid), dim3(256), dyn, c.st, a);
  else if (g.tile_bits == 11)
    hipLaunchKernelGGL((tnk::k_chain<11, 0>), dim3(grid), dim3(256), dyn, c.st, a);
  else if (small)
    hipLaunchKernelGGL((tnk::k_chain<12, 2>), dim3(grid), dim3(256), dyn, c.st, a);
  else if (heavy)
    hipLaunchKernelGGL((tnk::k_chain<12, 0>), dim3(grid), dim3(256), dyn, c.st, a);
  else
    hipLaunchKernelGGL((tnk::k_chain<12, 1>), dim3(grid), dim3(256), dyn, c.st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TN_E_HIP, std::string("chain launch: ") + hipGetErrorString(e));
  if (timed) {
    TN_HIP_CHECK(hipEventRecord(probe->stop, c.st));
    probe->done = true;
  }
  return TN_OK;
}

}  // namespace

// Control region of the persistent segments: a 256-byte header whose first
// word collects timed-out waits of every segment launch, then for every
// (segment, execution) the device descriptors, the item -> step table and
// zeroed counters, built on the host and copied with one transfer at the
// start of tn_contract.
struct SegLayout {
  int64_t off_desc, off_items, off_ctr;
};

static int64_t al256(int64_t x) { return (x + 255) / 256 * 256; }

static void build_persist_blob(const Ctx& c, std::vector<char>& blob,
                               std::vector<std::vector<SegLayout>>& lay) {
  const tn::Plan& p = c.p;
  const int n = p.n_tensors;
  const uint64_t n_it = 1ull << p.outer_bits;
  blob.assign((size_t)p.persist_bytes, 0);
  lay.assign(p.segments.size(), {});
  std::vector<int32_t> pos_of(p.steps.size(), -1);
  for (size_t q = 0; q < p.sched.size(); ++q) pos_of[p.sched[q]] = (int32_t)q;
  int64_t off = p.segments.empty() ? 0 : 256;   // header: error word
  for (size_t gi = 0; gi < p.segments.size(); ++gi) {
    const tn::Segment& g = p.segments[gi];
    const int len = g.end - g.begin;
    const uint64_t execs = g.phase ? n_it : 1;
    for (uint64_t e = 0; e < execs; ++e) {
      SegLayout L;
      L.off_desc = off;
      L.off_items = L.off_desc + al256((int64_t)len * tn::kSmallStepBytes);
      L.off_ctr = L.off_items + al256((int64_t)4 * g.n_items);
      off = L.off_ctr + al256((int64_t)4 * tnk::kCtrStride * (len + 2));
      tnk::SmallStep* d = reinterpret_cast<tnk::SmallStep*>(blob.data() + L.off_desc);
      int32_t* items = reinterpret_cast<int32_t*>(blob.data() + L.off_items);
      int32_t item = 0;
      for (int i = 0; i < len; ++i) {
        const tn::StepDesc& S = p.steps[p.sched[g.begin + i]];
        tnk::SmallStep& D = d[i];
        memset(&D, 0, sizeof D);
        D.A = node_ptr(c, S.a, e);
        D.B = node_ptr(c, S.b, e);
        D.C = reinterpret_cast<float2*>(c.ws + S.c_off);
        D.nb = (int32_t)S.bA.size();
        D.nm = (int32_t)S.mA.size();
        D.nn = (int32_t)S.nB.size();
        D.nk = (int32_t)S.kA.size();
        copy_bits(D.sA_b, S.bA); copy_bits(D.sB_b, S.bB); copy_bits(D.sC_b, S.bC);
        copy_bits(D.sA_m, S.mA); copy_bits(D.sC_m, S.mC);
        copy_bits(D.sB_n, S.nB); copy_bits(D.sC_n, S.nC);
        copy_bits(D.sA_k, S.kA); copy_bits(D.sB_k, S.kB);
        const int64_t outs = (int64_t)1 << (D.nb + D.nm + D.nn);
        D.n_items = (int32_t)((outs + 255) / 256);
        D.item0 = item;
        for (int32_t q = 0; q < D.n_items; ++q) items[item + q] = i;
        item += D.n_items;
        int32_t dep[2] = {-1, -1};
        int nd = 0;
        for (int x : {S.a, S.b}) {
          if (x < n) continue;
          int32_t ps = pos_of[x - n];
          if (ps >= g.begin && ps < g.end) dep[nd++] = ps - g.begin;
        }
        D.dep0 = dep[0];
        D.dep1 = dep[1];
      }
      lay[gi].push_back(L);
    }
  }
}

static tn_status launch_segment(const Ctx& c, const tn::Segment& g, const SegLayout& L,
                                char* pbase) {
  const int len = g.end - g.begin;
  int32_t* ctr = reinterpret_cast<int32_t*>(pbase + L.off_ctr);
  unsigned grid = (unsigned)(g.n_items < 2048 ? g.n_items : 2048);
  hipLaunchKernelGGL(tnk::k_persistent, dim3(grid), dim3(256), 0, c.st,
                     reinterpret_cast<const tnk::SmallStep*>(pbase + L.off_desc),
                     reinterpret_cast<const int32_t*>(pbase + L.off_items), g.n_items, ctr,
                     reinterpret_cast<int32_t*>(pbase));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TN_E_HIP, std::string("persistent launch: ") + hipGetErrorString(e));
  return TN_OK;
}

// Keeps a host buffer that a queued host-to-device copy reads from alive
// until the stream has passed that copy: on every exit from the call that
// queued it, the stream is synchronised before the buffer is released.
struct StagedUpload {
  std::vector<char> buf;
  hipStream_t st = nullptr;
  bool queued = false;
  ~StagedUpload() {
    if (queued) (void)hipStreamSynchronize(st);
  }
};

static tn_status contract_impl(tn_plan_t plan, const void* const* leaves,
                               const int64_t* slice_ids, int64_t n_slice_ids, int32_t out_mode,
                               void* out, void* ws, size_t ws_bytes, void* stream, Probe* probe,
                               uint32_t call_flags = 0);

extern "C" {

const char* tn_last_error(void) { return g_err.c_str(); }

tn_status tn_plan_create(int32_t n_tensors, const int32_t* ranks, const int32_t* index_ids,
                         int32_t n_index, const int32_t* index_dims, int32_t n_open,
                         const int32_t* open_ids, int32_t n_steps, const int32_t* path,
                         int32_t n_sliced, const int32_t* sliced_ids,
                         const tn_plan_options* opts, tn_plan_t* out) {
  if (!out) return fail(TN_E_INVALID, "out is NULL");
  *out = nullptr;
  tn_plan_options o;
  memset(&o, 0, sizeof o);
  o.max_resident_bits = -1;
  o.gemm_config = -1;
  if (opts) o = *opts;
  try {
    // an amplitude batch: one more index, the leading axis of the batched
    // leaves and the leading open index
    std::vector<int32_t> b_ranks, b_ids, b_dims, b_open;
    if (o.batch > 1) {
      if (o.batch & (o.batch - 1)) return fail(TN_E_UNSUPPORTED, "batch is not a power of two");
      if (n_tensors < 1 || !ranks || !index_ids || !index_dims || (n_open > 0 && !open_ids))
        return fail(TN_E_INVALID, "NULL network arrays");
      if (o.n_batched < 1 || !o.batched_leaves) return fail(TN_E_INVALID, "no batched leaf");
      std::vector<char> bat(n_tensors, 0);
      for (int32_t i = 0; i < o.n_batched; ++i) {
        const int32_t t = o.batched_leaves[i];
        if (t < 0 || t >= n_tensors || bat[t]) return fail(TN_E_INVALID, "bad batched leaf list");
        bat[t] = 1;
      }
      int64_t pos = 0;
      for (int32_t t = 0; t < n_tensors; ++t) {
        if (ranks[t] < 0) return fail(TN_E_INVALID, "negative rank");
        b_ranks.push_back(ranks[t] + bat[t]);
        if (bat[t]) b_ids.push_back(n_index);
        for (int32_t j = 0; j < ranks[t]; ++j) b_ids.push_back(index_ids[pos + j]);
        pos += ranks[t];
      }
      b_dims.assign(index_dims, index_dims + n_index);
      b_dims.push_back(o.batch);
      b_open.push_back(n_index);
      for (int32_t j = 0; j < n_open; ++j) b_open.push_back(open_ids[j]);
      ranks = b_ranks.data();
      index_ids = b_ids.data();
      index_dims = b_dims.data();
      n_index += 1;
      open_ids = b_open.data();
      n_open += 1;
    }
    tn_plan_s* h = new tn_plan_s();
    bool unsup = false;
    std::string err = tn::build_plan(h->p, n_tensors, ranks, index_ids, n_index, index_dims,
                                     n_open, open_ids, n_steps, path, n_sliced, sliced_ids,
                                     o.precision, o.max_resident_bits, o.workspace_limit,
                                     o.flags, o.gemm_config, o.tune, o.n_tune,
                                     o.checkpoint_policy, o.variable_leaves, o.n_variable,
                                     &unsup);
    if (!err.empty()) {
      delete h;
      return fail(unsup ? TN_E_UNSUPPORTED : TN_E_INVALID, err);
    }
    *out = h;
    return TN_OK;
  } catch (const std::bad_alloc&) {
    return fail(TN_E_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(TN_E_INVALID, e.what());
  }
}

void tn_plan_destroy(tn_plan_t plan) { delete plan; }

tn_status tn_plan_query(tn_plan_t plan, tn_plan_info* out) {
  if (!plan || !out) return fail(TN_E_INVALID, "NULL argument");
  const tn::Plan& p = plan->p;
  memset(out, 0, sizeof *out);
  out->n_tensors = p.n_tensors;
  out->n_steps = p.n_tensors - 1;
  out->n_index = p.n_index;
  out->n_sliced = (int32_t)p.sliced_ids.size();
  out->n_open_bits = p.open_bits;
  out->n_resident_bits = p.resident_bits;
  out->n_outer_bits = p.outer_bits;
  out->max_log2_per_slice = p.max_log2_sl;
  out->max_log2_resident = p.max_log2_res;
  out->n_launches = p.n_launches;
  out->n_slices = p.n_slices;
  out->out_elems = (int64_t)1 << p.open_bits;
  out->workspace_bytes = p.workspace_bytes;
  out->workspace_backward_bytes = p.workspace_bwd_bytes;
  out->arena_bytes = p.arena_bytes;
  out->bytes_no_deletion = p.bytes_no_deletion;
  out->cmac_reuse = p.cmac_reuse;
  out->cmac_noreuse = p.cmac_noreuse;
  out->cmac_exec = p.cmac_exec;
  out->cmac_per_slice = p.cmac_sl;
  out->f_sl = p.f_sl;
  out->bytes_min_exec = p.bytes_min_exec;
  copy_bits(out->root_open_log2, p.root_open_log2);
  copy_bits(out->root_res_log2, p.root_res_log2);
  for (int j = 0; j < p.resident_bits; ++j) out->res_slicebit[j] = (int8_t)p.res_slicebit[j];
  for (int j = 0; j < p.outer_bits; ++j) out->outer_slicebit[j] = (int8_t)p.outer_slicebit[j];
  out->n_chains = (int32_t)p.chains.size();
  out->n_segments = (int32_t)p.segments.size();
  out->segment_table_bytes = p.persist_bytes;
  out->segment_table_offset = al256(p.arena_bytes) + al256(p.scratch_bytes) + p.ctrl_bytes;
  out->n_phase0 = p.n_phase0;
  out->backward_policy = p.bwd.policy;
  out->backward_blocks = (int32_t)p.bwd.block_begin.size();
  out->cmac_backward_recompute = p.bwd.cmac_recompute;
  out->n_invariant = p.n_invariant;
  {
    double cm = 0;
    int32_t skipped = 0;
    std::vector<uint8_t> chain_done(p.chains.size(), 0);
    std::vector<int32_t> tiny_end(p.sched.size(), -1);   // batch start -> its end
    for (const tn::Segment& g : p.tiny_runs) tiny_end[g.begin] = g.end;
    for (int q = 0; q < p.n_invariant; ++q) {
      const tn::StepDesc& S = p.steps[p.sched[q]];
      cm += S.cmac;
      if (tiny_end[q] >= 0) {   // a batch of tiny steps: one launch
        ++skipped;
        for (int r = q + 1; r < tiny_end[q]; ++r) cm += p.steps[p.sched[r]].cmac;
        q = tiny_end[q] - 1;
      } else if (S.chain >= 0 && !(p.flags & 64u)) {   // one launch per fused chain
        if (!chain_done[S.chain]) ++skipped;
        chain_done[S.chain] = 1;
      } else {
        ++skipped;   // segments, split-k and multi-launch GEMM steps count once
      }
    }
    out->cmac_invariant = cm;
    out->n_launches_reuse = p.n_launches - skipped;
  }
  return TN_OK;
}

tn_status tn_plan_step(tn_plan_t plan, int32_t step, tn_step_info* out) {
  if (!plan || !out) return fail(TN_E_INVALID, "NULL argument");
  const tn::Plan& p = plan->p;
  if (step < 0 || step >= p.n_tensors - 1) return fail(TN_E_INVALID, "step out of range");
  const tn::StepDesc& S = p.steps[step];
  memset(out, 0, sizeof *out);
  out->a = S.a;
  out->b = S.b;
  out->c = S.c;
  out->phase = S.phase;
  out->kind = S.kind;
  out->nb = (int32_t)S.bA.size();
  out->nm = (int32_t)S.mA.size();
  out->nn = (int32_t)S.nB.size();
  out->nk = (int32_t)S.kA.size();
  out->inst_bits = S.inst_bits;
  out->tile = S.tile;
  out->cmac = S.cmac;
  copy_bits(out->sA_b, S.bA);
  copy_bits(out->sB_b, S.bB);
  copy_bits(out->sC_b, S.bC);
  copy_bits(out->sA_m, S.mA);
  copy_bits(out->sC_m, S.mC);
  copy_bits(out->sB_n, S.nB);
  copy_bits(out->sC_n, S.nC);
  copy_bits(out->sA_k, S.kA);
  copy_bits(out->sB_k, S.kB);
  out->c_offset = S.c_off;
  out->c_bytes = S.c_bytes;
  out->chain = S.chain;
  out->chunks = S.splitk_chunks > 1 ? S.splitk_chunks : 1;
  out->tiny_batch = -1;
  out->tiny_level = 0;
  for (size_t gi = 0; gi < p.tiny_runs.size(); ++gi)
    for (int q = p.tiny_runs[gi].begin; q < p.tiny_runs[gi].end; ++q)
      if (p.sched[q] == step) {
        out->tiny_batch = (int32_t)gi;
        out->tiny_level = p.tiny_level[q];
      }
  out->tile_run = S.kind == tn::KIND_GEMM
                      ? tn::tile_run(S.tile, (int)S.bA.size(), (int)S.mA.size(), (int)S.nB.size(),
                                     (int)S.kA.size(), S.splitk_chunks, p.precision)
                      : -1;
  return TN_OK;
}

tn_status tn_plan_chain(tn_plan_t plan, int32_t i, tn_chain_info* out) {
  if (!plan || !out) return fail(TN_E_INVALID, "NULL argument");
  const tn::Plan& p = plan->p;
  if (i < 0 || i >= (int32_t)p.chains.size()) return fail(TN_E_INVALID, "chain index out of range");
  const tn::ChainGroup& g = p.chains[i];
  memset(out, 0, sizeof *out);
  out->first = g.first;
  out->last = g.last;
  out->phase = g.phase;
  out->tile_bits = g.tile_bits;
  out->n_in = (int32_t)g.in_slot.size();
  out->n_out = (int32_t)g.out_slot.size();
  out->n_passive = (int32_t)g.pas_in.size();
  out->n_steps = (int32_t)g.st.size();
  copy_bits(out->in_slot, g.in_slot);
  copy_bits(out->in_log2, g.in_log2);
  copy_bits(out->out_slot, g.out_slot);
  copy_bits(out->out_log2, g.out_log2);
  copy_bits(out->pas_in, g.pas_in);
  copy_bits(out->pas_out, g.pas_out);
  for (size_t q = 0; q < g.st.size(); ++q) {
    const tn::ChainStepDesc& d = g.st[q];
    tn_chain_step_info& t = out->st[q];
    if (d.kslot.size() > 8 || d.nslot.size() > 8 || d.rslot.size() > 12 || d.bB.size() > 12)
      return fail(TN_E_INVALID, "chain step exceeds its descriptor");
    t.step = d.step;
    t.nrow = d.nrow;
    t.nk = (int32_t)d.kslot.size();
    t.nn = (int32_t)d.nslot.size();
    t.nbb = (int32_t)d.bB.size();
    copy_bits(t.kslot, d.kslot);
    copy_bits(t.nslot, d.nslot);
    copy_bits(t.kB, d.kB);
    copy_bits(t.nB, d.nB);
    copy_bits(t.rslot, d.rslot);
    copy_bits(t.bB, d.bB);
    copy_bits(t.bpas, d.bpas);
  }
  return TN_OK;
}

tn_status tn_plan_segment_tables(tn_plan_t plan, const void* const* leaves, void* ws,
                                 void* blob, int64_t blob_bytes, tn_segment_layout* lay,
                                 int32_t max_lay, int32_t* n_lay) {
  if (!plan || !leaves || !blob || !n_lay) return fail(TN_E_INVALID, "NULL argument");
  const tn::Plan& p = plan->p;
  if (blob_bytes < p.persist_bytes) return fail(TN_E_INVALID, "blob smaller than the tables");
  for (int t = 0; t < p.n_tensors; ++t)
    if (!leaves[t]) return fail(TN_E_INVALID, "NULL leaf pointer");
  try {
    Ctx c{p, leaves, static_cast<char*>(ws), nullptr, nullptr};
    std::vector<char> b;
    std::vector<std::vector<SegLayout>> L;
    build_persist_blob(c, b, L);
    if (!b.empty()) memcpy(blob, b.data(), b.size());
    int32_t k = 0;
    for (size_t gi = 0; gi < L.size(); ++gi)
      for (size_t e = 0; e < L[gi].size(); ++e, ++k) {
        if (k >= max_lay || !lay) continue;
        tn_segment_layout& o = lay[k];
        memset(&o, 0, sizeof o);
        o.segment = (int32_t)gi;
        o.execution = (int32_t)e;
        o.n_steps = p.segments[gi].end - p.segments[gi].begin;
        o.n_items = p.segments[gi].n_items;
        o.first_pos = p.segments[gi].begin;
        o.off_desc = L[gi][e].off_desc;
        o.off_items = L[gi][e].off_items;
        o.off_ctr = L[gi][e].off_ctr;
      }
    *n_lay = k;
    if (k > max_lay) return fail(TN_E_INVALID, "layout array too short");
    return TN_OK;
  } catch (const std::bad_alloc&) {
    return fail(TN_E_OOM, "host allocation failed");
  }
}

tn_status tn_plan_backward_tables(tn_plan_t plan, int8_t* keep, int8_t* frontier,
                                  int64_t* value_off, int64_t* recompute_off, int64_t* grad_off,
                                  int32_t* block_of, int8_t* fuse_chain) {
  if (!plan || !keep || !frontier || !value_off || !recompute_off || !grad_off || !block_of)
    return fail(TN_E_INVALID, "NULL argument");
  const tn::BwdPlan& B = plan->p.bwd;
  const size_t nodes = (size_t)(2 * plan->p.n_tensors - 1);
  for (size_t v = 0; v < nodes; ++v) {
    const bool has = v < B.keep.size();
    keep[v] = has ? (int8_t)B.keep[v] : 0;
    frontier[v] = has ? (int8_t)B.frontier[v] : 0;
    value_off[v] = has ? B.fwd_off[v] : -1;
    recompute_off[v] = has ? B.rec_off[v] : -1;
    grad_off[v] = has ? B.grad_off[v] : -1;
  }
  for (size_t q = 0; q < B.block_of.size(); ++q) block_of[q] = B.block_of[q];
  if (fuse_chain)
    for (size_t g = 0; g < B.fuse_chain.size(); ++g) fuse_chain[g] = (int8_t)B.fuse_chain[g];
  return TN_OK;
}

tn_status tn_plan_schedule(tn_plan_t plan, int32_t* order, int32_t n) {
  if (!plan || !order) return fail(TN_E_INVALID, "NULL argument");
  const tn::Plan& p = plan->p;
  if (n < (int32_t)p.sched.size()) return fail(TN_E_INVALID, "order array too short");
  for (size_t i = 0; i < p.sched.size(); ++i) order[i] = p.sched[i];
  return TN_OK;
}

tn_status tn_contract(tn_plan_t plan, const void* const* leaves, const int64_t* slice_ids,
                      int64_t n_slice_ids, int32_t out_mode, void* out, void* ws,
                      size_t ws_bytes, void* stream) {
  return contract_impl(plan, leaves, slice_ids, n_slice_ids, out_mode, out, ws, ws_bytes, stream,
                       nullptr);
}

tn_status tn_contract_ex(tn_plan_t plan, const void* const* leaves, const int64_t* slice_ids,
                         int64_t n_slice_ids, int32_t out_mode, void* out, void* ws,
                         size_t ws_bytes, void* stream, uint32_t call_flags) {
  return contract_impl(plan, leaves, slice_ids, n_slice_ids, out_mode, out, ws, ws_bytes, stream,
                       nullptr, call_flags);
}

tn_status tn_contract_probe(tn_plan_t plan, const void* const* leaves, const int64_t* slice_ids,
                            int64_t n_slice_ids, int32_t out_mode, void* out, void* ws,
                            size_t ws_bytes, void* stream, int32_t probe_step, void* ev_start,
                            void* ev_stop) {
  if (!plan) return fail(TN_E_INVALID, "NULL plan");
  if (probe_step < 0 || probe_step >= plan->p.n_tensors - 1 || !ev_start || !ev_stop)
    return fail(TN_E_INVALID, "bad probe step or events");
  Probe pr;
  pr.step = probe_step;
  pr.start = static_cast<hipEvent_t>(ev_start);
  pr.stop = static_cast<hipEvent_t>(ev_stop);
  return contract_impl(plan, leaves, slice_ids, n_slice_ids, out_mode, out, ws, ws_bytes, stream,
                       &pr);
}

}  // extern "C"

static tn_status contract_impl(tn_plan_t plan, const void* const* leaves, const int64_t* slice_ids,
                        int64_t n_slice_ids, int32_t out_mode, void* out, void* ws,
                        size_t ws_bytes, void* stream, Probe* probe, uint32_t call_flags) {
  if (!plan || !leaves || !out) return fail(TN_E_INVALID, "NULL argument");
  const tn::Plan& p = plan->p;
  if (out_mode != TN_OUT_SUM && out_mode != TN_OUT_PER_SLICE)
    return fail(TN_E_INVALID, "unknown out_mode");
  if ((call_flags & ~TN_CALL_REUSE_INVARIANT) != 0) return fail(TN_E_INVALID, "unknown call flag");
  if ((call_flags & TN_CALL_REUSE_INVARIANT) &&
      std::find(p.leaf_variable.begin(), p.leaf_variable.end(), 1) == p.leaf_variable.end())
    return fail(TN_E_INVALID, "TN_CALL_REUSE_INVARIANT needs a plan with variable leaves");
  if ((int64_t)ws_bytes < p.workspace_bytes || (!ws && p.workspace_bytes > 0))
    return fail(TN_E_WORKSPACE, "workspace smaller than tn_plan_info.workspace_bytes");
  if (n_slice_ids < 0 || (n_slice_ids > 0 && !slice_ids))
    return fail(TN_E_INVALID, "bad slice list");
  for (int t = 0; t < p.n_tensors; ++t)
    if (!leaves[t]) return fail(TN_E_INVALID, "NULL leaf pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ctx c{p, leaves, static_cast<char*>(ws),
        reinterpret_cast<float2*>(static_cast<char*>(ws) + ((p.arena_bytes + 255) / 256) * 256), st};
  const int64_t n_out = (int64_t)1 << p.open_bits;

  // which (outer iteration, resident slice, row) triples are requested
  const bool all = (n_slice_ids == 0);
  std::map<uint64_t, std::vector<std::pair<int32_t, int32_t>>> sel;   // it -> (r, row)
  if (!all) {
    for (int64_t i = 0; i < n_slice_ids; ++i) {
      int64_t s = slice_ids[i];
      if (s < 0 || s >= p.n_slices) return fail(TN_E_INVALID, "slice id out of range");
      uint64_t it = 0, r = 0;
      for (int j = 0; j < p.outer_bits; ++j) it |= (uint64_t)((s >> p.outer_slicebit[j]) & 1) << j;
      for (int j = 0; j < p.resident_bits; ++j) r |= (uint64_t)((s >> p.res_slicebit[j]) & 1) << j;
      sel[it].push_back({(int32_t)r, (int32_t)i});
    }
  }
  double2* outp = static_cast<double2*>(out);
  if (out_mode == TN_OUT_SUM) {
    hipLaunchKernelGGL(tnk::k_fill_c128, dim3(grid_for(n_out)), dim3(tnk::kBlock), 0, st, outp,
                       n_out);
    TN_HIP_CHECK(hipGetLastError());
  }
  // persistent segments: descriptors for every execution, one upload
  std::vector<std::vector<SegLayout>> lay;
  std::vector<int32_t> seg_at(p.sched.size(), -1);
  char* pbase = c.ws + al256(p.arena_bytes) + al256(p.scratch_bytes) + p.ctrl_bytes;
  // The tables are copied from host memory; the copy may still read the
  // host buffer after hipMemcpyAsync returns, so the buffer lives until the
  // stream has passed the copy (StagedUpload synchronises on every exit).
  StagedUpload upload;
  upload.st = st;
  if (!p.segments.empty()) {
    build_persist_blob(c, upload.buf, lay);
    TN_HIP_CHECK(hipMemcpyAsync(pbase, upload.buf.data(), upload.buf.size(),
                                hipMemcpyHostToDevice, st));
    upload.queued = true;
    for (size_t gi = 0; gi < p.segments.size(); ++gi) seg_at[p.segments[gi].begin] = (int32_t)gi;
  }
  std::vector<int32_t> tiny_at(p.sched.size(), -1);
  for (size_t ti = 0; ti < p.tiny_runs.size(); ++ti) tiny_at[p.tiny_runs[ti].begin] = (int32_t)ti;
  auto run_range = [&](size_t from, size_t to, uint64_t it) -> tn_status {
    for (size_t i = from; i < to;) {
      if (tiny_at[i] >= 0) {   // a batch of tiny steps (inside one group, so inside the range)
        const tn::Segment& g = p.tiny_runs[tiny_at[i]];
        tn_status s = launch_tiny(c, g, it, probe);
        if (s != TN_OK) return s;
        i = g.end;
        continue;
      }
      const int32_t gi = seg_at[i];
      if (gi >= 0) {
        const tn::Segment& g = p.segments[gi];
        bool timed = false;
        if (probe && !probe->done)
          for (int q = g.begin; q < g.end; ++q) timed |= p.sched[q] == probe->step;
        if (timed) TN_HIP_CHECK(hipEventRecord(probe->start, st));
        tn_status s = launch_segment(c, g, lay[gi][g.phase ? it : 0], pbase);
        if (s != TN_OK) return s;
        if (timed) {
          TN_HIP_CHECK(hipEventRecord(probe->stop, st));
          probe->done = true;
        }
        i = g.end;
        continue;
      }
      const tn::StepDesc& S = p.steps[p.sched[i]];
      if (S.chain >= 0 && !(p.flags & 64u)) {   // a chain runs at the position of its last step
        const tn::ChainGroup& g = p.chains[S.chain];
        if (g.last == p.sched[i]) {
          tn_status s = run_chain(c, g, it, probe);
          if (s != TN_OK) return s;
        }
        ++i;
        continue;
      }
      tn_status s = run_step(c, p.sched[i], it, probe);
      if (s != TN_OK) return s;
      ++i;
    }
    return TN_OK;
  };
  // shared work: steps that depend on no outer index, once (the invariant
  // ones only if their results are not kept from an earlier call)
  {
    const bool reuse = (call_flags & TN_CALL_REUSE_INVARIANT) != 0;
    tn_status s = run_range(reuse ? p.n_invariant : 0, p.n_phase0, 0);
    if (s != TN_OK) return s;
  }
  const uint64_t n_it = 1ull << p.outer_bits;
  const int root_step = p.n_tensors - 2;
  for (uint64_t it = 0; it < n_it; ++it) {
    if (!all && sel.find(it) == sel.end()) continue;
    {
      tn_status s = run_range(p.n_phase0, p.sched.size(), it);
      if (s != TN_OK) return s;
    }
    tnk::SumArgs sa;
    memset(&sa, 0, sizeof sa);
    if (p.n_tensors == 1) {
      sa.root = static_cast<const float2*>(leaves[0]);
    } else {
      sa.root = reinterpret_cast<const float2*>(c.ws + p.steps[root_step].c_off);
    }
    sa.out = outp;
    sa.open_bits = p.open_bits;
    sa.res_bits = p.resident_bits;
    sa.mode = out_mode;
    copy_bits(sa.s_open, p.root_open_log2);
    copy_bits(sa.s_res, p.root_res_log2);
    for (int j = 0; j < p.resident_bits; ++j) sa.res_slicebit[j] = (int8_t)p.res_slicebit[j];
    int64_t base = 0;
    for (int j = 0; j < p.outer_bits; ++j) base |= (int64_t)((it >> j) & 1) << p.outer_slicebit[j];
    sa.row_base = base;
    if (all) {
      sa.n_sel = -1;
      hipLaunchKernelGGL(tnk::k_slice_sum, dim3(grid_for(n_out)), dim3(tnk::kBlock), 0,
                         st, sa);
      TN_HIP_CHECK(hipGetLastError());
    } else {
      const auto& v = sel[it];
      for (size_t i0 = 0; i0 < v.size(); i0 += tnk::kMaxSel) {
        size_t cnt = std::min(v.size() - i0, (size_t)tnk::kMaxSel);
        sa.n_sel = (int32_t)cnt;
        for (size_t i = 0; i < cnt; ++i) {
          sa.sel_r[i] = v[i0 + i].first;
          sa.sel_row[i] = v[i0 + i].second;
        }
        hipLaunchKernelGGL(tnk::k_slice_sum, dim3(grid_for(n_out)), dim3(tnk::kBlock),
                           0, st, sa);
        TN_HIP_CHECK(hipGetLastError());
      }
    }
  }
  if (!p.segments.empty()) {
    // a segment wait that timed out skipped its item's arithmetic: the
    // result is wrong, so the call fails
    int32_t err_word = 0;
    TN_HIP_CHECK(hipMemcpyAsync(&err_word, pbase, sizeof err_word, hipMemcpyDeviceToHost, st));
    TN_HIP_CHECK(hipStreamSynchronize(st));
    upload.queued = false;
    if (err_word != 0)
      return fail(TN_E_HIP, "a persistent segment wait timed out; the result is invalid");
  }
  return TN_OK;
}

struct tn_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~tn_graph_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// Records the launches `body` makes on an internal non-blocking stream
// (default priority) into a graph and instantiates it; nothing runs.
static tn_status capture_graph(const std::function<tn_status(hipStream_t)>& body,
                               tn_graph_t* graph) {
  hipStream_t cs = nullptr;
  TN_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  tn_graph_s* g = nullptr;
  try {
    g = new tn_graph_s();
  } catch (const std::bad_alloc&) {
    (void)hipStreamDestroy(cs);
    return fail(TN_E_OOM, "host allocation failed");
  }
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete g;
    (void)hipStreamDestroy(cs);
    return fail(TN_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  tn_status s = body(cs);
  hipGraph_t captured = nullptr;
  e = hipStreamEndCapture(cs, &captured);   // ends the capture on every path
  (void)hipStreamDestroy(cs);
  g->graph = captured;
  if (s != TN_OK) {
    delete g;
    return s;   // tn_last_error holds the body's message
  }
  if (e != hipSuccess || !captured) {
    delete g;
    return fail(TN_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    delete g;
    return fail(TN_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  *graph = g;
  return TN_OK;
}

tn_status tn_graph_create(tn_plan_t plan, const void* const* leaves, const int64_t* slice_ids,
                          int64_t n_slice_ids, int32_t out_mode, void* out, void* ws,
                          size_t ws_bytes, void* stream, tn_graph_t* graph) {
  (void)stream;
  if (!graph) return fail(TN_E_INVALID, "graph is NULL");
  *graph = nullptr;
  if (!plan) return fail(TN_E_INVALID, "NULL plan");
  if (!plan->p.segments.empty())
    return fail(TN_E_UNSUPPORTED, "plans with persistent segments are not captured");
  return capture_graph(
      [&](hipStream_t cs) {
        return contract_impl(plan, leaves, slice_ids, n_slice_ids, out_mode, out, ws, ws_bytes,
                             cs, nullptr);
      },
      graph);
}

tn_status tn_graph_launch(tn_graph_t graph, void* stream) {
  if (!graph || !graph->exec) return fail(TN_E_INVALID, "NULL graph");
  TN_HIP_CHECK(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
  return TN_OK;
}

void tn_graph_destroy(tn_graph_t graph) { delete graph; }

// Workspace of tn_contract_noalloc: a file-scope device array, one copy per
// GPU the library runs on, held until the process ends.  Host code never
// passes the array's name to a kernel or a copy: on each device its address
// comes from hipGetSymbolAddress, taken once with that device current.
static __device__ __align__(256) char scratch[TN_NOALLOC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

tn_status scratch_on_current_device(void** out) {
  int dev = -1;
  TN_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TN_E_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(TN_E_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TN_OK;
}
}  // namespace

extern "C" {

tn_status tn_contract_noalloc(tn_plan_t plan, const void* const* leaves, const int64_t* slice_ids,
                              int64_t n_slice_ids, int32_t out_mode, void* out, void* stream) {
  if (!plan) return fail(TN_E_INVALID, "NULL plan");
  if (plan->p.workspace_bytes > (int64_t)TN_NOALLOC_WORKSPACE_BYTES)
    return fail(TN_E_WORKSPACE,
                "plan needs " + std::to_string(plan->p.workspace_bytes) +
                    " workspace bytes; tn_contract_noalloc holds at most " +
                    std::to_string((long long)TN_NOALLOC_WORKSPACE_BYTES));
  void* ws = nullptr;
  tn_status s = scratch_on_current_device(&ws);
  if (s != TN_OK) return s;
  return contract_impl(plan, leaves, slice_ids, n_slice_ids, out_mode, out, ws,
                       (size_t)TN_NOALLOC_WORKSPACE_BYTES, stream, nullptr);
}

}  // extern "C"

extern "C" {

static tn_status backward_impl(tn_plan_t plan, const void* const* leaves, const void* grad_out,
                               void* const* grad_leaves, const int64_t* slice_ids,
                               int64_t n_slice_ids, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !leaves || !grad_out || !grad_leaves) return fail(TN_E_INVALID, "NULL argument");
  const tn::Plan& p = plan->p;
  const tn::BwdPlan& B = p.bwd;
  if ((int64_t)ws_bytes < p.workspace_bwd_bytes || !ws)
    return fail(TN_E_WORKSPACE, "workspace smaller than tn_plan_info.workspace_backward_bytes");
  if (n_slice_ids < 0 || (n_slice_ids > 0 && !slice_ids))
    return fail(TN_E_INVALID, "bad slice list");
  for (int t = 0; t < p.n_tensors; ++t)
    if (!leaves[t]) return fail(TN_E_INVALID, "NULL leaf pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* W = static_cast<char*>(ws);
  const int n = p.n_tensors;
  // selected resident slices per outer iteration, with multiplicity
  const bool all = n_slice_ids == 0;
  std::map<uint64_t, std::map<int32_t, int32_t>> sel;
  for (int64_t i = 0; i < n_slice_ids; ++i) {
    const int64_t s = slice_ids[i];
    if (s < 0 || s >= p.n_slices) return fail(TN_E_INVALID, "slice id out of range");
    uint64_t it = 0, r = 0;
    for (int j = 0; j < p.outer_bits; ++j) it |= (uint64_t)((s >> p.outer_slicebit[j]) & 1) << j;
    for (int j = 0; j < p.resident_bits; ++j) r |= (uint64_t)((s >> p.res_slicebit[j]) & 1) << j;
    sel[it][(int32_t)r]++;
  }
  if (n == 1) {   // the output is the leaf itself
    if (!grad_leaves[0]) return TN_OK;
    tnk::RootGradArgs rg;
    memset(&rg, 0, sizeof rg);
    rg.grad_out = static_cast<const double2*>(grad_out);
    rg.dst = static_cast<float2*>(grad_leaves[0]);
    rg.open_bits = p.open_bits;
    rg.accumulate = 1;
    rg.n_sel = -1;
    copy_bits(rg.s_open, p.root_open_log2);
    hipLaunchKernelGGL(tnk::k_root_grad, dim3(grid_for(1ull << p.open_bits)), dim3(tnk::kBlock),
                       0, st, rg);
    TN_HIP_CHECK(hipGetLastError());
    return TN_OK;
  }
  float2* scratch = reinterpret_cast<float2*>(W + al256(B.arena_bytes));
  Ctx c{p, leaves, W, scratch, st};
  const int root = n + (n - 1) - 1;
  // tiny products go out in batches (TN_FLAG_NO_TINY: one launch each)
  TinyBatcher tb(st, !(p.flags & 512u));
  auto issue = [&](int32_t kind, int32_t chunks, int32_t tile,
                   const tnk::StepArgs& a) -> tn_status {
    if (tb.fits(a, kind, chunks)) return tb.add(a);
    tn_status s = tb.flush();
    if (s != TN_OK) return s;
    return launch_step(kind, chunks, tile, a, scratch, p.precision, st, (p.flags & 1024u) != 0);
  };
  auto at = [&](int64_t off) { return reinterpret_cast<float2*>(W + off); };
  // value of node x: a leaf (offset for the outer iteration), or the stored /
  // recomputed result (rec: inside a block's adjoint, where values the block
  // both produces and consumes live at their recomputed offsets)
  auto val = [&](int x, uint64_t it, bool rec) -> float2* {
    if (x < n)
      return const_cast<float2*>(static_cast<const float2*>(leaves[x])) + leaf_outer_off(p, x, it);
    return at(rec && B.keep[x] == 0 ? B.rec_off[x] : B.fwd_off[x]);
  };
  auto grad = [&](int x, uint64_t it) -> float2* {
    if (x < n)
      return grad_leaves[x] ? static_cast<float2*>(grad_leaves[x]) + leaf_outer_off(p, x, it)
                            : nullptr;
    return at(B.grad_off[x]);
  };
  auto launch_fwd = [&](const tn::StepDesc& S, float2* A, float2* Bp, float2* C) {
    tnk::StepArgs a = make_args(S);
    a.A = A;
    a.B = Bp;
    a.C = C;
    return issue(S.kind, S.splitk_chunks, S.tile, a);
  };
  auto forward = [&](int q0, int q1, uint64_t it) -> tn_status {
    for (int q = q0; q < q1; ++q) {
      const int k = p.sched[q];
      const tn::StepDesc& S = p.steps[k];
      const bool fused = S.chain >= 0 && B.fuse_chain[S.chain];
      if (!fused && n + k == root) continue;   // the output value itself is not needed
      if (fused) {
        const tn::ChainGroup& g = p.chains[S.chain];
        if (g.last != k) continue;
        tn_status s = tb.flush();
        if (s != TN_OK) return s;
        s = run_chain_with(
            c, g, [&](int x) -> const float2* { return val(x, it, false); },
            at(B.fwd_off[n + k]), nullptr);
        if (s != TN_OK) return s;
        continue;
      }
      tn_status s = launch_fwd(S, val(S.a, it, false), val(S.b, it, false), at(B.fwd_off[n + k]));
      if (s != TN_OK) return s;
    }
    return TN_OK;
  };
  auto fill0 = [&](float2* dst, int64_t elems) -> tn_status {
    tn_status s = tb.flush();
    if (s != TN_OK) return s;
    hipLaunchKernelGGL(tnk::k_fill_c64, dim3(grid_for((uint64_t)elems, 1u << 20)),
                       dim3(tnk::kBlock), 0, st, dst, elems);
    TN_HIP_CHECK(hipGetLastError());
    return TN_OK;
  };
  // gradient of the root for one outer iteration: the output gradient at
  // every selected resident slice (times its multiplicity), zero elsewhere
  auto root_grad = [&](uint64_t it) -> tn_status {
    tn_status s = tb.flush();
    if (s != TN_OK) return s;
    tnk::RootGradArgs rg;
    memset(&rg, 0, sizeof rg);
    rg.grad_out = static_cast<const double2*>(grad_out);
    rg.dst = at(B.grad_off[root]);
    rg.open_bits = p.open_bits;
    rg.res_bits = p.resident_bits;
    copy_bits(rg.s_open, p.root_open_log2);
    copy_bits(rg.s_res, p.root_res_log2);
    const uint64_t n_all = 1ull << (p.open_bits + p.resident_bits);
    if (all) {
      rg.n_sel = -1;
      hipLaunchKernelGGL(tnk::k_root_grad, dim3(grid_for(n_all)), dim3(tnk::kBlock), 0, st, rg);
      TN_HIP_CHECK(hipGetLastError());
      return TN_OK;
    }
    s = fill0(rg.dst, (int64_t)n_all);
    if (s != TN_OK) return s;
    std::vector<std::pair<int32_t, int32_t>> v(sel[it].begin(), sel[it].end());
    for (size_t i0 = 0; i0 < v.size(); i0 += tnk::kMaxSel) {
      const size_t cnt = std::min(v.size() - i0, (size_t)tnk::kMaxSel);
      rg.n_sel = (int32_t)cnt;
      for (size_t i = 0; i < cnt; ++i) {
        rg.sel_r[i] = v[i0 + i].first;
        rg.sel_w[i] = (float)v[i0 + i].second;
      }
      hipLaunchKernelGGL(tnk::k_root_grad, dim3(grid_for((uint64_t)cnt << p.open_bits)),
                         dim3(tnk::kBlock), 0, st, rg);
      TN_HIP_CHECK(hipGetLastError());
    }
    return TN_OK;
  };
  // adjoint products of one step: dA (+)= dC . B^H, dB (+)= A^H . dC
  auto adjoint_step = [&](const tn::StepDesc& S, uint64_t it) -> tn_status {
    float2* gC = grad(S.c, it);
    const int nb = (int)S.bA.size(), nm = (int)S.mA.size(), nn = (int)S.nB.size(),
              nk = (int)S.kA.size();
    float2* dA = grad(S.a, it);
    float2* dB = grad(S.b, it);
    auto acc = [&](int x) { return x < n || B.frontier[x] ? 1 : 0; };
    if (dA) {
      tnk::StepArgs a;
      memset(&a, 0, sizeof a);
      a.nb = nb; a.nm = nm; a.nn = nk; a.nk = nn;
      copy_bits(a.sA_b, S.bC); copy_bits(a.sA_m, S.mC); copy_bits(a.sA_k, S.nC);
      copy_bits(a.sB_b, S.bB); copy_bits(a.sB_k, S.nB); copy_bits(a.sB_n, S.kB);
      copy_bits(a.sC_b, S.bA); copy_bits(a.sC_m, S.mA); copy_bits(a.sC_n, S.kA);
      a.A = gC;
      a.B = val(S.b, it, true);
      a.C = dA;
      a.conjB = 1;
      a.accumulate = acc(S.a);
      int32_t ch;
      int64_t scr;
      int32_t kind = tn::choose_kind(a.nb, a.nm, a.nn, a.nk, p.flags, &ch, &scr);
      int32_t tile = kind == tn::KIND_GEMM ? tn::choose_tile(p, a.nm, a.nn, a.nk) : -1;
      tn_status s = issue(kind, ch, tile, a);
      if (s != TN_OK) return s;
    }
    if (dB) {
      tnk::StepArgs a;
      memset(&a, 0, sizeof a);
      a.nb = nb; a.nm = nk; a.nn = nn; a.nk = nm;
      copy_bits(a.sA_b, S.bA); copy_bits(a.sA_m, S.kA); copy_bits(a.sA_k, S.mA);
      copy_bits(a.sB_b, S.bC); copy_bits(a.sB_k, S.mC); copy_bits(a.sB_n, S.nC);
      copy_bits(a.sC_b, S.bB); copy_bits(a.sC_m, S.kB); copy_bits(a.sC_n, S.nB);
      a.A = val(S.a, it, true);
      a.B = gC;
      a.C = dB;
      a.conjA = 1;
      a.accumulate = acc(S.b);
      int32_t ch;
      int64_t scr;
      int32_t kind = tn::choose_kind(a.nb, a.nm, a.nn, a.nk, p.flags, &ch, &scr);
      int32_t tile = kind == tn::KIND_GEMM ? tn::choose_tile(p, a.nm, a.nn, a.nk) : -1;
      tn_status s = issue(kind, ch, tile, a);
      if (s != TN_OK) return s;
    }
    return TN_OK;
  };
  // adjoint of the blocks of [q0, q1), last block first
  auto adjoint = [&](int q0, int q1, uint64_t it) -> tn_status {
    std::vector<std::pair<int, int>> bl;
    for (int q = q0; q < q1;) {
      int e = q;
      while (e < q1 && B.block_of[e] == B.block_of[q]) ++e;
      bl.push_back({q, e});
      q = e;
    }
    for (int bi = (int)bl.size() - 1; bi >= 0; --bi) {
      const int b0 = bl[bi].first, b1 = bl[bi].second;
      for (int q = b0; q < b1; ++q) {   // recompute what the block produces and consumes
        const tn::StepDesc& S = p.steps[p.sched[q]];
        if (B.keep[S.c] != 0) continue;
        tn_status s = launch_fwd(S, val(S.a, it, true), val(S.b, it, true), at(B.rec_off[S.c]));
        if (s != TN_OK) return s;
      }
      for (int q = b1 - 1; q >= b0; --q) {
        tn_status s = adjoint_step(p.steps[p.sched[q]], it);
        if (s != TN_OK) return s;
      }
    }
    return TN_OK;
  };
  const int n0 = p.n_phase0, N = (int)p.sched.size();
  tn_status s = forward(0, n0, 0);
  if (s != TN_OK) return s;
  if (n0 < N) {
    for (int v = n; v <= root; ++v)
      if (B.frontier[v]) {
        s = fill0(at(B.grad_off[v]), p.steps[v - n].c_bytes / 8);
        if (s != TN_OK) return s;
      }
    const uint64_t n_it = 1ull << p.outer_bits;
    for (uint64_t it = 0; it < n_it; ++it) {
      if (!all && sel.find(it) == sel.end()) continue;
      if ((s = forward(n0, N, it)) != TN_OK) return s;
      if ((s = root_grad(it)) != TN_OK) return s;
      if ((s = adjoint(n0, N, it)) != TN_OK) return s;
    }
  } else {
    if (!all && sel.find(0) == sel.end()) {
      // nothing selected: every gradient is zero (leaf gradients unchanged)
      return tb.flush();
    }
    if ((s = root_grad(0)) != TN_OK) return s;
  }
  if ((s = adjoint(0, n0, 0)) != TN_OK) return s;
  return tb.flush();
}

tn_status tn_contract_backward(tn_plan_t plan, const void* const* leaves, const void* grad_out,
                               void* const* grad_leaves, const int64_t* slice_ids,
                               int64_t n_slice_ids, void* ws, size_t ws_bytes, void* stream) {
  return backward_impl(plan, leaves, grad_out, grad_leaves, slice_ids, n_slice_ids, ws, ws_bytes,
                       stream);
}

tn_status tn_graph_create_backward(tn_plan_t plan, const void* const* leaves,
                                   const void* grad_out, void* const* grad_leaves,
                                   const int64_t* slice_ids, int64_t n_slice_ids, void* ws,
                                   size_t ws_bytes, void* stream, tn_graph_t* graph) {
  (void)stream;
  if (!graph) return fail(TN_E_INVALID, "graph is NULL");
  *graph = nullptr;
  if (!plan) return fail(TN_E_INVALID, "NULL plan");
  return capture_graph(
      [&](hipStream_t cs) {
        return backward_impl(plan, leaves, grad_out, grad_leaves, slice_ids, n_slice_ids, ws,
                             ws_bytes, cs);
      },
      graph);
}

tn_status tn_permute(const void* in, void* out, int32_t nbits, const int8_t* in_log2,
                     const int8_t* out_log2, void* stream) {
  if (!in || !out || !in_log2 || !out_log2) return fail(TN_E_INVALID, "NULL argument");
  if (nbits < 0 || nbits > 40) return fail(TN_E_INVALID, "nbits out of range");
  uint64_t seen_in = 0, seen_out = 0;
  for (int j = 0; j < nbits; ++j) {
    if (in_log2[j] < 0 || in_log2[j] >= nbits || out_log2[j] < 0 || out_log2[j] >= nbits)
      return fail(TN_E_INVALID, "stride outside the tensor");
    seen_in |= 1ull << in_log2[j];
    seen_out |= 1ull << out_log2[j];
  }
  uint64_t full = nbits == 64 ? ~0ull : ((1ull << nbits) - 1);
  if (seen_in != full || seen_out != full) return fail(TN_E_INVALID, "strides are not a permutation");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (nbits < 10) {   // at most 512 elements: one element per thread
    tnk::PermArgs a;
    memset(&a, 0, sizeof a);
    a.in = static_cast<const float2*>(in);
    a.out = static_cast<float2*>(out);
    a.nbits = nbits;
    for (int j = 0; j < nbits; ++j) {
      a.sin[j] = in_log2[j];
      a.sout[j] = out_log2[j];
    }
    hipLaunchKernelGGL(tnk::k_permute_plain, dim3(grid_for(1ull << nbits)), dim3(tnk::kBlock),
                       0, st, a);
  } else {
    tnk::PermTileArgs a;
    memset(&a, 0, sizeof a);
    a.in = static_cast<const float2*>(in);
    a.out = static_cast<float2*>(out);
    const int tb = nbits >= 12 ? 12 : 10, half = tb / 2;
    // tile bits: every bit with an input or output stride below 2^half, then
    // further bits by smallest stride until the tile has tb bits
    std::vector<int> tile, rest;
    for (int j = 0; j < nbits; ++j)
      if (in_log2[j] < half || out_log2[j] < half) tile.push_back(j);
    std::vector<int> others;
    for (int j = 0; j < nbits; ++j)
      if (!(in_log2[j] < half || out_log2[j] < half)) others.push_back(j);
    std::sort(others.begin(), others.end(), [&](int x, int y) {
      return std::min(in_log2[x], out_log2[x]) < std::min(in_log2[y], out_log2[y]);
    });
    for (int j : others) ((int)tile.size() < tb ? tile : rest).push_back(j);
    std::vector<int> rd = tile, wr = tile;
    std::sort(rd.begin(), rd.end(), [&](int x, int y) { return in_log2[x] < in_log2[y]; });
    std::sort(wr.begin(), wr.end(), [&](int x, int y) { return out_log2[x] < out_log2[y]; });
    std::sort(rest.begin(), rest.end(), [&](int x, int y) { return in_log2[x] < in_log2[y]; });
    a.tbits = tb;
    a.rbits = (int)rest.size();
    a.half = half;
    for (int p = 0; p < tb; ++p) {
      a.rin[p] = in_log2[rd[p]];
      a.wout[p] = out_log2[wr[p]];
      a.wpos[p] = (int8_t)(std::find(rd.begin(), rd.end(), wr[p]) - rd.begin());
    }
    for (int q = 0; q < a.rbits; ++q) {
      a.tin[q] = in_log2[rest[q]];
      a.tout[q] = out_log2[rest[q]];
    }
    const uint64_t n_tiles = 1ull << a.rbits;
    const unsigned grid = (unsigned)std::min<uint64_t>(n_tiles, 1u << 16);
    if (tb == 12)
      hipLaunchKernelGGL(tnk::k_permute_tile<12>, dim3(grid), dim3(tnk::kBlock), 0, st, a);
    else
      hipLaunchKernelGGL(tnk::k_permute_tile<10>, dim3(grid), dim3(tnk::kBlock), 0, st, a);
  }
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

}  // extern "C"
