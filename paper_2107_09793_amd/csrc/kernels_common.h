// Shared device-side definitions for the contraction kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tnk {

constexpr int kMaxBits = 48;

// One pairwise contraction C[b,m,n] (+)= sum_k op(A)[b,m,k] op(B)[b,k,n].
// Every index is a set of bits; each bit has a power-of-two stride (log2, in
// complex elements) in each operand that carries it.  Index bit j of m is
// the j-th entry of sA_m / sC_m, and so on.
struct StepArgs {
  const float2* A;
  const float2* B;
  float2* C;
  float2* scratch;       // split-k partials
  int32_t nb, nm, nn, nk;
  int32_t conjA, conjB;  // use conj(A) / conj(B)
  int32_t accumulate;    // C += result instead of C = result
  int32_t chunk_log2;    // split-k: log2 of k values per chunk
  int8_t sA_b[kMaxBits], sB_b[kMaxBits], sC_b[kMaxBits];
  int8_t sA_m[kMaxBits], sC_m[kMaxBits];
  int8_t sB_n[kMaxBits], sC_n[kMaxBits];
  int8_t sA_k[kMaxBits], sB_k[kMaxBits];
};

// Offset of the element whose index bits (lsb first) are ``idx`` given the
// log2 strides of those bits.
__device__ __forceinline__ int64_t scatter(uint64_t idx, const int8_t* s, int nbits) {
  int64_t off = 0;
  for (int j = 0; j < nbits; ++j) off += (int64_t)((idx >> j) & 1ull) << s[j];
  return off;
}

// Offset of index ``idx`` restricted to bits [lo, hi).
__device__ __forceinline__ int64_t scatter_range(uint64_t idx, const int8_t* s, int lo, int hi) {
  int64_t off = 0;
  for (int j = lo; j < hi; ++j) off += (int64_t)((idx >> j) & 1ull) << s[j];
  return off;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// acc += a * b (complex), four fused multiply-adds
__device__ __forceinline__ void cfma(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
}

__device__ __forceinline__ float2 maybe_conj(float2 v, int c) {
  return c ? make_float2(v.x, -v.y) : v;
}

// sum over k < 2^nk of A[oa + off_A(k)] B[ob + off_B(k)] (each operand
// conjugated on request), accumulated in increasing k.  The operands of 8
// consecutive k are loaded before their products, so a thread waits on
// memory once per 8 values of k instead of once per value; the order of the
// sum is that of the plain loop.
__device__ __forceinline__ float2 dot_k(const float2* A, int64_t oa, const int8_t* sA_k, int conjA,
                                        const float2* B, int64_t ob, const int8_t* sB_k, int conjB,
                                        int nk) {
  float2 acc = make_float2(0.f, 0.f);
  if (nk < 3) {
    for (uint32_t k = 0; k < (1u << nk); ++k)
      cfma(acc, maybe_conj(A[oa + scatter(k, sA_k, nk)], conjA),
           maybe_conj(B[ob + scatter(k, sB_k, nk)], conjB));
    return acc;
  }
  int64_t la[8], lb[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    la[u] = scatter(u, sA_k, 3);
    lb[u] = scatter(u, sB_k, 3);
  }
  const uint64_t K = 1ull << nk;
  for (uint64_t k = 0; k < K; k += 8) {
    const int64_t ha = oa + scatter_range(k, sA_k, 3, nk);
    const int64_t hb = ob + scatter_range(k, sB_k, 3, nk);
    float2 a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = A[ha + la[u]];
      b[u] = B[hb + lb[u]];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) cfma(acc, maybe_conj(a[u], conjA), maybe_conj(b[u], conjB));
  }
  return acc;
}

}  // namespace tnk
