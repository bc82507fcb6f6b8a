// Persistent executor for runs of small contraction steps.
//
// The many small steps of a contraction path (gate absorptions into small
// tensors, the shared prefix of every slice) would each cost a kernel launch.
// Here one launch runs a whole segment of them: workgroups claim work items
// -- (step, chunk of 256 outputs) -- from a global ticket in topological
// order, wait until the producer steps of their operands inside the segment
// have completed every item (agent-scope acquire), compute, and publish
// their item (agent-scope release).  An item only ever waits on items with
// smaller tickets, which were claimed by workgroups that are already running,
// so the segment always drains; each wait is also bounded and reports
// through an error word instead of spinning forever.
#pragma once

#include "kernels_common.h"

namespace tnk {

constexpr int kSmallBits = 24;   // bits of one class in a small step
constexpr int kSpinLimit = 1 << 16;
constexpr int kCtrStride = 32;   // counters 128 bytes apart: no shared cache line

struct SmallStep {
  const float2* A;
  const float2* B;
  float2* C;
  int32_t nb, nm, nn, nk;
  int32_t n_items, item0;   // work items of this step and the first one's ticket
  int32_t dep0, dep1;       // segment-local producer steps (-1: none in segment)
  int8_t sA_b[kSmallBits], sB_b[kSmallBits], sC_b[kSmallBits];
  int8_t sA_m[kSmallBits], sC_m[kSmallBits];
  int8_t sB_n[kSmallBits], sC_n[kSmallBits];
  int8_t sA_k[kSmallBits], sB_k[kSmallBits];
};

__device__ __forceinline__ int64_t scat_small(uint64_t idx, const int8_t* s, int n) {
  int64_t off = 0;
#pragma unroll 1
  for (int j = 0; j < n; ++j) off += (int64_t)((idx >> j) & 1ull) << s[j];
  return off;
}

// Poll with exponential backoff (s_sleep 1..64, about 64..4096 cycles) so a
// crowd of waiting workgroups does not saturate the counter's memory channel.
__device__ __forceinline__ bool wait_done(int32_t* cnt, int32_t need) {
  int spins = 0, nap = 1;
  while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
    if (nap == 1) __builtin_amdgcn_s_sleep(1);
    else if (nap == 2) __builtin_amdgcn_s_sleep(2);
    else if (nap <= 8) __builtin_amdgcn_s_sleep(8);
    else __builtin_amdgcn_s_sleep(64);
    nap = nap < 16 ? 2 * nap : 16;
    if (++spins > kSpinLimit) return false;
  }
  return true;
}

// ctr[0]: ticket; ctr[kCtrStride * (1 + s)]: completed items of segment step
// s; err[0]: set to 1 if a wait timed out.
__global__ void __launch_bounds__(256) k_persistent(const SmallStep* __restrict__ steps,
                                                    const int32_t* __restrict__ item_step,
                                                    int32_t n_items, int32_t* ctr, int32_t* err) {
  __shared__ int32_t s_item;
  __shared__ int32_t s_ok;
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(&ctr[0], 1);
    __syncthreads();
    const int32_t it = s_item;
    if (it >= n_items) return;
    const int32_t s = item_step[it];
    const SmallStep& S = steps[s];
    if (threadIdx.x == 0) {
      bool ok = true;
      if (S.dep0 >= 0) ok = ok && wait_done(&ctr[kCtrStride * (1 + S.dep0)], steps[S.dep0].n_items);
      if (S.dep1 >= 0) ok = ok && wait_done(&ctr[kCtrStride * (1 + S.dep1)], steps[S.dep1].n_items);
      if (!ok) atomicOr(err, 1);
      s_ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every wave sees the producers' data
    const int nb = S.nb, nm = S.nm, nn = S.nn, nk = S.nk;
    const uint64_t n_out = 1ull << (nb + nm + nn);
    const uint64_t o = (uint64_t)(it - S.item0) * 256 + threadIdx.x;
    if (s_ok && o < n_out) {
      const uint64_t n = o & ((1ull << nn) - 1);
      const uint64_t m = (o >> nn) & ((1ull << nm) - 1);
      const uint64_t b = o >> (nn + nm);
      const int64_t oa = scat_small(m, S.sA_m, nm) + scat_small(b, S.sA_b, nb);
      const int64_t ob = scat_small(n, S.sB_n, nn) + scat_small(b, S.sB_b, nb);
      float2 acc = make_float2(0.f, 0.f);
      const uint64_t K = 1ull << nk;
      for (uint64_t k = 0; k < K; ++k)
        cfma(acc, S.A[oa + scat_small(k, S.sA_k, nk)], S.B[ob + scat_small(k, S.sB_k, nk)]);
      S.C[scat_small(n, S.sC_n, nn) + scat_small(m, S.sC_m, nm) + scat_small(b, S.sC_b, nb)] = acc;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this wave's stores visible to the agent
    __syncthreads();   // ... for every wave, before the item is published
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(&ctr[kCtrStride * (1 + s)], 1, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t* p, int32_t n) {
  for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

}  // namespace tnk
