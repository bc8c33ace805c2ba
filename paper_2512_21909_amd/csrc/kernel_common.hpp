// Device helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "ladder_types.hpp"

namespace cdcc {

// Global-address-space view of a device pointer.  Pointers read from the
// descriptor tables are generic; loads through them would be flat loads, whose
// completion is also counted with LDS traffic, so every LDS wait would wait
// for the in-flight global prefetch too.
#define CDCC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const CDCC_GLOBAL T *as_global(const T *p) {
  return (const CDCC_GLOBAL T *)(p);
}

// s_waitcnt immediate (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt in
// 6:4, lgkmcnt in 11:8): wait for vmcnt <= v and lgkmcnt <= l.
constexpr int waitcnt_imm(int v, int l) { return (v & 15) | ((v >> 4) << 14) | (7 << 4) | (l << 8); }

// One 16-byte chunk per lane from global memory straight into LDS: lane l
// writes bytes [16 l, 16 l + 16) after the wave-uniform LDS pointer dst.
// The copies are counted on vmcnt; the caller waits for them with explicit
// s_waitcnt vmcnt and a barrier.
__device__ __forceinline__ void lds_copy16(const CDCC_GLOBAL unsigned char *src, unsigned char *dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(dst), 16, 0, 0);
}

// Claim the next tile; called by every lane of wave 0, the result is valid in
// all of them (-1 when every queue is empty).  `dead` is per-workgroup state
// (bit l: queue (xcd + l) % 8 known to be empty, in the XCD's stealing order).
// A claim is one atomic on the first live queue; a failed claim marks that
// queue dead, so a workgroup issues at most 8 failed atomics.  When its own
// queue runs dry, the other seven counters are read at once and the queues
// already drained are skipped (counters only grow, so a drained reading is
// final; a stale one just costs an atomic).
__device__ __forceinline__ int claim_tile(int *__restrict__ cnt, const Queues &Q, int xcd, unsigned &dead) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    if (dead == 0xffu) return -1;
    const int l = __builtin_ctz(~dead);
    const int q = (xcd + l) & 7;
    int i = 0;
    if (lane == 0) i = atomicAdd(cnt + q * kQueueStride, 1);
    i = __builtin_amdgcn_readfirstlane(i);
    if (i < Q.qb[q + 1] - Q.qb[q]) return Q.qb[q] + i;
    dead |= 1u << l;
    if (l == 0) {
      int e = 1;
      if (lane < 8) {
        const int qq = (xcd + lane) & 7;
        e = __hip_atomic_load(cnt + qq * kQueueStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
            Q.qb[qq + 1] - Q.qb[qq];
      }
      dead |= unsigned(__ballot(e)) & 0xffu;
    }
  }
}

// Claim a tile for the workgroup (wave 0 claims, LDS broadcasts); the result
// is wave-uniform, so the tile's descriptors are read with scalar loads.
__device__ __forceinline__ int next_tile(int *__restrict__ cnt, const Queues &Q, unsigned &dead, int *s_slot) {
  if (threadIdx.x < 64) {
    const int t = claim_tile(cnt, Q, int(blockIdx.x & 7), dead);
    if (threadIdx.x == 0) *s_slot = t;
  }
  __syncthreads();
  const int t = __builtin_amdgcn_readfirstlane(*s_slot);
  __syncthreads();
  return t;
}

}  // namespace cdcc
