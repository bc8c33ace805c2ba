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

// Claim the next tile (thread 0 only); returns -1 when every queue is empty.
// `tries` persists across calls and counts the queues found empty.
__device__ __forceinline__ int claim_tile(int *__restrict__ cnt, const Queues &Q, int xcd, int &tries) {
  while (tries < 8) {
    const int q = (xcd + tries) & 7;
    const int i = atomicAdd(cnt + q, 1);
    if (i < Q.qb[q + 1] - Q.qb[q]) return Q.qb[q] + i;
    ++tries;
  }
  return -1;
}

// Broadcast a tile index claimed by thread 0 to the workgroup.
__device__ __forceinline__ int next_tile(int *__restrict__ cnt, const Queues &Q, int &tries, int *s_slot) {
  if (threadIdx.x == 0) *s_slot = claim_tile(cnt, Q, int(blockIdx.x & 7), tries);
  __syncthreads();
  const int t = *s_slot;
  __syncthreads();
  return t;
}

}  // namespace cdcc
