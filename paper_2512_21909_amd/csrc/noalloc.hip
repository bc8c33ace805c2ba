// Allocation-free variant of the T2 ladder entry point, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// The plan tables and the workspace of a call live in one file-scope static
// device array of kScratchBytes.  Every GPU the library runs on holds its own
// copy of the array (at its own address) until the process ends.  Its device
// address is looked up once per device, on the entry point's first call
// there, and only that address is used afterwards: the array's name in host
// code is a host-side stand-in, not a device pointer.  Calls on one GPU share
// the array, so calls that overlap in time on that GPU (different streams, or
// different host threads without ordering) race; consecutive calls on one
// stream are ordered.  The array keeps the last call's contents; every byte a
// call's kernels read is written by that call first (the queue counters are
// cleared by a fill kernel at its start).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "../../include/cdcc.h"

int run_ladder_in_region(int32_t nsys, const cdcc_problem_t *probs, const cdcc_opts_t *opts, void *stream,
                         void *region, int64_t region_bytes);

namespace {

constexpr int64_t kScratchBytes = CDCC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> device address of that device's copy of `scratch`

}  // namespace

extern "C" int cdcc_ladder_t2_noalloc(int32_t nsys, const cdcc_problem_t *probs, const cdcc_opts_t *opts,
                                      void *stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CDCC_EDEVICE;
  void *ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
        (void)hipGetLastError();
        return CDCC_EDEVICE;
      }
      g_scratch_ptr[dev] = ptr;
    } else {
      ptr = it->second;
    }
  }
  return run_ladder_in_region(nsys, probs, opts, stream, ptr, kScratchBytes);
}
