// Bounds checks of the debug kernel build (compiled with -DMFPFF_BOUNDS).
//
// MFPFF_IN(i, n) is i where 0 <= i < n; outside that range it counts the access in a device
// counter of its translation unit and yields 0, so that a wrong index is reported, never turned
// into a memory fault.  Every source file that uses it defines MFPFF_BOUNDS_READER(name), a host
// function returning its counter; mfpff_debug_bounds_hits() sums them.  In the regular build the
// macro is the index itself and nothing else is compiled.
#pragma once

#ifdef MFPFF_BOUNDS
#include <hip/hip_runtime.h>

namespace mfpff {
namespace {
__device__ unsigned int g_bounds_hits;  // one counter per translation unit
__device__ __forceinline__ long long bounds_in(long long i, long long n) {
  if (i < 0 || i >= n) {
    atomicAdd(&g_bounds_hits, 1u);
    return 0;
  }
  return i;
}
}  // namespace
}  // namespace mfpff

#define MFPFF_IN(i, n) ::mfpff::bounds_in((long long)(i), (long long)(n))
#define MFPFF_BOUNDS_READER(name)                                                         \
  namespace mfpff {                                                                       \
  unsigned int name() {                                                                   \
    unsigned int v = 0;                                                                   \
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_bounds_hits), sizeof(v)) != hipSuccess) return ~0u; \
    return v;                                                                             \
  }                                                                                       \
  }
#else
#define MFPFF_IN(i, n) (i)
#define MFPFF_BOUNDS_READER(name)
#endif
