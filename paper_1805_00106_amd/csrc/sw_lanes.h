// Moving 64-bit values between the lanes of a wavefront with 32-bit shuffles.
// Kept free of HIP types so that the host tests can compile it with a stand-in
// shuffle.
#pragma once

#include <stdint.h>

#ifndef SW_HD
#if defined(__HIPCC__) || defined(__HIP__)
#define SW_HD __host__ __device__
#else
#define SW_HD
#endif
#endif

namespace swk {

// Lane `src`'s 64-bit value: each half travels through `shfl32(int value, int
// lane)` on its own, and both are put back together as unsigned words.  (Cast
// back through int, the low half would be sign-extended and every value with
// bit 31 set, such as a reference position at or past 2^31, would come out
// negative.)
template <class Shfl32>
SW_HD inline int64_t shfl_i64(Shfl32 shfl32, int64_t v, int src) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)shfl32((int)(uint32_t)u, src);
  const uint32_t hi = (uint32_t)shfl32((int)(uint32_t)(u >> 32), src);
  return (int64_t)(((uint64_t)hi << 32) | (uint64_t)lo);
}

}  // namespace swk
