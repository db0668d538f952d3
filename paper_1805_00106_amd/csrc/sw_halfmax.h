// The packed half-precision three-way maximum the int16 scoring kernels use on
// int16 bit patterns (device code only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swk {

typedef _Float16 v2h_t __attribute__((ext_vector_type(2)));

// Per 16-bit half, the maximum of three int16 bit patterns taken in [0, 0x7BFF]
// (patterns of [0x8000, 0xFBFF] rank below all of them): one
// v_pk_maximum3_f16, exact on these patterns since they are the finite
// non-negative halves in increasing order (and the others negative halves).
// sw_check_half_max verifies this ordering on the device for every pair.
__device__ __forceinline__ uint32_t half_max3(uint32_t a, uint32_t b, uint32_t c) {
  const v2h_t m = __builtin_elementwise_maximum(
      __builtin_elementwise_maximum(__builtin_bit_cast(v2h_t, a), __builtin_bit_cast(v2h_t, b)),
      __builtin_bit_cast(v2h_t, c));
  return __builtin_bit_cast(uint32_t, m);
}

}  // namespace swk
