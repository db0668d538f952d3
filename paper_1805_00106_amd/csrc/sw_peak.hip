// Calibration kernels: the sustained integer VALU rate of the device, from
// every compute unit running independent chains of packed 16-bit (or 32-bit)
// add + max, the two operations the dynamic program is made of; and the check
// of the ordering the int16 sweep takes from the packed half-precision maximum.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>

#include "sw_halfmax.h"

namespace swk {

namespace {

typedef short v2s __attribute__((ext_vector_type(2)));

constexpr int kChains = 8;  // independent accumulators per lane (no dependency stalls)

__global__ __launch_bounds__(256) void k_alu_peak16(int64_t iters, uint32_t seed, uint32_t *out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  v2s a[kChains], c[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    a[k] = __builtin_bit_cast(v2s, seed ^ (tid * 2654435761u + k));
    c[k] = __builtin_bit_cast(v2s, (seed + k) * 40503u);
  }
  const v2s b = __builtin_bit_cast(v2s, seed | 0x00010001u);
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = __builtin_elementwise_max(a[k] + b, c[k]);
  }
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) x ^= __builtin_bit_cast(uint32_t, a[k]);
  out[tid] = x;
}

__global__ __launch_bounds__(256) void k_alu_peak32(int64_t iters, uint32_t seed, uint32_t *out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t a[kChains], c[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    a[k] = (int32_t)(seed ^ (tid * 2654435761u + k));
    c[k] = (int32_t)((seed + k) * 40503u);
  }
  const int32_t b = (int32_t)(seed | 1u);
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = max(a[k] + b, c[k]);
  }
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) x ^= (uint32_t)a[k];
  out[tid] = x;
}

// Rank of a pattern in the order the int16 sweep needs: [0x8000, 0xFBFF]
// below everything, then [0, 0x7BFF] in integer order.
__device__ __forceinline__ uint32_t sweep_rank(uint32_t v) { return v >= 0x8000u ? 0u : v + 1u; }

// One thread per first operand x (the sweep's range and the wall patterns),
// against every second operand y of the sweep's range, with zero as the third:
// out[t] = number of halves where the packed half maximum is not an operand
// of the highest rank.
__global__ __launch_bounds__(256) void k_half_max_check(const uint32_t *zero, uint32_t nx, uint32_t *out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nx) return;
  const uint32_t x = t < 0x7C00u ? t : 0x8000u + (t - 0x7C00u);
  const uint32_t z = zero[0];
  const uint32_t X = x * 0x00010001u;
  uint32_t bad = 0;
  for (uint32_t y = 0; y < 0x7C00u; y += 2) {
    const uint32_t Y = y | ((y + 1) << 16);
    const uint32_t r = half_max3(X, Y, z);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t yy = y + h, got = (r >> (16 * h)) & 0xFFFFu;
      const uint32_t want = max(max(sweep_rank(x), sweep_rank(yy)), sweep_rank(0u));
      if (sweep_rank(got) != want || (got != x && got != yy && got != 0u)) ++bad;
    }
  }
  out[t] = bad;
}

}  // namespace

// Number of first operands checked by k_half_max_check.
constexpr uint32_t kHalfCheckN = 2u * 0x7C00u;

hipError_t check_half_max(int64_t *n_bad, hipStream_t st) {
  uint32_t *buf = nullptr;
  hipError_t e = hipMalloc(&buf, sizeof(uint32_t) * (kHalfCheckN + 1));
  if (e != hipSuccess) return e;
  uint32_t *zero = buf + kHalfCheckN;
  e = hipMemsetAsync(zero, 0, sizeof(uint32_t), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_half_max_check, dim3((kHalfCheckN + 255) / 256), dim3(256), 0, st, zero, kHalfCheckN, buf);
    e = hipGetLastError();
  }
  uint32_t *host = nullptr;
  if (e == hipSuccess) {
    host = new (std::nothrow) uint32_t[kHalfCheckN];
    if (!host) e = hipErrorOutOfMemory;
  }
  if (e == hipSuccess) e = hipMemcpyAsync(host, buf, sizeof(uint32_t) * kHalfCheckN, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) {
    int64_t n = 0;
    for (uint32_t i = 0; i < kHalfCheckN; ++i) n += host[i];
    *n_bad = n;
  }
  delete[] host;
  hipFree(buf);
  return e;
}

// Runs the chain kernel on `blocks` blocks of 256 threads and returns the rate
// in integer lane-ops per second (a packed 16-bit op counts as two).
hipError_t measure_alu_peak(int bits, int64_t iters, int blocks, uint32_t *out, hipStream_t st, double *ops_per_s) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    hipEventDestroy(e0);
    return e;
  }
  auto launch = [&](int64_t n) {
    if (bits == 16)
      hipLaunchKernelGGL(k_alu_peak16, dim3(blocks), dim3(256), 0, st, n, 0x9E37u, out);
    else
      hipLaunchKernelGGL(k_alu_peak32, dim3(blocks), dim3(256), 0, st, n, 0x9E37u, out);
  };
  launch(iters / 16);  // warm-up (clocks up)
  hipEventRecord(e0, st);
  launch(iters);
  hipEventRecord(e1, st);
  e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) e = hipGetLastError();
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  const double per_lane = 2.0 * kChains * (double)iters * (bits == 16 ? 2.0 : 1.0);  // add + max per chain step
  *ops_per_s = per_lane * (double)blocks * 256.0 / (ms * 1e-3);
  return hipSuccess;
}

}  // namespace swk
