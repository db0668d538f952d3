// Calibration kernels: the sustained integer VALU rate of the device, from
// every compute unit running independent chains of packed 16-bit (or 32-bit)
// add + max, the two operations the dynamic program is made of.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

}  // namespace

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
