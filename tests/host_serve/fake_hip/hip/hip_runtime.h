// CPU stand-in for the part of the HIP runtime that the served path uses, so
// that its host logic and its gather/scatter kernels can run under the host
// sanitizers without a GPU.  TEST INFRASTRUCTURE ONLY.
//
// Memory calls are malloc/free (device and mapped host addresses are the same
// pointer), copies are synchronous memcpy, streams and events complete at once,
// and a kernel launch runs every (block, thread) of its grid on the calling
// thread, in order.  Only kernels without shared memory or barriers can run.
#pragma once

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cstddef>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define HIP_KERNEL_NAME(...) __VA_ARGS__

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidDevice = 101,
  hipErrorNotReady = 600,
} hipError_t;

typedef struct fake_stream *hipStream_t;
typedef struct fake_event *hipEvent_t;

enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };

#define hipHostMallocDefault 0x0
#define hipHostMallocMapped 0x2
#define hipHostMallocCoherent 0x40000000
#define hipStreamNonBlocking 0x1
#define hipEventDisableTiming 0x2

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint2 {
  unsigned x, y;
};
inline uint2 make_uint2(unsigned a, unsigned b) { return uint2{a, b}; }

inline thread_local dim3 blockIdx, threadIdx, blockDim, gridDim;

namespace fakehip {
template <class F, class... A>
void launch(F kernel, dim3 grid, dim3 block, A... args) {
  gridDim = grid;
  blockDim = block;
  for (unsigned b = 0; b < grid.x; ++b)
    for (unsigned t = 0; t < block.x; ++t) {
      blockIdx = dim3(b);
      threadIdx = dim3(t);
      kernel(args...);
    }
}
inline void *alloc(size_t n) { return aligned_alloc(256, (n + 255) / 256 * 256 + 256); }
}  // namespace fakehip

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  fakehip::launch(kernel, dim3(grid), dim3(block), __VA_ARGS__)

inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipMalloc(void **p, size_t n) {
  *p = fakehip::alloc(n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void *p) {
  free(p);
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
inline hipError_t hipHostFree(void *p) { return hipFree(p); }
inline hipError_t hipHostGetDevicePointer(void **d, void *h, unsigned) {
  *d = h;
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
  memcpy(d, s, n);
  return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = reinterpret_cast<hipStream_t>(fakehip::alloc(1));
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) { return hipFree(s); }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
  *e = reinterpret_cast<hipEvent_t>(fakehip::alloc(1));
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) { return hipFree(e); }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
