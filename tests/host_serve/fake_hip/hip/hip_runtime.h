// CPU stand-in for the part of the HIP runtime that the served path uses, so
// that its host logic and its gather/scatter kernels can run under the host
// sanitizers without a GPU.  TEST INFRASTRUCTURE ONLY.
//
// The stand-in keeps the runtime's asynchrony, so that lifetime races between
// the host threads and queued device work show up:
// * every stream has a worker thread that runs its queued operations (kernel
//   grids, copies, event markers) in order, later than they were issued, with
//   random delays, so the host runs ahead of the "device" as it does on a GPU;
// * an event completes when its stream's worker reaches it (an event never
//   recorded counts as complete, as in HIP);
// * hipMemcpyAsync reads its source when the worker runs it, and aborts if the
//   host has changed the source bytes since the call (a host buffer rewritten
//   while a copy from it is still queued);
// * hipFree does not wait for queued work, so freeing a buffer that queued work
//   still uses is a use-after-free for the address sanitizer;
// * device and mapped host addresses are the same pointer; a launch runs every
//   (block, thread) of its grid in order on the stream's worker.  Only kernels
//   without shared memory or barriers can run.
#pragma once

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <deque>
#include <functional>
#include <mutex>
#include <set>
#include <thread>

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

inline void die(const char *what) {
  fprintf(stderr, "fake HIP runtime: %s\n", what);
  fflush(stderr);
  abort();
}

// Operations of one stream, run in order by its worker thread.
struct Stream {
  std::mutex mu;
  std::condition_variable cv, cv_idle;
  std::deque<std::function<void()>> q;
  uint64_t issued = 0, done = 0;  // operations queued / completed
  bool busy = false, stop = false;
  std::thread worker;
  uint64_t rng;

  explicit Stream(uint64_t seed) : rng(seed * 0x9E3779B97F4A7C15ull + 1) {
    worker = std::thread([this] { run(); });
  }
  uint64_t next_rand() {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
  }
  void run() {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      cv.wait(lk, [&] { return stop || !q.empty(); });
      if (q.empty()) break;
      auto op = std::move(q.front());
      q.pop_front();
      busy = true;
      const uint64_t r = next_rand();
      lk.unlock();
      // the device lags behind the host by a random amount
      if (r % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(r % 300));
      op();
      lk.lock();
      busy = false;
      ++done;
      cv_idle.notify_all();
    }
  }
  uint64_t push(std::function<void()> op) {
    std::lock_guard<std::mutex> lk(mu);
    q.push_back(std::move(op));
    cv.notify_one();
    return ++issued;
  }
  bool reached(uint64_t seq) {
    std::lock_guard<std::mutex> lk(mu);
    return done >= seq;
  }
  void sync() {
    std::unique_lock<std::mutex> lk(mu);
    cv_idle.wait(lk, [&] { return q.empty() && !busy; });
  }
  ~Stream() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
      cv.notify_one();
    }
    worker.join();
  }
};

struct Registry {
  std::mutex mu;
  std::set<Stream *> streams;
  uint64_t seed = 1;
  Stream *null_stream = nullptr;
};
inline Registry &reg() {
  static Registry r;
  return r;
}

inline Stream *null_stream() {
  auto &R = reg();
  std::lock_guard<std::mutex> lk(R.mu);
  if (!R.null_stream) {
    R.null_stream = new Stream(R.seed++);
    R.streams.insert(R.null_stream);
  }
  return R.null_stream;
}

inline Stream *as_stream(void *s) { return s ? static_cast<Stream *>(s) : null_stream(); }

inline void sync_all() {
  std::set<Stream *> all;
  {
    auto &R = reg();
    std::lock_guard<std::mutex> lk(R.mu);
    all = R.streams;
  }
  for (Stream *s : all) s->sync();
}

struct Event {
  Stream *stream = nullptr;  // stream of the last record (null: never recorded)
  uint64_t seq = 0;
};

template <class F, class... A>
void run_grid(F kernel, dim3 grid, dim3 block, A... args) {
  gridDim = grid;
  blockDim = block;
  for (unsigned b = 0; b < grid.x; ++b)
    for (unsigned t = 0; t < block.x; ++t) {
      blockIdx = dim3(b);
      threadIdx = dim3(t);
      kernel(args...);
    }
}

template <class F, class... A>
void launch(void *stream, F kernel, dim3 grid, dim3 block, A... args) {
  as_stream(stream)->push([=] { run_grid(kernel, grid, block, args...); });
}

inline uint64_t checksum(const void *p, size_t n) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

inline void *alloc(size_t n) { return aligned_alloc(256, (n + 255) / 256 * 256 + 256); }

}  // namespace fakehip

typedef struct fakehip_stream_tag *hipStream_t;
typedef struct fakehip_event_tag *hipEvent_t;

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  fakehip::launch((void *)(stream), kernel, dim3(grid), dim3(block), __VA_ARGS__)

inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() {
  fakehip::sync_all();
  return hipSuccess;
}
inline hipError_t hipMalloc(void **p, size_t n) {
  *p = fakehip::alloc(n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
// No implicit wait: queued work that still uses the buffer turns into a
// use-after-free for the address sanitizer.
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
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t st) {
  const uint64_t h = fakehip::checksum(s, n);
  fakehip::as_stream(st)->push([=] {
    if (fakehip::checksum(s, n) != h) fakehip::die("the source of a queued copy changed before the copy ran");
    memcpy(d, s, n);
  });
  return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  auto &R = fakehip::reg();
  std::lock_guard<std::mutex> lk(R.mu);
  auto *st = new fakehip::Stream(R.seed++);
  R.streams.insert(st);
  *s = reinterpret_cast<hipStream_t>(st);
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
  auto *st = reinterpret_cast<fakehip::Stream *>(s);
  st->sync();
  {
    auto &R = fakehip::reg();
    std::lock_guard<std::mutex> lk(R.mu);
    R.streams.erase(st);
  }
  delete st;
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t s) {
  fakehip::as_stream(s)->sync();
  return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
  *e = reinterpret_cast<hipEvent_t>(new fakehip::Event());
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete reinterpret_cast<fakehip::Event *>(e);
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  auto *ev = reinterpret_cast<fakehip::Event *>(e);
  fakehip::Stream *st = fakehip::as_stream(s);
  ev->stream = st;
  ev->seq = st->push([] {});
  return hipSuccess;
}
inline hipError_t hipEventQuery(hipEvent_t e) {
  auto *ev = reinterpret_cast<fakehip::Event *>(e);
  if (!ev->stream || ev->stream->reached(ev->seq)) return hipSuccess;
  return hipErrorNotReady;
}
