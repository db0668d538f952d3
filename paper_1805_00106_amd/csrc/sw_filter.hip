// CAL Filter for gfx950 (section 3.3 of the paper): duplicate CALs of a read are
// combined into one reference lookup before scoring.  Two CALs of one read are
// duplicates when they name the same reference and their positions share the
// bucket pos >> bucket_bits; the first CAL of each bucket (input order) is
// kept, with the union of the strand masks of its duplicates.
//
// One thread per read.  A read's CALs are few (tens), so each thread compares
// every CAL with the ones before it; the per-read counts go through a device
// exclusive scan (hipCUB) to place each read's output run.
#include <hip/hip_runtime.h>
#include <hipcub/device/device_scan.hpp>
#include <stdint.h>

#include "sw_filter.h"

namespace swk {

namespace {

__device__ __forceinline__ void read_range(const FilterArgs &A, int64_t r, int64_t &a, int64_t &b) {
  // clamp a malformed row pointer into [0, n_cals] so no access leaves the arrays
  a = A.cal_ptr[r];
  b = A.cal_ptr[r + 1];
  a = a < 0 ? 0 : (a > A.n_cals ? A.n_cals : a);
  b = b < a ? a : (b > A.n_cals ? A.n_cals : b);
}

__device__ __forceinline__ bool dup(const FilterArgs &A, int64_t x, int64_t y) {
  return A.cal_ref[x] == A.cal_ref[y] && (A.cal_pos[x] >> A.bucket_bits) == (A.cal_pos[y] >> A.bucket_bits);
}

__global__ void k_filter_count(const FilterArgs A, int64_t *__restrict__ cnt) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > A.n_reads) return;
  if (r == A.n_reads) {
    cnt[r] = 0;  // the scan's last entry becomes the total
    return;
  }
  int64_t a, b;
  read_range(A, r, a, b);
  int64_t n = 0;
  for (int64_t c = a; c < b; ++c) {
    bool first = true;
    for (int64_t d = a; d < c && first; ++d) first = !dup(A, d, c);
    n += first;
  }
  cnt[r] = n;
}

__global__ void k_filter_write(const FilterArgs A) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.n_reads) return;
  int64_t a, b;
  read_range(A, r, a, b);
  int64_t o = A.out_ptr[r];
  for (int64_t c = a; c < b; ++c) {
    int64_t f = c;
    for (int64_t d = a; d < c; ++d)
      if (dup(A, d, c)) {
        f = d;
        break;
      }
    if (f == c) {
      uint8_t m = A.strand[c];
      for (int64_t d = c + 1; d < b; ++d)
        if (dup(A, c, d)) m |= A.strand[d];
      // a row pointer that is not non-decreasing can overlap reads and overfill the
      // outputs: such entries are dropped rather than written past the arrays
      if (o < A.n_cals) {
        A.out_pos[o] = A.cal_pos[c];
        A.out_ref[o] = A.cal_ref[c];
        A.out_strand[o] = m;
      }
      A.cal_map[c] = o;
      ++o;
    } else {
      A.cal_map[c] = A.cal_map[f];  // written earlier by this thread
    }
  }
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

size_t scan_temp_bytes(int32_t n_reads) {
  size_t t = 0;
  hipcub::DeviceScan::ExclusiveSum(nullptr, t, (const int64_t *)nullptr, (int64_t *)nullptr, (int)n_reads + 1);
  return t;
}

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

size_t filter_workspace_bytes(int32_t n_reads) {
  return align256(sizeof(int64_t) * ((size_t)n_reads + 1)) + align256(scan_temp_bytes(n_reads));
}

hipError_t launch_filter(const FilterArgs &A, void *workspace, size_t workspace_bytes, hipStream_t st) {
  int64_t *cnt = static_cast<int64_t *>(workspace);
  void *tmp = static_cast<char *>(workspace) + align256(sizeof(int64_t) * ((size_t)A.n_reads + 1));
  size_t tmp_bytes = workspace_bytes - align256(sizeof(int64_t) * ((size_t)A.n_reads + 1));
  if (A.n_cals > 0)
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((A.n_cals + 255) / 256)), dim3(256), 0, st, A.cal_map, A.n_cals,
                       (int64_t)-1);
  const unsigned nb = (unsigned)(((int64_t)A.n_reads + 1 + 255) / 256);
  hipLaunchKernelGGL(k_filter_count, dim3(nb), dim3(256), 0, st, A, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, A.out_ptr, (int)A.n_reads + 1, st);
  if (e != hipSuccess) return e;
  if (A.n_reads > 0)
    hipLaunchKernelGGL(k_filter_write, dim3((unsigned)(((int64_t)A.n_reads + 255) / 256)), dim3(256), 0, st, A);
  return hipGetLastError();
}

}  // namespace swk
