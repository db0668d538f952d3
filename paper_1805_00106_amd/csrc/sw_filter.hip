// CAL Filter for gfx950 (section 3.3 of the paper): duplicate CALs of a read are
// combined into one reference lookup before scoring.  Two CALs of one read are
// duplicates when they name the same reference and their positions share the
// bucket pos >> bucket_bits; the first CAL of each bucket (input order) is
// kept, with the union of the strand masks of its duplicates.
//
// One wavefront per read.  A read's CALs (tens, rarely hundreds) are staged in
// LDS as 48-bit keys (reference, bucket); each lane tests its CALs against the
// earlier ones, ballots give the kept CALs' ranks, and LDS atomics collect the
// strand unions.  The per-read counts go through a device exclusive scan
// (hipCUB) to place each read's output run.  A read with more CALs than the LDS
// holds is handled by one lane with the same comparisons on device memory.
#include <hip/hip_runtime.h>
#include <hipcub/device/device_scan.hpp>
#include <stdint.h>

#include <algorithm>

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

constexpr int kFilterLds = 512;  // CALs of one read staged in LDS

// (bucket, reference) of a CAL, compared as a pair: any int64 position and any
// int16 reference id (invalid ones included) keep their own identity.
struct CalKey {
  int64_t bucket;
  int32_t ref;
};
__device__ __forceinline__ bool operator==(const CalKey &x, const CalKey &y) {
  return x.bucket == y.bucket && x.ref == y.ref;
}
__device__ __forceinline__ bool operator!=(const CalKey &x, const CalKey &y) { return !(x == y); }
__device__ __forceinline__ CalKey cal_key(const FilterArgs &A, int64_t c) {
  return CalKey{A.cal_pos[c] >> A.bucket_bits, (int32_t)A.cal_ref[c]};
}

// Stage keys and masks, then mark each CAL's first duplicate (its own index if it
// is the first of its bucket).  Returns the read's number of kept CALs.
__device__ int wave_firsts(const FilterArgs &A, int64_t a, int n, CalKey *key, uint32_t *mask, int32_t *first,
                           int lane) {
  for (int x = lane; x < n; x += 64) {
    key[x] = cal_key(A, a + x);
    mask[x] = 0u;
  }
  __syncthreads();
  int kept = 0;
  for (int base = 0; base < n; base += 64) {
    const int x = base + lane;
    int f = x;
    if (x < n) {
      const CalKey kx = key[x];
      for (int d = 0; d < x; ++d)
        if (key[d] == kx) {
          f = d;
          break;
        }
      first[x] = f;
    }
    kept += __popcll(__ballot(x < n && f == x));
  }
  __syncthreads();
  return kept;
}

__global__ __launch_bounds__(64) void k_filter_count_wave(const FilterArgs A, int64_t *__restrict__ cnt) {
  __shared__ CalKey key[kFilterLds];
  __shared__ uint32_t mask[kFilterLds];
  __shared__ int32_t first[kFilterLds];
  const int lane = threadIdx.x;
  for (int64_t r = blockIdx.x; r <= A.n_reads; r += gridDim.x) {
    if (r == A.n_reads) {
      if (lane == 0) cnt[r] = 0;  // the scan's last entry becomes the total
      continue;
    }
    int64_t a, b;
    read_range(A, r, a, b);
    const int64_t n = b - a;
    int64_t kept = 0;
    if (n <= kFilterLds) {
      kept = wave_firsts(A, a, (int)n, key, mask, first, lane);
    } else {
      // too many for LDS: the same test, each lane scanning device memory
      for (int64_t base = 0; base < n; base += 64) {
        const int64_t x = base + lane;
        bool f = x < n;
        if (f) {
          const CalKey kx = cal_key(A, a + x);
          for (int64_t d = 0; d < x && f; ++d) f = cal_key(A, a + d) != kx;
        }
        kept += __popcll(__ballot(f));
      }
    }
    if (lane == 0) cnt[r] = kept;
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void k_filter_write_wave(const FilterArgs A) {
  __shared__ CalKey key[kFilterLds];
  __shared__ uint32_t mask[kFilterLds];
  __shared__ int32_t first[kFilterLds];
  __shared__ int32_t rank[kFilterLds];
  const int lane = threadIdx.x;
  for (int64_t r = blockIdx.x; r < A.n_reads; r += gridDim.x) {
    int64_t a, b;
    read_range(A, r, a, b);
    const int64_t n = b - a;
    const int64_t o = A.out_ptr[r];
    if (n > kFilterLds) {
      // too many for LDS: chunks of 64 CALs, each lane scanning device memory.  A
      // CAL's first duplicate is a kept CAL of this or an earlier chunk, whose
      // map entry is written (and fenced) before the duplicates read it.
      int64_t run = 0;
      for (int64_t base = 0; base < n; base += 64) {
        const int64_t x = base + lane;
        int64_t f = x;
        if (x < n) {
          const CalKey kx = cal_key(A, a + x);
          for (int64_t d = 0; d < x; ++d)
            if (cal_key(A, a + d) == kx) {
              f = d;
              break;
            }
        }
        const bool keep = x < n && f == x;
        const uint64_t bal = __ballot(keep);
        if (keep) {
          const int64_t oo = o + run + __popcll(bal & ((1ull << lane) - 1ull));
          uint8_t m = A.strand[a + x];
          const CalKey kx = cal_key(A, a + x);
          for (int64_t d = x + 1; d < n; ++d)
            if (cal_key(A, a + d) == kx) m |= A.strand[a + d];
          if (oo < A.n_cals) {
            A.out_pos[oo] = A.cal_pos[a + x];
            A.out_ref[oo] = A.cal_ref[a + x];
            A.out_strand[oo] = m;
          }
          A.cal_map[a + x] = oo;
        }
        run += __popcll(bal);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (x < n && !keep) A.cal_map[a + x] = A.cal_map[a + f];
      }
      __syncthreads();
      continue;
    }
    const int nn = (int)n;
    wave_firsts(A, a, nn, key, mask, first, lane);
    // ranks of the kept CALs (ballot prefix counts), and strand unions
    int run = 0;
    for (int base = 0; base < nn; base += 64) {
      const int x = base + lane;
      const bool keep = x < nn && first[x] == x;
      const uint64_t bal = __ballot(keep);
      if (keep) rank[x] = run + __popcll(bal & ((1ull << lane) - 1ull));
      run += __popcll(bal);
      if (x < nn) atomicOr(&mask[first[x]], (uint32_t)A.strand[a + x]);
    }
    __syncthreads();
    for (int x = lane; x < nn; x += 64) {
      const int f = first[x];
      const int64_t oo = o + rank[f];
      if (f == x && oo < A.n_cals) {
        A.out_pos[oo] = A.cal_pos[a + x];
        A.out_ref[oo] = A.cal_ref[a + x];
        A.out_strand[oo] = (uint8_t)mask[x];
      }
      A.cal_map[a + x] = oo;
    }
    __syncthreads();
  }
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
  // one wavefront per read, on a grid that covers the chip several times over
  const unsigned grid = (unsigned)std::min<int64_t>((int64_t)A.n_reads + 1, 65536);
  hipLaunchKernelGGL(k_filter_count_wave, dim3(grid), dim3(64), 0, st, A, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, A.out_ptr, (int)A.n_reads + 1, st);
  if (e != hipSuccess) return e;
  if (A.n_reads > 0) hipLaunchKernelGGL(k_filter_write_wave, dim3(grid), dim3(64), 0, st, A);
  return hipGetLastError();
}

}  // namespace swk
