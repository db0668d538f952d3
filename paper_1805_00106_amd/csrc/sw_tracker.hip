// Score Tracker kernels for gfx950 (sections 3.6 and 4.2 of the paper): per
// read and reference the best slot, the k best slots of a read, the flags of
// the slots tied for a read's best, and the two-reference classification.
//
// Every kernel runs one thread per read over the read's CSR row of CALs.  The
// row is clamped to [0, n_cals] first, as the scoring path does, so a malformed
// row pointer yields fewer slots and never an access outside the arrays.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_launch.h"

namespace swk {

namespace {

__device__ __forceinline__ void row_range(const int64_t *cal_ptr, int64_t r, int64_t n_cals, int64_t &a,
                                          int64_t &b) {
  a = cal_ptr[r];
  b = cal_ptr[r + 1];
  a = a < 0 ? 0 : (a > n_cals ? n_cals : a);
  b = b < a ? a : (b > n_cals ? n_cals : b);
}

// Best slot per reference, lowest slot among ties, tie count.
__global__ void k_reduce_best(const int64_t *__restrict__ cal_ptr, const int16_t *__restrict__ cal_ref,
                              int32_t n_reads, int32_t n_refs, int64_t n_cals, const int32_t *__restrict__ score,
                              int32_t *__restrict__ best_score, int64_t *__restrict__ best_slot,
                              int32_t *__restrict__ n_tied) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  const int64_t o = r * n_refs;
  int64_t ca, cb;
  row_range(cal_ptr, r, n_cals, ca, cb);
  if (n_refs <= 8) {
    // per-reference state in registers (the unrolled compare keeps the index static)
    int32_t bs[8];
    int64_t bl[8];
    int32_t nt[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      bs[k] = -1;
      bl[k] = -1;
      nt[k] = 0;
    }
    for (int64_t c = ca; c < cb; ++c) {
      const int k = cal_ref[c];
      if (k < 0 || k >= n_refs) continue;
      const int2 s2 = *reinterpret_cast<const int2 *>(score + 2 * c);
      const int32_t sv[2] = {s2.x, s2.y};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int32_t s = sv[h];
        if (s < 0) continue;
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          if (kk == k) {
            if (s > bs[kk]) {
              bs[kk] = s;
              bl[kk] = 2 * c + h;
              nt[kk] = 1;
            } else if (s == bs[kk]) {
              nt[kk] += 1;
            }
          }
        }
      }
    }
    for (int k = 0; k < n_refs; ++k) {
      best_score[o + k] = bs[k];
      best_slot[o + k] = bl[k];
      n_tied[o + k] = nt[k];
    }
  } else {
    for (int k = 0; k < n_refs; ++k) {
      best_score[o + k] = -1;
      best_slot[o + k] = -1;
      n_tied[o + k] = 0;
    }
    for (int64_t c = ca; c < cb; ++c) {
      const int k = cal_ref[c];
      if (k < 0 || k >= n_refs) continue;
      for (int h = 0; h < 2; ++h) {
        const int32_t s = score[2 * c + h];
        if (s < 0) continue;
        if (s > best_score[o + k]) {
          best_score[o + k] = s;
          best_slot[o + k] = 2 * c + h;
          n_tied[o + k] = 1;
        } else if (s == best_score[o + k]) {
          n_tied[o + k] += 1;
        }
      }
    }
  }
}

// The k best slots over all CALs and strands (highest score, then lowest slot),
// kept sorted in the output row by insertion.
__global__ void k_topk(const int64_t *__restrict__ cal_ptr, int32_t n_reads, int64_t n_cals,
                       const int32_t *__restrict__ score, int32_t k, int32_t *__restrict__ top_score,
                       int64_t *__restrict__ top_slot) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  int32_t *ts = top_score + r * k;
  int64_t *tl = top_slot + r * k;
  int64_t ca, cb;
  row_range(cal_ptr, r, n_cals, ca, cb);
  int n = 0;                 // entries filled
  int32_t last = INT32_MAX;  // score of entry k-1 once the list is full
  for (int64_t slot = 2 * ca; slot < 2 * cb; ++slot) {
    const int32_t s = score[slot];
    if (s < 0) continue;
    // slots arrive in increasing order, so an equal score never displaces an entry
    if (n == k && s <= last) continue;
    int pos = n < k ? n : k - 1;
    while (pos > 0 && ts[pos - 1] < s) {
      ts[pos] = ts[pos - 1];
      tl[pos] = tl[pos - 1];
      --pos;
    }
    ts[pos] = s;
    tl[pos] = slot;
    if (n < k) ++n;
    if (n == k) last = ts[k - 1];
  }
  for (int i = n; i < k; ++i) {
    ts[i] = -1;
    tl[i] = -1;
  }
}

// Flag every slot whose score equals the read's best.
__global__ void k_tied(const int64_t *__restrict__ cal_ptr, int32_t n_reads, int64_t n_cals,
                       const int32_t *__restrict__ score, uint8_t *__restrict__ flags) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  int64_t ca, cb;
  row_range(cal_ptr, r, n_cals, ca, cb);
  int32_t best = -1;
  for (int64_t slot = 2 * ca; slot < 2 * cb; ++slot) best = max(best, score[slot]);
  for (int64_t slot = 2 * ca; slot < 2 * cb; ++slot) flags[slot] = (best >= 0 && score[slot] == best) ? 1 : 0;
}

// Two-reference (or more) classification from the per-reference bests:
// unaligned (-1) below the threshold, tie (-2), else the winning reference.
__global__ void k_classify(const int32_t *__restrict__ best_score, int32_t n_reads, int32_t n_refs,
                           int32_t threshold, int32_t *__restrict__ cls) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  int32_t top = -1, arg = -1, cnt = 0;
  for (int k = 0; k < n_refs; ++k) {
    const int32_t v = best_score[r * n_refs + k];
    if (v > top) {
      top = v;
      arg = k;
      cnt = 1;
    } else if (v == top) {
      cnt++;
    }
  }
  cls[r] = top < threshold ? -1 : (cnt > 1 ? -2 : arg);
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_reduce(const int64_t *cal_ptr, const int16_t *cal_ref, int32_t n_reads, int32_t n_refs,
                         int64_t n_cals, const int32_t *score, int32_t *bs, int64_t *bl, int32_t *nt,
                         hipStream_t st) {
  if (n_reads == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_best, dim3(blocks_for(n_reads, 256)), dim3(256), 0, st, cal_ptr, cal_ref, n_reads,
                     n_refs, n_cals, score, bs, bl, nt);
  return hipGetLastError();
}

hipError_t launch_topk(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, const int32_t *score, int32_t k,
                       int32_t *ts, int64_t *tl, hipStream_t st) {
  if (n_reads == 0) return hipSuccess;
  hipLaunchKernelGGL(k_topk, dim3(blocks_for(n_reads, 256)), dim3(256), 0, st, cal_ptr, n_reads, n_cals, score, k,
                     ts, tl);
  return hipGetLastError();
}

hipError_t launch_tied(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, const int32_t *score,
                       uint8_t *flags, hipStream_t st) {
  if (n_reads == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tied, dim3(blocks_for(n_reads, 256)), dim3(256), 0, st, cal_ptr, n_reads, n_cals, score,
                     flags);
  return hipGetLastError();
}

hipError_t launch_classify(const int32_t *bs, int32_t n_reads, int32_t n_refs, int32_t thr, int32_t *cls,
                           hipStream_t st) {
  if (n_reads == 0) return hipSuccess;
  hipLaunchKernelGGL(k_classify, dim3(blocks_for(n_reads, 256)), dim3(256), 0, st, bs, n_reads, n_refs, thr, cls);
  return hipGetLastError();
}

}  // namespace swk
