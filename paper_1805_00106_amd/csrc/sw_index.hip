// Seed index and CAL finder for gfx950 (sections 3.1 and 3.2 of the paper).
//
// Index: every overlapping reference seed of S bases is reduced to its
// canonical form (the smaller of the seed and its reverse complement, with a
// strand bit saying which one the reference holds), hashed by an invertible
// mix of its 2S bits so that buckets fill evenly, and sorted by hash with a
// device radix sort (stable: equal seeds stay in reference order).  The sorted
// array is the CAL table; the top A hash bits address the pointer table, whose
// entry a is the first CAL-table index of address a.  Since the hash is a
// bijection, a full-hash comparison inside the bucket is an exact seed match.
//
// Seed values put the first base in the most significant bit pair.  The
// packed words hold base i at bits 2(i mod 16) (first base least significant),
// so the raw bit string of S bases read from the words is the seed reversed:
// complementing it gives the reverse complement directly, and reversing its
// bit pairs gives the seed.
//
// CAL finder: one thread per (read, seed slot); a first pass counts each
// seed's CALs, a device scan places them, and a second pass writes them in
// (seed, reference, position) order.
#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>
#include <hipcub/device/device_scan.hpp>
#include <stdint.h>

#include "sw_index.h"

namespace swk {

namespace {

__device__ __forceinline__ uint64_t mask_bits(int nbits) { return nbits >= 64 ? ~0ull : ((1ull << nbits) - 1ull); }

// Reverse the order of the 32 bit pairs of x.
__device__ __forceinline__ uint64_t rev_pairs(uint64_t x) {
  x = __builtin_bitreverse64(x);
  return ((x >> 1) & 0x5555555555555555ull) | ((x & 0x5555555555555555ull) << 1);
}

// Invertible mix of an nbits-wide value (odd multiplications and xor-shifts
// modulo 2^nbits are bijections).
__device__ __forceinline__ uint64_t mix(uint64_t v, int nbits) {
  const uint64_t m = mask_bits(nbits);
  const int sh = nbits / 2 > 0 ? nbits / 2 : 1;
  v = (v * 0x9E3779B97F4A7C15ull) & m;
  v ^= v >> sh;
  v = (v * 0xC2B2AE3D27D4EB4Full) & m;
  v ^= v >> sh;
  return v;
}

// S bases starting at base g of a packed sequence whose last word is `last`, as
// the raw LSB-first string.  Words past `last` are not read (the bases needed
// never reach them).
__device__ __forceinline__ uint64_t raw_bases(const uint32_t *words, int64_t g, int S, int64_t last) {
  const int64_t w = g >> 4;
  const uint32_t sh = 2u * (uint32_t)(g & 15);
  const uint64_t w0 = words[w];
  const uint64_t w1 = w + 1 <= last ? words[w + 1] : 0u;
  uint64_t raw = (w0 | (w1 << 32)) >> sh;
  if (sh && w + 2 <= last) raw |= (uint64_t)words[w + 2] << (64 - sh);
  return raw & mask_bits(2 * S);
}

struct Canon {
  uint64_t hash;
  int strand;      // 1: the sequence holds the reverse complement of the canonical seed
  bool palindrome;
};

__device__ __forceinline__ Canon canon_of_raw(uint64_t raw, int S) {
  const uint64_t m = mask_bits(2 * S);
  const uint64_t v = rev_pairs(raw) >> (64 - 2 * S);  // seed value, first base most significant
  const uint64_t rc = raw ^ m;                       // reverse complement value
  Canon c;
  c.strand = rc < v ? 1 : 0;
  c.palindrome = rc == v;
  c.hash = mix(c.strand ? rc : v, 2 * S);
  return c;
}

__global__ void k_index_seeds(const SeedRefs R, const SeedParams P, int64_t n, uint64_t *__restrict__ key,
                              uint64_t *__restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int k = 0;
  while (k + 1 < R.n_refs && R.occ_off[k + 1] <= i) ++k;
  const int64_t x = i - R.occ_off[k];
  const uint64_t raw = raw_bases(R.words + R.word_off[k], x, P.seed_len, (R.len[k] - 1) >> 4);
  const Canon c = canon_of_raw(raw, P.seed_len);
  key[i] = c.hash;
  val[i] = ((uint64_t)k << 41) | ((uint64_t)x << 1) | (uint64_t)c.strand;
}

__global__ void k_index_ptr(const uint64_t *__restrict__ key, int64_t n, int shift, int64_t n_addr,
                            int64_t *__restrict__ ptr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  const int64_t a_prev = i == 0 ? -1 : (int64_t)(key[i - 1] >> shift);
  const int64_t a_here = i == n ? n_addr : (int64_t)(key[i] >> shift);
  for (int64_t a = a_prev + 1; a <= a_here; ++a) ptr[a] = i;
}

// Run [lo, hi) of entries whose key equals h (keys ascending inside the bucket).
__device__ __forceinline__ void find_run(const IndexView &I, uint64_t h, int64_t &lo, int64_t &hi) {
  const int64_t a = (int64_t)(h >> (2 * I.p.seed_len - I.p.addr_bits));
  int64_t b0 = I.ptr[a], b1 = I.ptr[a + 1];
  int64_t l = b0, r = b1;
  while (l < r) {
    const int64_t m = l + (r - l) / 2;
    if (I.key[m] < h) l = m + 1; else r = m;
  }
  lo = l;
  r = b1;
  while (l < r) {
    const int64_t m = l + (r - l) / 2;
    if (I.key[m] <= h) l = m + 1; else r = m;
  }
  hi = l;
}

struct SeedSlot {
  bool live;
  int32_t L;
  int32_t o;
  Canon c;
};

__device__ __forceinline__ SeedSlot seed_slot(const FindArgs &A, int64_t t) {
  SeedSlot s{};
  const int64_t r = t / A.max_seeds;
  const int j = (int)(t - r * A.max_seeds);
  const int S = A.ix.p.seed_len;
  s.L = A.read_len[r];
  s.o = j * A.stride;
  s.live = s.L >= 1 && s.L <= A.max_read_len && s.o + S <= s.L;
  if (s.live) {
    const uint64_t raw = raw_bases(A.reads + A.read_word_off[r], s.o, S, (s.L - 1) >> 4);
    s.c = canon_of_raw(raw, S);
  }
  return s;
}

__global__ void k_find_count(const FindArgs A, int64_t n_slots, int64_t *__restrict__ cnt,
                             int64_t *__restrict__ run_lo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_slots) return;
  if (t == n_slots) {
    cnt[t] = 0;
    return;
  }
  const SeedSlot s = seed_slot(A, t);
  int64_t n = 0, lo = 0, hi = 0;
  if (s.live) {
    find_run(A.ix, s.c.hash, lo, hi);
    n = (hi - lo) * (s.c.palindrome ? 2 : 1);
    if (A.max_cals_per_seed > 0 && n > A.max_cals_per_seed) n = 0;
  }
  cnt[t] = n;
  run_lo[t] = lo;  // the write pass starts here without searching again
}

__global__ void k_find_ptr(const FindArgs A, const int64_t *__restrict__ offs) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > A.n_reads) return;
  A.cal_ptr[r] = offs[r * A.max_seeds];
}

// Reads outside [1, max_read_len] got no CALs: count them once, with the write
// pass (a caller may run the count pass again after growing its buffers).
__global__ void k_find_errors(const FindArgs A) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.n_reads) return;
  const int32_t L = A.read_len[r];
  if (L < 1 || L > A.max_read_len) atomicAdd(A.err, 1ull);
}

__global__ void k_find_write(const FindArgs A, int64_t n_slots, const int64_t *__restrict__ offs,
                             const int64_t *__restrict__ run_lo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_slots) return;
  int64_t out = offs[t];
  const int64_t end = offs[t + 1];
  if (out == end) return;
  const SeedSlot s = seed_slot(A, t);
  // the run has (end - out) / (2 if palindrome) entries starting at run_lo[t]
  const int64_t lo = run_lo[t], hi = lo + (end - out) / (s.c.palindrome ? 2 : 1);
  const int S = A.ix.p.seed_len;
  for (int64_t e = lo; e < hi && out < end; ++e) {
    const uint64_t v = A.ix.val[e];
    const int k = (int)(v >> 41);
    const int64_t x = (int64_t)((v >> 1) & ((1ull << 40) - 1));
    const int ref_strand = (int)(v & 1);
    const int64_t len = A.ref_len[k];
    for (int pass = 0; pass < (s.c.palindrome ? 2 : 1); ++pass) {
      const bool fwd = s.c.palindrome ? pass == 0 : ref_strand == s.c.strand;
      int64_t p = fwd ? x - s.o : x - (s.L - s.o - S);
      p = p < 0 ? 0 : (p >= len ? len - 1 : p);
      A.cal_pos[out] = p;
      A.cal_ref[out] = (int16_t)k;
      A.strand[out] = fwd ? 1 : 2;
      ++out;
    }
  }
}

inline unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

size_t index_sort_temp_bytes(int64_t n, int seed_len) {
  size_t t = 0;
  hipcub::DoubleBuffer<uint64_t> k(nullptr, nullptr), v(nullptr, nullptr);
  hipcub::DeviceRadixSort::SortPairs(nullptr, t, k, v, (int)n, 0, 2 * seed_len);
  return t;
}

hipError_t launch_index_build(const SeedRefs &R, const SeedParams &P, int64_t n, uint64_t *key, uint64_t *val,
                              uint64_t *key_alt, uint64_t *val_alt, void *temp, size_t temp_bytes, int64_t *ptr,
                              hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_index_seeds, dim3(blocks(n, 256)), dim3(256), 0, st, R, P, n, key_alt, val_alt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipcub::DoubleBuffer<uint64_t> kb(key_alt, key), vb(val_alt, val);
  if (n > 0) {
    e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, kb, vb, (int)n, 0, 2 * P.seed_len, st);
    if (e != hipSuccess) return e;
    // the sorted result must end in key/val
    if (kb.Current() != key) {
      e = hipMemcpyAsync(key, kb.Current(), (size_t)n * 8, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
      e = hipMemcpyAsync(val, vb.Current(), (size_t)n * 8, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
    }
  }
  const int64_t n_addr = 1ll << P.addr_bits;
  hipLaunchKernelGGL(k_index_ptr, dim3(blocks(n + 1, 256)), dim3(256), 0, st, key, n, 2 * P.seed_len - P.addr_bits,
                     n_addr, ptr);
  return hipGetLastError();
}

size_t find_temp_bytes(int64_t n_slots) {
  size_t t = 0;
  hipcub::DeviceScan::ExclusiveSum(nullptr, t, (const int64_t *)nullptr, (int64_t *)nullptr, (int)(n_slots + 1));
  return t;
}

hipError_t launch_find_count(const FindArgs &A, int64_t *cnt, int64_t *offs, int64_t *run_lo, void *temp,
                             size_t temp_bytes, hipStream_t st) {
  const int64_t n_slots = (int64_t)A.n_reads * A.max_seeds;
  hipLaunchKernelGGL(k_find_count, dim3(blocks(n_slots + 1, 256)), dim3(256), 0, st, A, n_slots, cnt, run_lo);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::ExclusiveSum(temp, temp_bytes, cnt, offs, (int)(n_slots + 1), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_find_ptr, dim3(blocks((int64_t)A.n_reads + 1, 256)), dim3(256), 0, st, A, offs);
  return hipGetLastError();
}

hipError_t launch_find_write(const FindArgs &A, const int64_t *offs, const int64_t *run_lo, hipStream_t st) {
  const int64_t n_slots = (int64_t)A.n_reads * A.max_seeds;
  if (n_slots > 0)
    hipLaunchKernelGGL(k_find_write, dim3(blocks(n_slots, 256)), dim3(256), 0, st, A, n_slots, offs, run_lo);
  if (A.n_reads > 0) hipLaunchKernelGGL(k_find_errors, dim3(blocks(A.n_reads, 256)), dim3(256), 0, st, A);
  return hipGetLastError();
}

}  // namespace swk
