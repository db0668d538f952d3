// Seed index (pointer table + CAL table) and CAL finder launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sw_align.h"

namespace swk {

// Reference layout the index kernels need (device words, per-reference data).
struct SeedRefs {
  const uint32_t *words;
  int64_t word_off[SW_MAX_REFS];
  int64_t len[SW_MAX_REFS];
  int64_t occ_off[SW_MAX_REFS + 1];  // first occurrence index of each reference
  int32_t n_refs;
};

struct SeedParams {
  int32_t seed_len;   // S, 1..32
  int32_t addr_bits;  // A <= 2S
};

// Sorted CAL table: key = invertible hash of the canonical seed (2S bits);
// value = (reference << 41) | (position << 1) | strand bit of the reference seed.
struct IndexView {
  const uint64_t *key;
  const uint64_t *val;
  const int64_t *ptr;  // [2^A + 1] first entry of each address
  int64_t n;
  SeedParams p;
};

// Temporary bytes of the build's radix sort for n entries.
size_t index_sort_temp_bytes(int64_t n, int seed_len);
// Fills key/val (unsorted) for every reference seed, sorts them into key/val
// (using the alternate buffers), then builds the pointer table.
hipError_t launch_index_build(const SeedRefs &R, const SeedParams &P, int64_t n, uint64_t *key, uint64_t *val,
                              uint64_t *key_alt, uint64_t *val_alt, void *temp, size_t temp_bytes, int64_t *ptr,
                              hipStream_t st);

struct FindArgs {
  IndexView ix;
  const uint32_t *reads;
  const int64_t *read_word_off;
  const int32_t *read_len;
  int32_t n_reads;
  int32_t stride;
  int32_t max_cals_per_seed;
  int32_t max_read_len;
  int32_t max_seeds;           // seeds per read slot: (max_read_len - S) / stride + 1
  const int64_t *ref_len;      // device [n_refs]
  int64_t *cal_ptr;
  int64_t *cal_pos;
  int16_t *cal_ref;
  uint8_t *strand;
  unsigned long long *err;
};

size_t find_temp_bytes(int64_t n_slots);
// Pass 1: per (read, seed) CAL counts and their exclusive scan (cnt, offs hold
// n_slots + 1 entries); cal_ptr is filled.  The total is offs[n_slots].
// run_lo (n_slots entries) keeps each seed's first CAL-table entry for pass 2.
hipError_t launch_find_count(const FindArgs &A, int64_t *cnt, int64_t *offs, int64_t *run_lo, void *temp,
                             size_t temp_bytes, hipStream_t st);
// Pass 2: writes every CAL (needs offs[n_slots] <= the output capacity).
hipError_t launch_find_write(const FindArgs &A, const int64_t *offs, const int64_t *run_lo, hipStream_t st);

}  // namespace swk
