// Stand-in "scoring" for the host test of the served path: a deterministic
// function of a read's bases and one CAL, so that a result routed to the wrong
// request, read, CAL or strand slot is caught.  TEST INFRASTRUCTURE ONLY (it
// replaces the device scoring calls, whose parity the GPU tests check).
#pragma once

#include <stdint.h>

inline uint64_t stub_read_hash(const uint8_t *codes, int L) {
  uint64_t h = 1469598103934665603ull ^ (uint64_t)L;
  for (int i = 0; i < L; ++i) h = (h ^ (codes[i] & 3u)) * 1099511628211ull;
  return h;
}

// One slot (CAL, strand h): -1 everywhere when the strand is not requested.
inline void stub_slot(uint64_t rh, int L, int64_t pos, int ref, int mask, int h, int32_t *score, int64_t *ref_end,
                      int16_t *read_end) {
  if (!((mask >> h) & 1)) {
    *score = -1;
    *ref_end = -1;
    *read_end = -1;
    return;
  }
  uint64_t x = rh ^ ((uint64_t)pos * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)(ref + 1) << 40) ^ (h ? 0xABCDEFull : 0);
  x ^= x >> 29;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 32;
  *score = (int32_t)(x % 41);  // a small range: many ties per read
  *ref_end = pos + (int64_t)(x % 5);
  *read_end = (int16_t)(L > 0 ? (int)((x >> 8) % (uint64_t)L) : -1);
}
