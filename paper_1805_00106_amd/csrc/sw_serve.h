// Served path: chunk descriptors and the gather/scatter launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace swk {

// One chunk of one admitted request inside a step: request reads [r0, r1)
// (and their CALs) placed at step read r0 -> step_r0, CAL -> step_c0, word -> step_w0.
struct ServeChunk {
  // request inputs (device)
  const uint32_t *words;
  const int64_t *word_off;
  const int32_t *len;
  const int64_t *cal_ptr;
  const int64_t *cal_pos;
  const int16_t *cal_ref;
  const uint8_t *strand;
  // request outputs (device)
  int32_t *score;
  int64_t *ref_end;
  int16_t *read_end;
  int32_t *best_score;
  int64_t *best_slot;
  int32_t *n_tied;
  int64_t r0, r1;
  int64_t step_r0, step_c0, step_w0;
};

hipError_t launch_serve_gather(const ServeChunk *ch, int n_chunks, int64_t n_reads, int64_t n_cals, uint32_t *words,
                               int64_t *word_off, int32_t *read_len, int64_t *cal_ptr, int64_t *cal_pos,
                               int16_t *cal_ref, uint8_t *strand, hipStream_t st);
hipError_t launch_serve_scatter(const ServeChunk *ch, int n_chunks, int64_t n_reads, int64_t n_cals, int32_t n_refs,
                                const int32_t *score, const int64_t *ref_end, const int16_t *read_end,
                                const int32_t *best_score, const int64_t *best_slot, const int32_t *n_tied,
                                hipStream_t st);

}  // namespace swk
