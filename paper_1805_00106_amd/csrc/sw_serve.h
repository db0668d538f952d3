// Served path: chunk descriptors and the gather/scatter launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace swk {

// One chunk of one admitted request inside a step: a run of the request's reads
// with their CALs, placed at step read step_r0, step CAL step_c0 and step word
// step_w0.  Every pointer is a device address already offset to the chunk's
// first read (words, per-read bests) or first CAL (CAL arrays, slots), and every
// count is computed on the host, so the kernels form no address from data they
// read: whatever the staged bytes hold, each access stays inside its chunk.
struct ServeChunk {
  // inputs in the staging arena
  const uint32_t *words;  // n_words packed words of the chunk's reads
  const int64_t *cal_pos;  // n_cals entries each
  const int16_t *cal_ref;
  const uint8_t *strand;
  // outputs in the staging arena
  int32_t *score;  // 2 * n_cals entries each
  int64_t *ref_end;
  int16_t *read_end;
  int32_t *best_score;  // n_reads * n_refs entries each
  int64_t *best_slot;
  int32_t *n_tied;
  int64_t n_reads, n_cals, n_words;
  int64_t step_r0, step_c0, step_w0;
  int64_t slot_shift;  // request slot index minus step slot index, for best_slot
};

// Copies the chunks' words and CAL arrays into the step buffers (the per-read
// arrays of the step come from the host).
hipError_t launch_serve_gather(const ServeChunk *ch, int n_chunks, int64_t n_words, int64_t n_cals, uint32_t *words,
                               int64_t *cal_pos, int16_t *cal_ref, uint8_t *strand, hipStream_t st);
hipError_t launch_serve_scatter(const ServeChunk *ch, int n_chunks, int64_t n_reads, int64_t n_cals, int32_t n_refs,
                                const int32_t *score, const int64_t *ref_end, const int16_t *read_end,
                                const int32_t *best_score, const int64_t *best_slot, const int32_t *n_tied,
                                hipStream_t st);

}  // namespace swk
