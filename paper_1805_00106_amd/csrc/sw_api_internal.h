// Internal helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/sw_align.h"
#include "sw_device.h"

namespace swapi {

struct ScoreMode {
  bool int16;
  int max_read_len;
  int wcap;  // widest window: max_read_len + 2 * band
};

struct PlainPlan {
  ScoreMode mode;
  bool intra;  // one wavefront per task instead of one CAL per lane
  int strip_rows;
  int64_t n_tasks;
  int wwords, rwords;
  int grid;
  size_t cal_read_off, scratch_off, bytes;
  size_t queue_off;  // one CAL per lane: the tile counter the blocks pop from (zeroed per call)
};

typedef swk::DpConst DpConstHost;

extern thread_local int g_last_hip;
int hip_fail(hipError_t e);
int validate_scoring(const sw_scoring_t *sc, ScoreMode *mode);
int validate_refs(const sw_refset_t *refs, int64_t n_cals, swk::RefTable *T);
int validate_batch(const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                   int32_t n_reads, const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref,
                   const uint8_t *strand, int64_t n_cals, int32_t *score, int64_t *ref_end,
                   int16_t *read_end);
DpConstHost make_consts(const sw_scoring_t *sc);
// int16 pairs: tag bits K (6, 5 or 4) and bias beta of the scoring; 0 if none fits
int int16_layout(const sw_scoring_t *sc, int32_t *kbits, int32_t *beta);
int choose_strip_rows(bool int16, int rows);
int strip_rows_supported(bool int16, int R);
int device_cus();
int blocks_per_cu(bool int16, int R);
int make_plan(int64_t n_cals, const sw_scoring_t *sc, int strip_override, PlainPlan *p);
// AUTO kernel choice: one wavefront per task while the call needs at most this
// many wavefronts per compute unit (one per CAL in int16 pairs, two in int32)
constexpr int kIntraWavesPerCu = 64;

}  // namespace swapi
