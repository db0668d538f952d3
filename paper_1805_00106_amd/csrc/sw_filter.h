// CAL Filter launchers (duplicate CALs of a read folded into one lookup).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace swk {

struct FilterArgs {
  const int64_t *cal_ptr;
  const int64_t *cal_pos;
  const int16_t *cal_ref;
  const uint8_t *strand;
  int32_t n_reads;
  int64_t n_cals;
  int32_t bucket_bits;
  int64_t *out_ptr;
  int64_t *out_pos;
  int16_t *out_ref;
  uint8_t *out_strand;
  int64_t *cal_map;
};

// Workspace of launch_filter for n_reads reads (counts + scan temporary storage).
size_t filter_workspace_bytes(int32_t n_reads);
hipError_t launch_filter(const FilterArgs &A, void *workspace, size_t workspace_bytes, hipStream_t st);

}  // namespace swk
