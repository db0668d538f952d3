// Host-side launchers of the HIP kernels (defined in sw_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_device.h"

// Strip heights (read rows held in registers per lane) compiled for each kernel.
#define SW_INTER16_STRIPS(X) X(24) X(32) X(40) X(48) X(50) X(56)
#define SW_INTER32_STRIPS(X) X(24) X(32) X(38) X(48)

namespace swk {

hipError_t launch_pack(const uint8_t *codes, int64_t n, uint32_t *words, hipStream_t st);
hipError_t launch_expand(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, int32_t *cal_read,
                         hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_inter(bool int16, const AlignArgs &A, const RefTable &T, int grid, hipStream_t st);
hipError_t launch_reduce(const int64_t *cal_ptr, const int16_t *cal_ref, int32_t n_reads, int32_t n_refs,
                         const int32_t *score, int32_t *bs, int64_t *bl, int32_t *nt, hipStream_t st);
hipError_t launch_classify(const int32_t *bs, int32_t n_reads, int32_t n_refs, int32_t thr, int32_t *cls,
                           hipStream_t st);
// Resident waves of the inter kernel with R strip rows on this device (occupancy query).
int inter_blocks_per_cu(bool int16, int strip_rows);
// Address of the library's device-resident invalid-task counter on the current device.
unsigned long long *error_counter();

}  // namespace swk
