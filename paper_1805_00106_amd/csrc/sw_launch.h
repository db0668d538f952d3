// Host-side launchers of the HIP kernels (defined in sw_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_device.h"

// Strip heights (read rows held in registers per lane) compiled for each kernel.
#define SW_INTER16_STRIPS(X) X(24) X(32) X(40) X(44) X(48) X(50)
#define SW_INTER32_STRIPS(X) X(24) X(32) X(38) X(48)
// Strip heights available to the batched (work-queue) kernels, ascending.
#define SW_QUEUE16_STRIPS(X) X(24) X(32) X(34) X(36) X(38) X(40) X(42) X(44) X(46) X(48) X(50)
#define SW_QUEUE32_STRIPS(X) X(24) X(32) X(34) X(40) X(48) X(50)

namespace swk {

// Parameters of the length binning of the batched path.
struct BinParams {
  int32_t nb;            // number of length bins; bin nb collects invalid tasks
  int32_t bin_width;     // read lengths per bin
  int32_t max_read_len;
  int32_t per_cal;       // tasks per CAL: 1 (int16 pairs) or 2 (int32)
  int32_t descending;    // 1: longest bin first
  int32_t n_strips;      // compiled strip heights available
  int32_t strips[16];    // ascending
  int32_t strip_cap;     // tallest strip height a bin may take (0: any)
  int32_t strip_slack;   // padding rows worth one strip hand-over in the choice (0: padding only)
};

// Strip height of a length bin whose reads are at most `Lb` bases: among the
// compiled heights up to strip_cap (the lowest is always allowed), the one with
// the fewest padded rows plus strip_slack per strip, the taller on ties.  The
// planning kernel and the host's plan description both call it.
__host__ __device__ inline int bin_strip_height(const BinParams &P, int Lb) {
  int best = P.strips[0], best_cost = 0x7fffffff;
  for (int j = 0; j < P.n_strips; ++j) {
    const int R = P.strips[j];
    if (j > 0 && P.strip_cap > 0 && R > P.strip_cap) continue;
    const int ns = (Lb + R - 1) / R;
    const int cost = ns * R + P.strip_slack * ns;
    if (cost < best_cost || (cost == best_cost && R > best)) {
      best_cost = cost;
      best = R;
    }
  }
  return best;
}

// Device buffers of the batched path (owned by a context).
struct BatchBufs {
  int32_t *cal_read, *order;
  int32_t *bin_count, *bin_off, *bin_cursor, *tile_off, *tile_bin, *strip_of_bin;
  int32_t *tiles, *tile_len, *tile_strips;
  int32_t *n_tiles, *queue;
};

hipError_t launch_pack(const uint8_t *codes, int64_t n, uint32_t *words, hipStream_t st);
hipError_t launch_expand(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, int32_t *cal_read,
                         hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_inter(bool int16, const AlignArgs &A, const RefTable &T, int grid, hipStream_t st);
// Score Tracker launchers (sw_tracker.hip); CSR rows are clamped to [0, n_cals].
hipError_t launch_reduce(const int64_t *cal_ptr, const int16_t *cal_ref, int32_t n_reads, int32_t n_refs,
                         int64_t n_cals, const int32_t *score, int32_t *bs, int64_t *bl, int32_t *nt,
                         hipStream_t st);
hipError_t launch_topk(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, const int32_t *score, int32_t k,
                       int32_t *ts, int64_t *tl, hipStream_t st);
hipError_t launch_tied(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, const int32_t *score,
                       uint8_t *flags, hipStream_t st);
hipError_t launch_classify(const int32_t *bs, int32_t n_reads, int32_t n_refs, int32_t thr, int32_t *cls,
                           hipStream_t st);
// Resident waves of the inter kernel with R strip rows on this device (occupancy query).
int inter_blocks_per_cu(bool int16, int strip_rows);
hipError_t launch_batch_plan(const BatchBufs &B, const int32_t *read_len, int32_t n_reads, int64_t n_tasks,
                             const BinParams &P, hipStream_t st);
hipError_t launch_inter_queue(bool int16, const AlignArgs &A, const RefTable &T, int grid, hipStream_t st);
int queue_blocks_per_cu(bool int16);
// One wavefront per task: int32 (one strand per wavefront) or int16 pairs (one
// CAL per wavefront, both strands in the 16-bit halves).
hipError_t launch_intra(bool int16, const AlignArgs &A, const RefTable &T, int grid, hipStream_t st);
int intra_blocks_per_cu(bool int16, size_t lds);
// Traceback: LDS layout and plane storage of one launch.
constexpr size_t kTraceLdsLimit = 64 * 1024;  // plane buffers move to device memory above this
struct TracePlan {
  int q_bytes, win_words, run_cap;
  size_t planes_lds_off, planes_bytes, lds;
  bool lds_planes;
};
TracePlan trace_plan(int max_read_len, int wcap);
int trace_blocks_per_cu(const TracePlan &P);
hipError_t launch_trace(const TraceArgs &A, const RefTable &T, const TracePlan &P, int grid, hipStream_t st);
// Address of the library's device-resident invalid-task counter on the current device.
unsigned long long *error_counter();

}  // namespace swk
