// Traceback with one traced slot per lane (64 slots per wavefront).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sw_device.h"

namespace swk {

constexpr int kTraceRows = 32;  // rows per strip held in registers
constexpr int kTraceGroups = kTraceRows / 8;  // 32-bit words per column (8 cells of 4 bits)

struct TraceInterArgs {
  TraceArgs a;               // the common arguments (planes_* unused)
  const int32_t *cal_read;   // owner read of every CAL
  uint32_t *bits;            // per block: [strip][column][group][lane] words of 4-bit cell codes
  uint2 *bscr;               // per block: [column][lane] strip-boundary (H, F)
  int64_t bits_stride;       // words per block
  int64_t bscr_stride;       // entries per block
  int32_t wcap;              // widest window (columns)
  int32_t rwords, wwords;    // LDS words per lane for the read and the window
  int32_t beta;              // two-slots-per-lane kernel: bias of its int16 values
};

// Per-block device bytes of the one-slot-per-lane traceback for these shapes.
size_t trace_inter_block_bytes(int max_read_len, int wcap);
int trace_inter_blocks_per_cu();
hipError_t launch_trace_inter(const TraceInterArgs &A, const RefTable &T, int grid, hipStream_t st);

// Two traced slots per lane in int16 halves (128 slots per wavefront), when the
// layout holds the scoring's values (trace_pair_fits, which sets beta).
// Strip heights (rows per lane in registers) compiled for it; the one used is a
// function of the read-length bound.
#define SW_TRACE_PAIR_ROWS(X) X(24) X(28) X(32) X(34)
int trace_pair_rows(int max_read_len);
size_t trace_pair_block_bytes(int max_read_len, int wcap);
int trace_pair_blocks_per_cu(int max_read_len);
int trace_pair_fits(int match, int mismatch, int goe, int ge, int max_read_len, int wcap, int32_t *beta);
hipError_t launch_trace_pair(const TraceInterArgs &A, const RefTable &T, int grid, hipStream_t st);

}  // namespace swk
