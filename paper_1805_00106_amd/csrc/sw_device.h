// Device-side declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sw_align.h"

namespace swk {

// Reference table, copied into LDS by each wave at kernel start.
struct RefTable {
  int64_t word_off[SW_MAX_REFS];
  int64_t len[SW_MAX_REFS];
};

// Constants of the tagged dynamic program.
//
// Every DP value of column c is kept as N = V * 2^K + tag(c) with
// tag(c) = 2^K - 1 - (c mod 2^K): the low K bits name the column inside a tile
// of 2^K columns, so a max over values of one column orders by V exactly and a
// running max over a row orders by (V, then smallest column).  Moving one
// column right lowers the tag by one, so every penalty of a move that consumes
// a window base (diagonal, horizontal gap) carries an extra -1; vertical gap
// moves carry none.  With these constants every term reaching a cell carries
// that cell's tag, and the maximum needs no separate position bookkeeping.
//
// The int16 pairs also carry a bias: N = (V + beta) * 2^K + tag(c), with beta
// at least the largest single penalty (|mismatch|, gap_open + gap_extend + 1
// for the gap terms of a tile's last column, whose tag is -1, and the 256 of
// the padding rows), so that every operand of the three-way maxima of the
// sweep is a non-negative int16 below 0x7C00.  On those bit patterns the packed
// half-precision maximum orders exactly as the integer one (they are the finite
// non-negative halves, in increasing order), so H = max(diagonal, E, F) and the
// clamped gap term E = max(E - ge, H - go - ge, 0) are one v_pk_maximum3_f16
// each; a wall column (substitution 0x8000) makes the diagonal operand a
// negative half, below every other operand.
//
// In the one-CAL-per-lane sweep, row r of a strip (r < kInt16StripRowsMax)
// further carries r * gap_extend * 2^K.  A vertical gap move then keeps its
// value (F = max(F, H - gap_open)), a diagonal move carries + gap_extend * 2^K in
// its substitution, and the zero of row r is the column's zero plus the row's
// offset (a wave-uniform value).  K is the largest of 6, 5, 4 for which
// (beta + top + 1 + (kInt16StripRowsMax - 1) * gap_extend) * 2^K stays below
// 0x7C00, top = match * (longest read): chosen for the call's read-length bound,
// and again per tile of 64 CALs for the tile's longest read (shorter reads allow
// the wider tag).
constexpr int kInt16StripRowsMax = 50;

struct DpConst {
  // int16 pairs, both halves hold the same constant
  uint32_t goe_e16, ge_e16, goe_f16, ge_f16;  // ge_f16 is also the row step
  uint32_t tag16;    // 2^K
  uint32_t bias16;   // beta * 2^K
  int32_t kbits16;   // K
  int32_t beta16;    // beta
  uint32_t xlo, dlo, xhi, dhi;  // substitution (with the row step) table bytes
  int32_t match, mismatch, goe, ge;  // the scoring (goe = gap_open + gap_extend)
  // int32 (K = 12)
  int32_t goe_e32, ge_e32, goe_f32, ge_f32, sm32, sx32, e0_32;
  // int32 substitution by byte permutation in the one-CAL-per-lane sweep, whose
  // diagonal moves also carry the row step gap_extend * 4096: usable when s' = s +
  // gap_extend lies in [-15, 16] for both scores.  s' * 4096 - 1 is then 0xFF in
  // byte 0, a score-dependent byte 1 and the sign in bytes 2 and 3, so a table of
  // byte 1 (low word) and of the sign byte (high word) per base yields it with one
  // v_perm_b32
  int32_t perm32;
  uint32_t xlo32, dlo32, xhi32, dhi32;
  // 1: only the last read row may hold the best cell (read-end-anchored scoring)
  int32_t final_row;
};

// Sets the int16 fields of K for the widest tag whose biased values hold scores
// up to `top`; returns 0 (leaving K unchanged) if no width does.
__host__ __device__ inline int set_int16_layout(DpConst &K, int64_t top) {
  for (int kb = 6; kb >= 4; --kb) {
    const int32_t U = 1 << kb;
    int32_t b = -K.mismatch;
    if (K.goe + 1 > b) b = K.goe + 1;
    // the padding rows' substitution (-256) on a strip's row 0, whose diagonal
    // operand is handed over as H - gap_extend * 2^K
    if ((256 + U - 1) / U + K.ge > b) b = (256 + U - 1) / U + K.ge;
    const int64_t rows = (int64_t)(kInt16StripRowsMax - 1) * K.ge;
    if (b > 0x7BFF || ((int64_t)b + top + 1 + rows) * U > 0x7BFF) continue;
    const uint32_t pair1 = 0x00010001u;
    K.goe_e16 = (uint32_t)(uint16_t)(K.goe * U + 1) * pair1;
    K.ge_e16 = (uint32_t)(uint16_t)(K.ge * U + 1) * pair1;
    K.goe_f16 = (uint32_t)(uint16_t)(K.goe * U) * pair1;
    K.ge_f16 = (uint32_t)(uint16_t)(K.ge * U) * pair1;
    K.tag16 = (uint32_t)U * pair1;
    K.bias16 = (uint32_t)(b * U) * pair1;
    K.kbits16 = kb;
    K.beta16 = b;
    // substitution s * 2^K - 1 (the tag step of a diagonal move) plus the row
    // step gap_extend * 2^K, as bytes
    const uint32_t sm = (uint16_t)((K.match + K.ge) * U - 1), sx = (uint16_t)((K.mismatch + K.ge) * U - 1);
    const uint32_t lo_m = sm & 0xFFu, hi_m = sm >> 8, lo_x = sx & 0xFFu, hi_x = sx >> 8;
    K.xlo = lo_x * 0x01010101u;
    K.dlo = lo_x ^ lo_m;
    K.xhi = hi_x * 0x01010101u;
    K.dhi = hi_x ^ hi_m;
    return 1;
  }
  return 0;
}

struct AlignArgs {
  const uint32_t *reads;
  const int64_t *read_word_off;
  const int32_t *read_len;
  int32_t n_reads;
  int32_t n_refs;
  const uint32_t *ref_words;
  const int64_t *cal_pos;
  const int16_t *cal_ref;
  const uint8_t *strand;
  const int32_t *cal_read;  // owning read of each CAL (from the expansion kernel)
  const int32_t *order;     // task position -> CAL index; null means identity
  int64_t n_cals;
  int64_t n_tasks;          // lanes to run (CALs for int16 pairs, 2*CALs for int32)
  int32_t *score;
  int64_t *ref_end;
  int16_t *read_end;
  uint2 *scratch;           // strip-boundary rows, [grid][wcap][64]
  unsigned long long *err;  // invalid-task counter
  const int32_t *tiles;     // batched: [n_tiles] first task position of each tile (64 tasks max)
  const int32_t *tile_len;  // batched: tasks in each tile
  const int32_t *tile_strips; // batched: strip rows R of each tile
  int32_t *queue;           // batched: tile counter (work queue), null for static striding
  const int32_t *n_tiles_dev; // batched: number of tiles (device), null -> ceil(n_tasks/64)
  int32_t wcap;             // widest window (columns) of the call
  int32_t wwords;           // LDS words per lane for the window
  int32_t rwords;           // LDS words per lane for the read
  int32_t max_read_len;
  int32_t band;
  int32_t strip_rows;       // R of the launch (plain path)
  DpConst k;
};

// Traceback launch (start position and CIGAR of selected slots).
struct TraceArgs {
  const uint32_t *reads;
  const int64_t *read_word_off;
  const int32_t *read_len;
  int32_t n_reads;
  int32_t n_refs;
  const uint32_t *ref_words;
  const int64_t *cal_ptr;
  const int64_t *cal_pos;
  const int16_t *cal_ref;
  int64_t n_cals;
  const int32_t *score;      // scoring outputs, indexed by slot
  const int64_t *ref_end;
  const int16_t *read_end;
  const int64_t *slots;      // [n_slots] slot to trace, -1 to skip
  int64_t n_slots;
  int32_t cap;               // CIGAR entries per traced slot
  int64_t *ref_start;
  int16_t *read_start;
  int32_t *n_ops;
  uint32_t *cigar;           // [n_slots][cap]
  uint64_t *planes_global;   // per-block plane buffers when they do not fit in LDS
  int64_t planes_stride;     // 64-bit words per block in planes_global
  unsigned long long *err;
  int32_t max_read_len, band;
  int32_t match, mismatch, goe, ge;
  int32_t q_bytes, win_words, run_cap;
  int64_t planes_lds_off;
};

}  // namespace swk
