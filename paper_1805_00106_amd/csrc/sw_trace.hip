// Traceback kernel for gfx950: start position and CIGAR of selected tasks.
//
// One wavefront per traced slot.  The task's dynamic program is rebuilt over
// the rectangle that ends at its reported end cell (rows 0..read_end, window
// columns 0..ref_end - ws): every value of that rectangle depends only on
// cells above and to the left, so it equals the scoring pass.  Lane j holds
// window column 64*s + j of strip s and the strip is swept along
// anti-diagonals (step t: lane j computes row t - j), as in the wavefront-
// per-task scoring kernel but with plain int32 values: no position tracking is
// needed here.
//
// Each step stores four 64-bit ballots (one bit per lane, so one bit per
// cell) to a plane buffer:
//   P0, P1  source of H(i,j):  0 diagonal, 1 gap consuming a read base (F),
//           2 gap consuming a window base (E), 3 H(i,j) = 0
//           (the first source in this order that reaches the value)
//   P2      E(i,j+1) is opened from H(i,j)  (open preferred on a tie)
//   P3      F(i+1,j) is opened from H(i,j)  (open preferred on a tie)
// The walk then runs backwards from the end cell with those rules; it is wave
// uniform and its only memory traffic is one plane word per move.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_device.h"
#include "sw_halfmax.h"
#include "sw_launch.h"

namespace swk {

namespace {

__device__ __forceinline__ int32_t shr1(int32_t old, int32_t src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xf, 0xf, false);  // wave_shr:1
}

// Owner read of CAL c: the r with cal_ptr[r] <= c < cal_ptr[r+1], by a 64-way
// search (each round the lanes probe 64 evenly spaced row pointers).  Returns
// -1 when c is outside [cal_ptr[0], cal_ptr[n_reads]).  Terminates for any
// contents of cal_ptr: the interval shrinks every round.
__device__ int64_t owner_read(const int64_t *cal_ptr, int32_t n_reads, int64_t c, int lane) {
  if (n_reads < 1 || c < cal_ptr[0] || c >= cal_ptr[n_reads]) return -1;
  int64_t lo = 0, hi = n_reads;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t p = lo + (int64_t)lane * step;
    const bool le = p < hi && cal_ptr[p] <= c;
    const uint64_t m = __ballot(le);
    const int k = 63 - __builtin_clzll(m | 1ull);
    const int64_t nlo = lo + (int64_t)k * step;
    hi = nlo + step < hi ? nlo + step : hi;
    lo = nlo;
  }
  return lo;
}

__device__ __forceinline__ int plane_bit(const uint64_t *planes, int stride, int i, int j, int k) {
  const int s = j >> 6, l = j & 63;
  return (int)((planes[((int64_t)s * stride + i + l) * 4 + k] >> l) & 1ull);
}

}  // namespace

template <bool LDS_PLANES>
__global__ __launch_bounds__(64) void k_trace(const TraceArgs A, const RefTable T) {
  extern __shared__ __align__(16) uint8_t tsm[];
  __shared__ int64_t rt_off[SW_MAX_REFS], rt_len[SW_MAX_REFS];
  const int lane = threadIdx.x;
  for (int i = 0; i < A.n_refs; ++i)
    if (lane == i) {
      rt_off[i] = T.word_off[i];
      rt_len[i] = T.len[i];
    }
  __syncthreads();
  // LDS: rows (H, E of lane 63 per row) | read codes | window words | runs | planes
  int2 *rows = reinterpret_cast<int2 *>(tsm);
  uint8_t *qc = tsm + 8 * A.max_read_len;
  uint32_t *win = reinterpret_cast<uint32_t *>(qc + A.q_bytes);
  uint32_t *runs = win + A.win_words;
  uint64_t *planes = LDS_PLANES ? reinterpret_cast<uint64_t *>(tsm + A.planes_lds_off)
                                : A.planes_global + (size_t)blockIdx.x * A.planes_stride;
  const int32_t goe = A.goe, ge = A.ge;

  for (int64_t t = blockIdx.x; t < A.n_slots; t += gridDim.x) {
    const int64_t slot = A.slots[t];
    int32_t status = 0;  // 0 ok, -2 invalid
    if (slot == -1) {
      if (lane == 0) {
        A.ref_start[t] = -1;
        A.read_start[t] = -1;
        A.n_ops[t] = 0;
      }
      continue;
    }
    int64_t r = -1;
    int L = 0, k = 0, ie = 0, je = 0, n_cols = 0, h = 0;
    int64_t ws = 0, p = 0;
    int32_t sc = 0;
    if (slot < 0 || slot >= 2 * A.n_cals) {
      status = -2;
    } else {
      sc = A.score[slot];
      if (sc > 0) {
        const int64_t c = slot >> 1;
        h = (int)(slot & 1);
        r = owner_read(A.cal_ptr, A.n_reads, c, lane);
        if (r < 0) {
          status = -2;
        } else {
          L = A.read_len[r];
          k = A.cal_ref[c];
          p = A.cal_pos[c];
          if (L < 1 || L > A.max_read_len || k < 0 || k >= A.n_refs || p < 0 || p >= rt_len[k]) {
            status = -2;
          } else {
            ws = p - A.band < 0 ? 0 : p - A.band;
            const int64_t we = min(rt_len[k], p + L + A.band);
            const int W = (int)(we - ws);
            ie = A.read_end[slot];
            const int64_t je64 = A.ref_end[slot] - ws;
            if (ie < 0 || ie >= L || je64 < 0 || je64 >= W) status = -2;
            je = (int)je64;
            n_cols = je + 1;
          }
        }
      }
    }
    if (status != 0 || sc <= 0) {
      if (lane == 0) {
        A.ref_start[t] = -1;
        A.read_start[t] = -1;
        A.n_ops[t] = status;
        if (status) atomicAdd(A.err, 1ull);
      }
      continue;
    }
    const int n_rows = ie + 1;
    __syncthreads();
    // stage the oriented read rows and the window columns of the rectangle
    {
      const uint32_t *rp = A.reads + A.read_word_off[r];
      for (int i = lane; i < n_rows; i += 64) {
        const int src = h == 0 ? i : L - 1 - i;
        const uint32_t b = (rp[src >> 4] >> (2 * (src & 15))) & 3u;
        qc[i] = (uint8_t)(h == 0 ? b : 3u - b);
      }
      const int64_t first = rt_off[k] + (ws >> 4);
      const int64_t last = rt_off[k] + ((rt_len[k] - 1) >> 4);
      const uint32_t sh = 2u * (uint32_t)(ws & 15);
      const int nww = (n_cols + 15) >> 4;
      for (int q = lane; q < nww; q += 64) {
        const uint32_t lo = A.ref_words[first + q];
        const uint32_t hi = (first + q + 1 <= last) ? A.ref_words[first + q + 1] : 0u;
        win[q] = (uint32_t)((((uint64_t)hi << 32) | lo) >> sh);
      }
    }
    __syncthreads();

    // ---- sweep
    const int stride = n_rows + 63;  // steps per strip in the plane buffer
    const int nstrips = (n_cols + 63) >> 6;
    int32_t endv = 0;
    for (int s = 0; s < nstrips; ++s) {
      const int col = 64 * s + lane;
      const int32_t w = col < n_cols ? (int32_t)((win[col >> 4] >> (2 * (col & 15))) & 3u) : 5;
      const int width = min(64, n_cols - 64 * s);
      const int nsteps = n_rows + width - 1;
      int32_t H = 0;          // lane's H of its last row (row -1: 0)
      int32_t Hd1 = 0;        // H(i-1, col-1) for the coming step
      int32_t F = -goe;       // F(0, col)
      int32_t Eout = 0, q = 0;
      for (int st = 0; st < nsteps; ++st) {
        int32_t q_b = 4, e_b = -goe, h_b = 0;
        if (st < n_rows) {
          q_b = qc[st];
          if (s > 0) {
            const int2 rb = rows[st];
            h_b = rb.x;
            e_b = rb.y;
          }
        }
        q = shr1(q_b, q);
        const int32_t Ein = shr1(e_b, Eout);
        const int32_t Hs = shr1(h_b, H);
        const int i = st - lane;
        const bool act = i >= 0 && i < n_rows && col < n_cols;
        bool b0 = false, b1 = false, eo = false, fo = false;
        if (act) {
          const int32_t diag = Hd1 + (q == w ? A.match : A.mismatch);
          const int32_t Hn = max(max(diag, Ein), max(F, 0));
          const bool z = Hn == 0;
          const bool d = !z && Hn == diag;
          const bool fsrc = Hn == F;
          b0 = z || (!d && fsrc);
          b1 = z || (!d && !fsrc);
          const int32_t U = Hn - goe;
          eo = U >= Ein - ge;
          fo = U >= F - ge;
          Eout = max(Ein - ge, U);
          F = max(F - ge, U);
          H = Hn;
          if (lane == 63) rows[i] = make_int2(Hn, Eout);
          if (i == ie && col == je) endv = Hn;
        }
        Hd1 = Hs;
        const uint64_t P0 = __ballot(b0), P1 = __ballot(b1), P2 = __ballot(eo), P3 = __ballot(fo);
        if (lane == 0) {
          ulonglong2 *dst = reinterpret_cast<ulonglong2 *>(planes + ((int64_t)s * stride + st) * 4);
          dst[0] = make_ulonglong2(P0, P1);
          dst[1] = make_ulonglong2(P2, P3);
        }
      }
      __syncthreads();
    }
    endv = __shfl(endv, je & 63, 64);
    if (endv != sc) {
      if (lane == 0) {
        A.ref_start[t] = -1;
        A.read_start[t] = -1;
        A.n_ops[t] = -2;
        atomicAdd(A.err, 1ull);
      }
      continue;
    }

    // ---- walk (wave uniform), runs collected end first
    int n = 0;
    uint32_t cur_op = 0, cur_len = 0;
    auto emit = [&](uint32_t op) {
      if (op == cur_op) {
        ++cur_len;
      } else {
        if (cur_len) {
          if (lane == 0 && n < A.run_cap) runs[n] = (cur_len << 4) | cur_op;
          ++n;
        }
        cur_op = op;
        cur_len = 1;
      }
    };
    if (L - 1 - ie > 0) {
      cur_op = 4;
      cur_len = (uint32_t)(L - 1 - ie);
    }
    int i = ie, j = je, state = 0;  // 0 H, 1 F, 2 E
    for (;;) {
      if (state == 0) {
        if (i < 0 || j < 0) break;
        const int code = plane_bit(planes, stride, i, j, 0) | (plane_bit(planes, stride, i, j, 1) << 1);
        if (code == 3) break;
        if (code == 0) {
          const uint32_t wb = (win[j >> 4] >> (2 * (j & 15))) & 3u;
          emit(qc[i] == wb ? 7u : 8u);
          --i;
          --j;
        } else {
          state = code;
        }
      } else if (state == 1) {
        // F(i,j) opened from H(i-1,j)?  (row 0 cannot be in a gap: F(0,j) < 0)
        emit(1u);
        if (i == 0 || plane_bit(planes, stride, i - 1, j, 3)) state = 0;
        --i;
      } else {
        // E(i,j) opened from H(i,j-1)?  (column 0 likewise)
        emit(2u);
        if (j == 0 || plane_bit(planes, stride, i, j - 1, 2)) state = 0;
        --j;
      }
    }
    // (i, j) is the cell before the first aligned pair
    const int read_start = i + 1;
    if (read_start > 0) {  // the head clip covers every unaligned read base
      emit(4u);
      cur_len = (uint32_t)read_start;
    }
    if (lane == 0 && n < A.run_cap) runs[n] = (cur_len << 4) | cur_op;
    ++n;
    __syncthreads();
    if (n > A.cap) {
      uint32_t *out = A.cigar + t * (int64_t)A.cap;
      for (int x = lane; x < A.cap; x += 64) out[x] = 0u;  // an over-capacity row is cleared
      if (lane == 0) {
        A.ref_start[t] = -1;
        A.read_start[t] = -1;
        A.n_ops[t] = -1;
      }
    } else {
      uint32_t *out = A.cigar + t * (int64_t)A.cap;
      for (int x = lane; x < n; x += 64) out[x] = runs[n - 1 - x];
      if (lane == 0) {
        A.ref_start[t] = ws + j + 1;
        A.read_start[t] = (int16_t)read_start;
        A.n_ops[t] = n;
      }
    }
    __syncthreads();
  }
}

TracePlan trace_plan(int max_read_len, int wcap) {
  TracePlan P{};
  P.q_bytes = (max_read_len + 15) / 16 * 16;
  P.win_words = wcap / 16 + 2;
  P.run_cap = max_read_len + wcap + 2;
  const size_t head = 8 * (size_t)max_read_len + P.q_bytes + 4 * (size_t)(P.win_words + P.run_cap);
  P.planes_lds_off = (head + 31) / 32 * 32;
  const int nstrips = (wcap + 63) / 64;
  P.planes_bytes = (size_t)nstrips * (size_t)(max_read_len + 63) * 32;
  P.lds_planes = P.planes_lds_off + P.planes_bytes <= kTraceLdsLimit;
  P.lds = P.lds_planes ? P.planes_lds_off + P.planes_bytes : P.planes_lds_off;
  return P;
}

int trace_blocks_per_cu(const TracePlan &P) {
  int n = 0;
  const void *f = P.lds_planes ? reinterpret_cast<const void *>(&k_trace<true>)
                               : reinterpret_cast<const void *>(&k_trace<false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64, P.lds) != hipSuccess) return 1;
  return n < 1 ? 1 : n;
}

hipError_t launch_trace(const TraceArgs &A, const RefTable &T, const TracePlan &P, int grid, hipStream_t st) {
  if (A.n_slots == 0) return hipSuccess;
  if (P.lds_planes)
    hipLaunchKernelGGL(k_trace<true>, dim3(grid), dim3(64), P.lds, st, A, T);
  else
    hipLaunchKernelGGL(k_trace<false>, dim3(grid), dim3(64), P.lds, st, A, T);
  return hipGetLastError();
}

}  // namespace swk

// --------------------------------------------------------------------------- one slot per lane
//
// The wavefront traces 64 slots at once, one per lane, with the read rows of a
// strip in registers and the window columns swept left to right, as in the
// scoring kernels (plain int32 values: the end cell is known).  For every
// cell the lane records 4 bits: the source of H (0 diagonal, 1 F, 2 E, 3
// diagonal from a zero cell or the boundary, i.e. the first aligned pair) and
// whether the E and F leaving the cell are opened from its H.  Eight cells of
// a column form one 32-bit word per lane, stored coalesced as
// [strip][column][group][lane] in the block's device buffer; each lane then
// walks its own path back through its words.

#include "sw_trace.h"

namespace swk {

namespace {

__device__ __forceinline__ uint32_t code_at(const uint32_t *bits, int cmax, int lane, int i, int j) {
  const int s = i / kTraceRows, r = i - s * kTraceRows;
  const uint32_t w = bits[(((int64_t)s * cmax + j) * kTraceGroups + (r >> 3)) * 64 + lane];
  return (w >> (4 * (r & 7))) & 15u;
}

}  // namespace

// P: substitution by byte permutation (both scores within -128..127): a table of
// the score's low byte and of its sign byte per base, built per column, gives
// the sign-extended score with one v_perm_b32; else compare and select.  With P
// the rows below a lane's end row and the columns right of its end column take
// ordinary substitutions: no cell of the traced rectangle depends on them.
template <bool P>
__global__ __launch_bounds__(64) void k_trace_inter(const TraceInterArgs I, const RefTable T) {
  extern __shared__ uint32_t tism[];
  __shared__ int64_t rt_off[SW_MAX_REFS], rt_len[SW_MAX_REFS];
  const TraceArgs &A = I.a;
  const int lane = threadIdx.x;
  for (int i = 0; i < A.n_refs; ++i)
    if (lane == i) {
      rt_off[i] = T.word_off[i];
      rt_len[i] = T.len[i];
    }
  __syncthreads();
  uint32_t *rdw = tism;                  // [rwords][64] read words
  uint32_t *win = tism + I.rwords * 64;  // [wwords][64] window words
  uint32_t *bits = I.bits + (size_t)blockIdx.x * I.bits_stride;
  uint2 *bscr = I.bscr + (size_t)blockIdx.x * I.bscr_stride;
  const int32_t goe = A.goe, ge = A.ge;
  // substitution tables (P): low byte and sign byte of the score, per base
  const uint32_t lo_m = (uint32_t)A.match & 0xFFu, lo_x = (uint32_t)A.mismatch & 0xFFu;
  const uint32_t hi_m = A.match < 0 ? 0xFFu : 0u, hi_x = A.mismatch < 0 ? 0xFFu : 0u;
  const uint32_t xlo = lo_x * 0x01010101u, dlo = lo_x ^ lo_m, xhi = hi_x * 0x01010101u, dhi = hi_x ^ hi_m;

  for (int64_t first = (int64_t)blockIdx.x * 64; first < A.n_slots; first += (int64_t)gridDim.x * 64) {
    const int64_t t = first + lane;
    // ---- this lane's task; n_rows = 0 leaves the lane idle
    int status = 0, L = 0, h = 0, k = 0, ie = -1, je = -1;
    int64_t r = -1, ws = 0, slot = -1;
    int32_t sc = 0;
    bool live = false;
    if (t < A.n_slots) {
      slot = A.slots[t];
      if (slot != -1) {
        if (slot < 0 || slot >= 2 * A.n_cals) {
          status = -2;
        } else if ((sc = A.score[slot]) > 0) {
          const int64_t c = slot >> 1;
          h = (int)(slot & 1);
          r = I.cal_read[c];
          const int64_t p = A.cal_pos[c];
          k = A.cal_ref[c];
          L = r >= 0 && r < A.n_reads ? A.read_len[r] : 0;
          if (r < 0 || L < 1 || L > A.max_read_len || k < 0 || k >= A.n_refs || p < 0 || p >= rt_len[k]) {
            status = -2;
          } else {
            ws = p - A.band < 0 ? 0 : p - A.band;
            const int64_t we = min(rt_len[k], p + L + A.band);
            ie = A.read_end[slot];
            const int64_t je64 = A.ref_end[slot] - ws;
            if (ie < 0 || ie >= L || je64 < 0 || je64 >= we - ws) status = -2;
            else {
              je = (int)je64;
              live = true;
            }
          }
        }
      }
      if (!live) {
        A.ref_start[t] = -1;
        A.read_start[t] = -1;
        A.n_ops[t] = status;
        if (status) atomicAdd(A.err, 1ull);
      }
    }
    const int n_rows = live ? ie + 1 : 0, n_cols = live ? je + 1 : 0;
    int rmax = n_rows, cmax = n_cols, lmax = live ? L : 0;
    for (int m = 32; m; m >>= 1) {
      rmax = max(rmax, __shfl_xor(rmax, m, 64));
      cmax = max(cmax, __shfl_xor(cmax, m, 64));
      lmax = max(lmax, __shfl_xor(lmax, m, 64));
    }
    if (rmax == 0) continue;
    // ---- stage the lane's read and window words ([word][lane] in LDS); the whole
    // read is needed: a reverse-strand row i reads original base L-1-i
    __syncthreads();
    {
      const int nrw = (lmax + 15) >> 4, nww = (cmax + 15) >> 4;
      if (live) {
        const uint32_t *rp = A.reads + A.read_word_off[r];
        const int lw = (L + 15) >> 4;
        for (int q = 0; q < nrw; ++q) rdw[q * 64 + lane] = q < lw ? rp[q] : 0u;
        const int64_t fw = rt_off[k] + (ws >> 4);
        const int64_t last = rt_off[k] + ((rt_len[k] - 1) >> 4);
        const uint32_t sh = 2u * (uint32_t)(ws & 15);
        uint32_t lo = A.ref_words[fw];
        for (int q = 0; q < nww; ++q) {
          const uint32_t hi = fw + q + 1 <= last ? A.ref_words[fw + q + 1] : 0u;
          win[q * 64 + lane] = (uint32_t)((((uint64_t)hi << 32) | lo) >> sh);
          lo = hi;
        }
      } else {
        for (int q = 0; q < nrw; ++q) rdw[q * 64 + lane] = 0u;
        for (int q = 0; q < nww; ++q) win[q * 64 + lane] = 0u;
      }
    }
    __syncthreads();
    auto qbase = [&](int i) -> int32_t {  // oriented read base of row i
      const int src = h == 0 ? i : L - 1 - i;
      const int32_t b = (int32_t)((rdw[(src >> 4) * 64 + lane] >> (2 * (src & 15))) & 3u);
      return h == 0 ? b : 3 - b;
    };
    auto wbase = [&](int j) -> int32_t {
      return (int32_t)((win[(j >> 4) * 64 + lane] >> (2 * (j & 15))) & 3u);
    };

    // ---- sweep: strips of kTraceRows rows, columns left to right
    int32_t endv = -1;
    const int nstrips = (rmax + kTraceRows - 1) / kTraceRows;
    for (int s = 0; s < nstrips; ++s) {
      const int r0 = s * kTraceRows;
      int32_t q[kTraceRows], Hl[kTraceRows], E[kTraceRows];
#pragma unroll
      for (int x = 0; x < kTraceRows; ++x) {
        if (P) {
          const int32_t b = r0 + x < n_rows ? qbase(r0 + x) : 0;
          q[x] = b | ((b | 4) << 8) | ((b | 4) << 16) | ((b | 4) << 24);  // selector
        } else {
          q[x] = r0 + x < n_rows ? qbase(r0 + x) : 4;  // 4 never equals a window base
        }
        Hl[x] = 0;                                    // H(i, -1)
        E[x] = -goe;                                  // E(i, 0)
      }
      int32_t hup_prev = 0;  // H(r0 - 1, -1)
      if (s > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      for (int c = 0; c < cmax; ++c) {
        const int32_t w = P ? wbase(c) : (c < n_cols ? wbase(c) : 5);
        uint32_t tlo = 0, thi = 0;
        if (P) {
          const uint32_t sh8 = (uint32_t)w << 3;
          tlo = xlo ^ (dlo << sh8);
          thi = xhi ^ (dhi << sh8);
        }
        int32_t hup, F;
        if (s == 0) {
          hup = 0;
          F = -goe;
        } else {
          const uint2 b = bscr[c * 64 + lane];
          hup = (int32_t)b.x;
          F = (int32_t)b.y;
        }
        int32_t Hd = hup_prev;
        hup_prev = hup;
        uint32_t word[kTraceGroups];
#pragma unroll
        for (int x = 0; x < kTraceRows; ++x) {
          const int32_t diag =
              Hd + (P ? (int32_t)__builtin_amdgcn_perm(thi, tlo, (uint32_t)q[x]) : (q[x] == w ? A.match : A.mismatch));
          const int32_t H = max(max(diag, E[x]), max(F, 0));
          const uint32_t code = H == diag ? (Hd == 0 ? 3u : 0u) : (H == F ? 1u : 2u);
          const int32_t U = H - goe;
          const int32_t e2 = E[x] - ge, f2 = F - ge;
          const bool eo = U >= e2, fo = U >= f2;
          E[x] = eo ? U : e2;
          F = fo ? U : f2;
          const uint32_t nib = code | (eo ? 4u : 0u) | (fo ? 8u : 0u);
          if ((x & 7) == 0)
            word[x >> 3] = nib;
          else
            word[x >> 3] |= nib << (4 * (x & 7));
          Hd = Hl[x];
          Hl[x] = H;
        }
#pragma unroll
        for (int g = 0; g < kTraceGroups; ++g) bits[(((int64_t)s * cmax + c) * kTraceGroups + g) * 64 + lane] = word[g];
        if (s + 1 < nstrips) bscr[c * 64 + lane] = make_uint2((uint32_t)Hl[kTraceRows - 1], (uint32_t)F);
        if (c == je && ie >= r0 && ie < r0 + kTraceRows) {
#pragma unroll
          for (int x = 0; x < kTraceRows; ++x)
            if (ie == r0 + x) endv = Hl[x];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __syncthreads();
    }

    // ---- walk (each lane its own path); runs go to the output row end first
    if (live) {
      if (endv != sc) {
        A.ref_start[t] = -1;
        A.read_start[t] = -1;
        A.n_ops[t] = -2;
        atomicAdd(A.err, 1ull);
      } else {
        uint32_t *out = A.cigar + t * (int64_t)A.cap;
        int n = 0;
        uint32_t cur_op = 0, cur_len = 0;
        auto flush = [&]() {
          if (cur_len) {
            if (n < A.cap) out[n] = (cur_len << 4) | cur_op;
            ++n;
          }
        };
        auto emit = [&](uint32_t op) {
          if (op != cur_op) {
            flush();
            cur_op = op;
            cur_len = 0;
          }
          ++cur_len;
        };
        if (L - 1 - ie > 0) {
          cur_op = 4;
          cur_len = (uint32_t)(L - 1 - ie);
        }
        int i = ie, j = je, state = 0, start_i = 0, start_j = 0;
        for (;;) {
          if (state == 0) {
            const uint32_t code = code_at(bits, cmax, lane, i, j) & 3u;
            if (code == 0u || code == 3u) {
              emit(qbase(i) == wbase(j) ? 7u : 8u);
              if (code == 3u) {
                start_i = i;
                start_j = j;
                break;
              }
              --i;
              --j;
              if (i < 0 || j < 0) {  // cannot happen: a diagonal from the boundary has code 3
                start_i = i + 1;
                start_j = j + 1;
                break;
              }
            } else {
              state = (int)code;
            }
          } else if (state == 1) {
            emit(1u);
            if (i == 0 || (code_at(bits, cmax, lane, i - 1, j) & 8u)) state = 0;
            --i;
            if (i < 0) break;  // cannot happen for a consistent matrix
          } else {
            emit(2u);
            if (j == 0 || (code_at(bits, cmax, lane, i, j - 1) & 4u)) state = 0;
            --j;
            if (j < 0) break;  // cannot happen for a consistent matrix
          }
        }
        if (start_i > 0) {
          emit(4u);
          cur_len = (uint32_t)start_i;
        }
        flush();
        if (n > A.cap) {
          for (int x = 0; x < A.cap; ++x) out[x] = 0u;  // an over-capacity row is cleared
          A.ref_start[t] = -1;
          A.read_start[t] = -1;
          A.n_ops[t] = -1;
        } else {
          for (int x = 0; x < n / 2; ++x) {
            const uint32_t a = out[x];
            out[x] = out[n - 1 - x];
            out[n - 1 - x] = a;
          }
          A.ref_start[t] = ws + start_j;
          A.read_start[t] = (int16_t)start_i;
          A.n_ops[t] = n;
        }
      }
    }
  }
}

// --------------------------------------------------------------------------- two slots per lane
//
// Two traced slots per lane in the 16-bit halves of every register (low half:
// slot first + lane, high half: slot first + 64 + lane), the rows of a strip
// in registers and the window columns swept left to right as in
// k_trace_inter.  Every value V of window column j is held as
// 16 * (V + beta + j * c) + tag, with c = -mismatch and beta at least
// |mismatch|, gap_open + gap_extend and gap_extend:
//   * with the column offset c every substitution plus c is non-negative, so a
//     per-column byte table of 16 * (s + c) + 8 per read base gives both halves'
//     diagonal terms with one v_perm_b32 (the high bytes select 0x00);
//   * every move that consumes a window base (diagonal, gap along the read's
//     row) adds c, a move down the column adds none, so every term reaching
//     cell (i, j) carries j * c and the zero of column j is 16 * (beta + j * c);
//   * beta keeps every operand of the three-way maxima non-negative and below
//     0x7C00, where the packed half-precision maximum orders exactly as the
//     integer one, so H = max(diagonal, E, F) and the clamped gap terms
//     max(E - ge, H - go - ge, 0) and max(F - ge, H - go - ge, 0) are one
//     v_pk_maximum3_f16 each (clamping E and F at zero leaves H unchanged).
// The 4 tag bits are the cell's choices.  Bits 3:2 name the source of H: 3 zero,
// 2 diagonal, 1 gap consuming a read base (F), 0 gap consuming a window base
// (E); on equal values the maximum takes the higher tag, which is the walk's
// order, with H = 0 ahead of all.  Bit 1 says F(i, j) was opened from H(i-1, j)
// and bit 0 that E(i, j) was opened from H(i, j-1) (an opening term carries the
// bit, an extension clears it, so opening wins on equal values).  A cell's
// 4-bit code is then the tag bits of H, F and E gathered with two and-or
// operations.  Codes of a column: 4 rows x 2 halves per 32-bit word, stored
// coalesced as [strip][column][group][lane]; each lane then walks both of its
// slots back through its words.

namespace {

struct PairTask {
  int live, L, h, k, ie, je, sc;
  int64_t r, ws;
};

// The lane's task for traced slot t; untraced and invalid slots are written out
// here (score <= 0: -1 and no operations; invalid: -2) and stay idle.
__device__ __forceinline__ PairTask pair_task(const TraceInterArgs &I, const int64_t *rt_len, int64_t t) {
  const TraceArgs &A = I.a;
  PairTask p{};
  p.ie = p.je = -1;
  p.r = -1;
  if (t >= A.n_slots) return p;
  int status = 0;
  const int64_t slot = A.slots[t];
  if (slot != -1) {
    if (slot < 0 || slot >= 2 * A.n_cals) {
      status = -2;
    } else if ((p.sc = A.score[slot]) > 0) {
      const int64_t c = slot >> 1;
      p.h = (int)(slot & 1);
      p.r = I.cal_read[c];
      const int64_t pos = A.cal_pos[c];
      p.k = A.cal_ref[c];
      p.L = p.r >= 0 && p.r < A.n_reads ? A.read_len[p.r] : 0;
      if (p.r < 0 || p.L < 1 || p.L > A.max_read_len || p.k < 0 || p.k >= A.n_refs || pos < 0 || pos >= rt_len[p.k]) {
        status = -2;
      } else {
        p.ws = pos - A.band < 0 ? 0 : pos - A.band;
        const int64_t we = min(rt_len[p.k], pos + p.L + A.band);
        p.ie = A.read_end[slot];
        const int64_t je64 = A.ref_end[slot] - p.ws;
        if (p.ie < 0 || p.ie >= p.L || je64 < 0 || je64 >= we - p.ws) {
          status = -2;
        } else {
          p.je = (int)je64;
          p.live = 1;
        }
      }
    }
  }
  if (!p.live) {
    A.ref_start[t] = -1;
    A.read_start[t] = -1;
    A.n_ops[t] = status;
    if (status) atomicAdd(A.err, 1ull);
  }
  return p;
}

typedef unsigned short v2u16 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t padd(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(v2u16, a) + __builtin_bit_cast(v2u16, b));
}

}  // namespace

template <int R>
__global__ __launch_bounds__(64) void k_trace_pair(const TraceInterArgs I, const RefTable T) {
  constexpr int G = (R + 3) / 4;  // code words per column per lane (4 rows x 2 halves each)
  extern __shared__ uint32_t tpsm[];
  __shared__ int64_t rt_off[SW_MAX_REFS], rt_len[SW_MAX_REFS];
  const TraceArgs &A = I.a;
  const int lane = threadIdx.x;
  for (int i = 0; i < A.n_refs; ++i)
    if (lane == i) {
      rt_off[i] = T.word_off[i];
      rt_len[i] = T.len[i];
    }
  __syncthreads();
  // LDS: read words of both halves, then window words of both halves, [word][lane]
  uint32_t *rdw0 = tpsm, *rdw1 = tpsm + I.rwords * 64;
  uint32_t *win0 = tpsm + 2 * I.rwords * 64, *win1 = win0 + I.wwords * 64;
  uint32_t *bits = I.bits + (size_t)blockIdx.x * I.bits_stride;
  uint2 *bscr = I.bscr + (size_t)blockIdx.x * I.bscr_stride;
  const int32_t c0 = -A.mismatch, beta = I.beta;
  const uint32_t P1 = 0x00010001u;
  const uint32_t sx = 8u, sm = (uint32_t)(16 * (A.match + c0) + 8);
  const uint32_t kue = (uint32_t)(uint16_t)(16 * (c0 - A.goe) + 1) * P1;  // E opened from H: tag bit 0
  const uint32_t kuf = (uint32_t)(uint16_t)(6 - 16 * A.goe) * P1;         // F opened from H: tags 01 and bit 1
  const uint32_t kee = (uint32_t)(uint16_t)(16 * (c0 - A.ge)) * P1;       // E extended
  const uint32_t kfe = (uint32_t)(uint16_t)(-16 * A.ge) * P1;             // F extended (bit 1 cleared first)
  const uint32_t zc = (uint32_t)(16 * c0) * P1;                           // zero: +16c per column
  const uint32_t z0 = (uint32_t)(16 * beta + 12) * P1;                    // zero of column 0, tag 3
  const uint32_t hleft = (uint32_t)(16 * (beta - c0)) * P1;               // H(i, -1) = 0, clean

  for (int64_t first = (int64_t)blockIdx.x * 128; first < A.n_slots; first += (int64_t)gridDim.x * 128) {
    const PairTask ta = pair_task(I, rt_len, first + lane), tb = pair_task(I, rt_len, first + 64 + lane);
    const int n_rows = max(ta.live ? ta.ie + 1 : 0, tb.live ? tb.ie + 1 : 0);
    const int n_cols = max(ta.live ? ta.je + 1 : 0, tb.live ? tb.je + 1 : 0);
    int rmax = n_rows, cmax = n_cols, lmax = max(ta.live ? ta.L : 0, tb.live ? tb.L : 0);
    for (int m = 32; m; m >>= 1) {
      rmax = max(rmax, __shfl_xor(rmax, m, 64));
      cmax = max(cmax, __shfl_xor(cmax, m, 64));
      lmax = max(lmax, __shfl_xor(lmax, m, 64));
    }
    if (rmax == 0) continue;
    // ---- stage both halves' read and window words
    __syncthreads();
    {
      const int nrw = (lmax + 15) >> 4, nww = (cmax + 15) >> 4;
      for (int hf = 0; hf < 2; ++hf) {
        const PairTask &p = hf ? tb : ta;
        uint32_t *rdw = hf ? rdw1 : rdw0, *win = hf ? win1 : win0;
        if (p.live) {
          const uint32_t *rp = A.reads + A.read_word_off[p.r];
          const int lw = (p.L + 15) >> 4;
          for (int q = 0; q < nrw; ++q) rdw[q * 64 + lane] = q < lw ? rp[q] : 0u;
          const int64_t fw = rt_off[p.k] + (p.ws >> 4);
          const int64_t last = rt_off[p.k] + ((rt_len[p.k] - 1) >> 4);
          const uint32_t sh = 2u * (uint32_t)(p.ws & 15);
          uint32_t lo = A.ref_words[fw];
          for (int q = 0; q < nww; ++q) {
            const uint32_t hi = fw + q + 1 <= last ? A.ref_words[fw + q + 1] : 0u;
            win[q * 64 + lane] = (uint32_t)((((uint64_t)hi << 32) | lo) >> sh);
            lo = hi;
          }
        } else {
          for (int q = 0; q < nrw; ++q) rdw[q * 64 + lane] = 0u;
          for (int q = 0; q < nww; ++q) win[q * 64 + lane] = 0u;
        }
      }
    }
    __syncthreads();
    auto qbase = [&](int hf, int i) -> uint32_t {  // oriented read base of row i (0 past the read)
      const PairTask &p = hf ? tb : ta;
      if (i >= p.L) return 0u;
      const uint32_t *rdw = hf ? rdw1 : rdw0;
      const int src = p.h == 0 ? i : p.L - 1 - i;
      const uint32_t b = (rdw[(src >> 4) * 64 + lane] >> (2 * (src & 15))) & 3u;
      return p.h == 0 ? b : 3u - b;
    };
    auto wbase = [&](int hf, int j) -> uint32_t {
      const uint32_t *win = hf ? win1 : win0;
      return (win[(j >> 4) * 64 + lane] >> (2 * (j & 15))) & 3u;
    };

    // ---- sweep: strips of R rows, columns left to right
    uint32_t endv0 = 0, endv1 = 0;
    const int nstrips = (rmax + R - 1) / R;
    for (int s = 0; s < nstrips; ++s) {
      const int r0 = s * R;
      uint32_t sel[R], Hl[R], E[R];
#pragma unroll
      for (int x = 0; x < R; ++x) {
        sel[x] = qbase(0, r0 + x) | (12u << 8) | ((4u + qbase(1, r0 + x)) << 16) | (12u << 24);
        Hl[x] = hleft;  // H(i, -1) = 0, clean
        E[x] = z0;      // E(i, 0) = zero
      }
      uint32_t hup_prev = hleft;  // H(r0 - 1, -1)
      uint32_t Zj = z0;
      if (s > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      for (int c = 0; c < cmax; ++c) {
        const uint32_t Zn = padd(Zj, zc);
        const uint32_t tlo = sx * 0x01010101u ^ ((sx ^ sm) << (8 * wbase(0, c)));
        const uint32_t thi = sx * 0x01010101u ^ ((sx ^ sm) << (8 * wbase(1, c)));
        uint32_t hup, F;
        if (s == 0) {
          hup = Zj & 0xFFF0FFF0u;  // H(-1, c) = 0, clean
          F = Zj;                  // F(0, c) clamped to zero
        } else {
          const uint2 b = bscr[c * 64 + lane];
          hup = b.x;
          F = b.y;
        }
        // the diagonal operand of row 0 (the row above, one column back)
        uint32_t diag = padd(hup_prev, __builtin_amdgcn_perm(thi, tlo, sel[0]));
        hup_prev = hup;
        uint32_t word[G];
#pragma unroll
        for (int x = 0; x < R; ++x) {
          // the diagonal of row x+1 is row x's previous H: consume it before row x's
          // new H takes its register (else every column ends rotating the H registers)
          uint32_t dn = 0;
          if (x + 1 < R) dn = padd(Hl[x], __builtin_amdgcn_perm(thi, tlo, sel[x + 1]));
          const uint32_t Ht = half_max3(diag, E[x], F);
          diag = dn;
          const uint32_t nib = (Ht & 0x000C000Cu) | (E[x] & 0x00010001u) | (F & 0x00020002u);
          if ((x & 3) == 0)
            word[x >> 2] = nib;
          else
            word[x >> 2] |= nib << (4 * (x & 3));
          const uint32_t Hc = Ht & 0xFFF0FFF0u;
          const uint32_t En = half_max3(padd(E[x] & 0xFFFEFFFEu, kee), padd(Hc, kue), Zn);
          F = half_max3(padd(F & 0xFFFDFFFDu, kfe), padd(Hc, kuf), Zj);
          Hl[x] = Hc;
          E[x] = En;
        }
#pragma unroll
        for (int g = 0; g < G; ++g) bits[(((int64_t)s * cmax + c) * G + g) * 64 + lane] = word[g];
        if (s + 1 < nstrips) bscr[c * 64 + lane] = make_uint2(Hl[R - 1], F);
        if ((c == ta.je && ta.ie >= r0 && ta.ie < r0 + R) || (c == tb.je && tb.ie >= r0 && tb.ie < r0 + R)) {
#pragma unroll
          for (int x = 0; x < R; ++x) {
            if (c == ta.je && ta.ie == r0 + x) endv0 = Hl[x] & 0xFFFFu;
            if (c == tb.je && tb.ie == r0 + x) endv1 = Hl[x] >> 16;
          }
        }
        Zj = Zn;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __syncthreads();
    }

    // ---- walk each half's slot back from its end cell
    auto code_at = [&](int hf, int i, int j) -> uint32_t {
      const int s = i / R, r = i - s * R;
      const uint32_t w = bits[(((int64_t)s * cmax + j) * G + (r >> 2)) * 64 + lane];
      return (w >> (16 * hf + 4 * (r & 3))) & 15u;
    };
    for (int hf = 0; hf < 2; ++hf) {
      const PairTask &p = hf ? tb : ta;
      if (!p.live) continue;
      const int64_t t = first + 64 * hf + lane;
      const int32_t endval = (int32_t)((hf ? endv1 : endv0) >> 4) - beta - p.je * c0;
      if (endval != p.sc) {
        A.ref_start[t] = -1;
        A.read_start[t] = -1;
        A.n_ops[t] = -2;
        atomicAdd(A.err, 1ull);
        continue;
      }
      uint32_t *out = A.cigar + t * (int64_t)A.cap;
      int n = 0;
      uint32_t cur_op = 0, cur_len = 0;
      auto flush = [&]() {
        if (cur_len) {
          if (n < A.cap) out[n] = (cur_len << 4) | cur_op;
          ++n;
        }
      };
      auto emit = [&](uint32_t op) {
        if (op != cur_op) {
          flush();
          cur_op = op;
          cur_len = 0;
        }
        ++cur_len;
      };
      if (p.L - 1 - p.ie > 0) {
        cur_op = 4;
        cur_len = (uint32_t)(p.L - 1 - p.ie);
      }
      // state 0: in H; 1: in a gap consuming read bases (F); 2: consuming window bases (E)
      int i = p.ie, j = p.je, state = 0, start_i = 0, start_j = 0;
      uint32_t code = code_at(hf, i, j);
      for (;;) {
        if (state == 0) {
          const uint32_t src = code >> 2;
          if (src == 2u) {
            emit(qbase(hf, i) == wbase(hf, j) ? 7u : 8u);
            start_i = i;
            start_j = j;
            if (i == 0 || j == 0) break;  // a diagonal from the boundary starts the alignment
            code = code_at(hf, i - 1, j - 1);
            if ((code >> 2) == 3u) break;  // a diagonal from a cell with H = 0 starts it
            --i;
            --j;
          } else if (src == 1u) {
            state = 1;
          } else if (src == 0u) {
            state = 2;
          } else {  // H = 0 on the path: cannot happen for a consistent matrix
            start_i = i + 1;
            start_j = j + 1;
            break;
          }
        } else if (state == 1) {
          emit(1u);
          const bool open = (code >> 1) & 1u;
          if (i == 0) break;  // cannot happen: F(0, j) is at most zero
          --i;
          if (open) state = 0;
          code = code_at(hf, i, j);
        } else {
          emit(2u);
          const bool open = code & 1u;
          if (j == 0) break;  // cannot happen: E(i, 0) is at most zero
          --j;
          if (open) state = 0;
          code = code_at(hf, i, j);
        }
      }
      if (start_i > 0) {
        emit(4u);
        cur_len = (uint32_t)start_i;
      }
      flush();
      if (n > A.cap) {
        for (int x = 0; x < A.cap; ++x) out[x] = 0u;  // an over-capacity row is cleared
        A.ref_start[t] = -1;
        A.read_start[t] = -1;
        A.n_ops[t] = -1;
      } else {
        for (int x = 0; x < n / 2; ++x) {
          const uint32_t a = out[x];
          out[x] = out[n - 1 - x];
          out[n - 1 - x] = a;
        }
        A.ref_start[t] = p.ws + start_j;
        A.read_start[t] = (int16_t)start_i;
        A.n_ops[t] = n;
      }
    }
  }
}

// Strip height of the two-slots-per-lane traceback for a read-length bound: the
// compiled height with the fewest swept rows, counting each strip's column
// overhead (table, boundary row, code stores) as four rows; the taller on ties.
int trace_pair_rows(int max_read_len) {
  int best = 0, best_cost = 0x7fffffff;
#define SW_TP_CHOOSE(RR)                                        \
  {                                                             \
    const int ns = (max_read_len + RR - 1) / RR;                \
    const int cost = ns * RR + 4 * ns;                          \
    if (cost < best_cost || (cost == best_cost && RR > best)) { \
      best_cost = cost;                                         \
      best = RR;                                                \
    }                                                           \
  }
  SW_TRACE_PAIR_ROWS(SW_TP_CHOOSE)
#undef SW_TP_CHOOSE
  return best;
}

size_t trace_pair_block_bytes(int max_read_len, int wcap) {
  const int R = trace_pair_rows(max_read_len);
  const size_t strips = (size_t)(max_read_len + R - 1) / R;
  return strips * (size_t)wcap * (size_t)((R + 3) / 4) * 64 * 4 + (size_t)wcap * 64 * 8;
}

int trace_pair_blocks_per_cu(int max_read_len) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (trace_pair_rows(max_read_len)) {
#define SW_TP_OCC(RR)                                                                                          \
  case RR:                                                                                                     \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_trace_pair<RR>), 64, \
                                                     16384);                                                   \
    break;
    SW_TRACE_PAIR_ROWS(SW_TP_OCC)
#undef SW_TP_OCC
    default:
      break;
  }
  if (e != hipSuccess) return 1;
  return n < 1 ? 1 : n;
}

// The int16-pair layout holds every value of the traced rectangles: scores up to
// match * max_read_len, column offsets up to (wcap - 1) * c, the bias and a tag,
// below 0x7C00 after scaling by 16; and each table byte 16 * (s + c) + 8 fits.
int trace_pair_fits(int match, int mismatch, int goe, int ge, int max_read_len, int wcap, int32_t *beta) {
  const int c = -mismatch;
  int b = c;
  if (goe > b) b = goe;
  if (ge > b) b = ge;
  if (16 * (match + c) + 8 > 255) return 0;
  const int64_t top = (int64_t)match * max_read_len + b + (int64_t)(wcap - 1) * c + 1;
  if (top * 16 > 0x7BFF) return 0;
  *beta = b;
  return 1;
}

hipError_t launch_trace_pair(const TraceInterArgs &A, const RefTable &T, int grid, hipStream_t st) {
  if (A.a.n_slots == 0) return hipSuccess;
  const size_t lds = (size_t)(A.rwords + A.wwords) * 2 * 64 * sizeof(uint32_t);
  switch (trace_pair_rows(A.a.max_read_len)) {
#define SW_TP_LAUNCH(RR)                                                                           \
  case RR:                                                                                         \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace_pair<RR>), dim3(grid), dim3(64), lds, st, A, T); \
    break;
    SW_TRACE_PAIR_ROWS(SW_TP_LAUNCH)
#undef SW_TP_LAUNCH
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t trace_inter_block_bytes(int max_read_len, int wcap) {
  const size_t strips = (size_t)(max_read_len + kTraceRows - 1) / kTraceRows;
  return strips * (size_t)wcap * kTraceGroups * 64 * 4 + (size_t)wcap * 64 * 8;
}

int trace_inter_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_trace_inter<true>), 64, 8192) !=
      hipSuccess)
    return 1;
  return n < 1 ? 1 : n;
}

hipError_t launch_trace_inter(const TraceInterArgs &A, const RefTable &T, int grid, hipStream_t st) {
  if (A.a.n_slots == 0) return hipSuccess;
  const size_t lds = (size_t)(A.rwords + A.wwords) * 64 * sizeof(uint32_t);
  if (A.a.match <= 127 && A.a.mismatch >= -128)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace_inter<true>), dim3(grid), dim3(64), lds, st, A, T);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace_inter<false>), dim3(grid), dim3(64), lds, st, A, T);
  return hipGetLastError();
}

}  // namespace swk
