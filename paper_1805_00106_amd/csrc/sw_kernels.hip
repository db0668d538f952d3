// HIP kernels for gfx950: 2-bit packing, task expansion, the inter-task Gotoh
// kernels (one CAL per lane), the per-read Score Tracker reduction and the
// two-reference classification.
//
// The recurrence is Gotoh's affine-gap local alignment (section 3.5 of the
// paper defers it to an external reference):
//   E(i,j) = max(E(i,j-1) - ge, H(i,j-1) - go - ge)
//   F(i,j) = max(F(i-1,j) - ge, H(i-1,j) - go - ge)
//   H(i,j) = max(0, H(i-1,j-1) + s(q_i, w_j), E(i,j), F(i,j))
// Rows i are read bases, columns j window bases (section 3.5: the read on the
// vertical axis, the reference on the horizontal one).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sw_device.h"
#include "sw_halfmax.h"
#include "sw_lanes.h"
#include "sw_launch.h"

namespace swk {

typedef short v2s __attribute__((ext_vector_type(2)));
typedef unsigned short v2u __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t bits(v2s a) { return __builtin_bit_cast(uint32_t, a); }
__device__ __forceinline__ v2s pair(uint32_t a) { return __builtin_bit_cast(v2s, a); }
__device__ __forceinline__ v2s vmax(v2s a, v2s b) { return __builtin_elementwise_max(a, b); }

__device__ __forceinline__ v2s vmax3h(v2s a, v2s b, v2s c) {
  return __builtin_bit_cast(v2s, half_max3(bits(a), bits(b), bits(c)));
}

// Wave-wide maximum and minimum; every lane holds the result, which is read
// from lane 0 so that the compiler keeps it in a scalar register.
__device__ __forceinline__ int wave_max(int v) {
  for (int m = 32; m; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int wave_min(int v) {
  for (int m = 32; m; m >>= 1) v = min(v, __shfl_xor(v, m, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

// --------------------------------------------------------------------------- packing

// One thread per output word: 16 codes -> 2 bits each, least significant first.
__global__ void k_pack_2bit(const uint8_t *__restrict__ codes, int64_t n, uint32_t *__restrict__ words,
                            int64_t n_words) {
  int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n_words) return;
  int64_t base = w * 16;
  uint32_t acc = 0;
  if (base + 16 <= n && (((uintptr_t)(codes + base)) & 15) == 0) {
    uint4 v = *reinterpret_cast<const uint4 *>(codes + base);
    uint32_t part[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc |= ((part[q] >> (8 * b)) & 3u) << (2 * (4 * q + b));
  } else {
    for (int k = 0; k < 16 && base + k < n; ++k) acc |= (uint32_t)(codes[base + k] & 3u) << (2 * k);
  }
  words[w] = acc;
}

// --------------------------------------------------------------------------- expansion

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Owner read of each CAL from the CSR row pointer (one thread per read).  CALs
// outside every read's range keep -1 and are reported as invalid tasks.
__global__ void k_cal_owner(const int64_t *__restrict__ cal_ptr, int32_t n_reads, int64_t n_cals,
                            int32_t *__restrict__ cal_read) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  int64_t a = cal_ptr[r], b = cal_ptr[r + 1];
  if (a < 0) a = 0;
  if (b > n_cals) b = n_cals;
  for (int64_t c = a; c < b; ++c) cal_read[c] = (int32_t)r;
}

// --------------------------------------------------------------------------- common lane setup

struct LaneTask {
  int64_t c;    // CAL index
  int64_t ws;   // window start (absolute, forward)
  int32_t L;    // read length (0: lane idle)
  int32_t W;    // window width
  int32_t mask; // strand mask handled by this lane
  int32_t k;    // reference id
  int32_t r;    // read id
};

__device__ __forceinline__ void write_slot(const AlignArgs &A, int64_t slot, int32_t s, int64_t re,
                                           int16_t qe) {
  A.score[slot] = s;
  A.ref_end[slot] = re;
  A.read_end[slot] = qe;
}

// Loads the task of one lane.  `strand_sel` restricts the strands handled by
// the lane (3 for a lane holding both strands).  Invalid tasks are written out
// here and leave the lane idle.
__device__ __forceinline__ LaneTask load_task(const AlignArgs &A, const int64_t *rt_len, int64_t c,
                                              int strand_sel) {
  LaneTask t;
  t.c = c;
  t.ws = 0;
  t.L = 0;
  t.W = 0;
  t.k = 0;
  t.r = 0;
  int mask = A.strand[c] & strand_sel;
  t.mask = mask;
  int32_t r = A.cal_read[c];
  int32_t k = A.cal_ref[c];
  int64_t p = A.cal_pos[c];
  bool ok = r >= 0 && r < A.n_reads && k >= 0 && k < A.n_refs;
  int32_t L = 0;
  if (ok) {
    L = A.read_len[r];
    ok = L >= 1 && L <= A.max_read_len && p >= 0 && p < rt_len[k];
  }
  if (!ok) {
    for (int h = 0; h < 2; ++h) {
      if ((mask >> h) & 1) write_slot(A, 2 * c + h, INT32_MIN, -1, -1);
      else if ((strand_sel >> h) & 1) write_slot(A, 2 * c + h, -1, -1, -1);
    }
    if (mask) atomicAdd(A.err, (unsigned long long)__builtin_popcount(mask));
    t.mask = 0;
    return t;
  }
  for (int h = 0; h < 2; ++h)
    if (((strand_sel >> h) & 1) && !((mask >> h) & 1)) write_slot(A, 2 * c + h, -1, -1, -1);
  if (!mask) return t;
  int64_t ws = p - A.band;
  if (ws < 0) ws = 0;
  int64_t we = p + L + A.band;
  if (we > rt_len[k]) we = rt_len[k];
  t.ws = ws;
  t.W = (int32_t)(we - ws);
  t.L = L;
  t.k = k;
  t.r = r;
  return t;
}

// Stage the lane's read words and its window words (re-aligned so that window
// column 0 sits at bit 0 of word 0) into LDS, [word][lane] layout.
__device__ __forceinline__ void stage(const AlignArgs &A, const int64_t *rt_off, const int64_t *rt_len,
                                      const LaneTask &t, int rwmax, int wwmax, uint32_t *rdw,
                                      uint32_t *win, int lane) {
  if (t.L > 0) {
    const uint32_t *rp = A.reads + A.read_word_off[t.r];
    int nrw = (t.L + 15) >> 4;
    for (int q = 0; q < rwmax; ++q) rdw[q * 64 + lane] = q < nrw ? rp[q] : 0u;
    int64_t first = rt_off[t.k] + (t.ws >> 4);
    int64_t last = rt_off[t.k] + ((rt_len[t.k] - 1) >> 4);
    uint32_t sh = 2u * (uint32_t)(t.ws & 15);
    uint32_t lo = A.ref_words[first];
    for (int q = 0; q < wwmax; ++q) {
      uint32_t hi = (first + q + 1 <= last) ? A.ref_words[first + q + 1] : 0u;
      win[q * 64 + lane] = (uint32_t)((((uint64_t)hi << 32) | lo) >> sh);
      lo = hi;
    }
  } else {
    for (int q = 0; q < rwmax; ++q) rdw[q * 64 + lane] = 0u;
    for (int q = 0; q < wwmax; ++q) win[q * 64 + lane] = 0u;
  }
}

__device__ __forceinline__ uint32_t base_at(const uint32_t *rdw, int lane, int i) {
  return (rdw[(i >> 4) * 64 + lane] >> (2 * (i & 15))) & 3u;
}

// Lexicographic best-cell key: score, then smallest column, then smallest row.
__device__ __forceinline__ uint64_t cell_key(int32_t v, int32_t col, int32_t row) {
  return ((uint64_t)(uint32_t)v << 32) | ((uint64_t)(0xFFFFu - (uint32_t)col) << 16) |
         (uint64_t)(0xFFFFu - (uint32_t)row);
}

__device__ __forceinline__ void write_result(const AlignArgs &A, int64_t slot, uint64_t key, int64_t ws) {
  int32_t v = (int32_t)(key >> 32);
  if (v > 0) {
    int32_t col = 0xFFFF - (int32_t)((key >> 16) & 0xFFFF);
    int32_t row = 0xFFFF - (int32_t)(key & 0xFFFF);
    write_slot(A, slot, v, ws + col, (int16_t)row);
  } else {
    write_slot(A, slot, 0, -1, -1);
  }
}

// Tile of task positions for this iteration (plain: fixed 64-wide tiles with
// static striding; batched: descriptors popped from a device work queue).
struct TileIter {
  int64_t next;
  int64_t n_tiles;
};

__device__ __forceinline__ bool next_tile(const AlignArgs &A, TileIter &it, int64_t &first, int &count,
                                          int64_t &t) {
  if (A.queue) {
    int v = 0;
    if (threadIdx.x == 0) v = atomicAdd(A.queue, 1);
    t = __shfl(v, 0, 64);
  } else {
    t = it.next;
    it.next += gridDim.x;
  }
  if (t >= it.n_tiles) return false;
  if (A.tiles) {
    first = A.tiles[t];
    count = A.tile_len[t];
  } else {
    first = t * 64;
    int64_t rem = A.n_tasks - first;
    count = rem < 64 ? (int)rem : 64;
  }
  return true;
}

__device__ __forceinline__ void load_ref_table(const RefTable &T, int n_refs, int64_t *rt_off,
                                               int64_t *rt_len, int lane) {
  for (int i = 0; i < n_refs; ++i) {
    int64_t o = T.word_off[i], l = T.len[i];
    if (lane == i) {
      rt_off[i] = o;
      rt_len[i] = l;
    }
  }
  __syncthreads();
}

// --------------------------------------------------------------------------- int16-pair kernel
//
// One lane holds one CAL; the low int16 half of every register is the forward
// strand task and the high half the reverse strand task (reverse complement of
// the read against the same window), so both halves always share the window.
// A lane keeps a strip of R read rows in registers and sweeps the window
// columns; between strips the strip's bottom row (H and the F entering the next
// row) goes through a per-wave scratch buffer.
//
// Substitution: for column j the lane builds an 8-byte table (lo bytes and hi
// bytes of s~(b, w_j) for b = 0..3) and each row holds a byte selector
// (q, q|4) per half, so v_perm_b32 yields both halves' scores in one
// instruction.  Rows past the read end use selector bytes 12/13 (0x00, 0xFF):
// every substitution is -256, so those rows only decrease and are never
// reported.  Columns past the lane's window use a table of 0x8000 (a wall: the
// diagonal operand becomes a negative half and never wins).
//
// Values are biased (N = (V + beta) * 2^K + tag, see DpConst), so the running
// maxima start at 0 (below every cell) and V = (N >> K) - beta.

// Fold the per-row maxima of one tile of 2^K columns (tile base tb) into the
// lexicographic best keys of both halves.  The packed maximum over the rows
// gives, per half, the best value and (through its tag) the smallest column;
// the smallest row holding exactly that value is then found with a packed
// equality scan.  Rows past the read end need no check: every value there
// derives from the rows above minus a positive penalty (their substitutions
// are -256), so it stays strictly below the best real cell and never wins.
template <int R>
__device__ __forceinline__ void fold16(const DpConst &K, const v2s (&M)[R], int r0, int tb, volatile uint64_t *best) {
  v2s mx = M[0];
#pragma unroll
  for (int r = 1; r < R; ++r) mx = vmax(mx, M[r]);
  const uint32_t mxb = bits(mx);
  const int kb = K.kbits16, tmask = (1 << kb) - 1;
  const int32_t vf = ((int32_t)(mxb & 0xFFFFu) >> kb) - K.beta16, vr = ((int32_t)(mxb >> 16) >> kb) - K.beta16;
  if (vf <= 0 && vr <= 0) return;
  uint32_t rows = 0xFFFFFFFFu;
  const v2u ONE = __builtin_bit_cast(v2u, 0x00010001u);
#pragma unroll
  for (int r = R - 1; r >= 0; --r) {
    // eq: 0xFFFF in the halves where M[r] equals the maximum
    const v2u d = __builtin_elementwise_min(__builtin_bit_cast(v2u, bits(M[r]) ^ mxb), ONE);
    const uint32_t eq = __builtin_bit_cast(uint32_t, (v2u)(d - ONE));
    rows = (rows & ~eq) | ((uint32_t)r * 0x00010001u & eq);
  }
  if (vf > 0) {
    const uint64_t kf = cell_key(vf, tb + tmask - (int32_t)(mxb & tmask), r0 + (int32_t)(rows & 0xFFFFu));
    if (kf > best[0]) best[0] = kf;
  }
  if (vr > 0) {
    const uint64_t kr = cell_key(vr, tb + tmask - (int32_t)((mxb >> 16) & tmask), r0 + (int32_t)(rows >> 16));
    if (kr > best[64]) best[64] = kr;
  }
}

// Final-row mode: fold the maximum of one row (both halves on row `row`).
__device__ __forceinline__ void fold16_row(const DpConst &K, v2s m, int row, int tb, volatile uint64_t *best) {
  const uint32_t mb = bits(m);
  const int kb = K.kbits16, tmask = (1 << kb) - 1;
  const int32_t vf = ((int32_t)(mb & 0xFFFFu) >> kb) - K.beta16, vr = ((int32_t)(mb >> 16) >> kb) - K.beta16;
  if (vf > 0) {
    const uint64_t kf = cell_key(vf, tb + tmask - (int32_t)(mb & tmask), row);
    if (kf > best[0]) best[0] = kf;
  }
  if (vr > 0) {
    const uint64_t kr = cell_key(vr, tb + tmask - (int32_t)((mb >> 16) & tmask), row);
    if (kr > best[64]) best[64] = kr;
  }
}

// A wave-uniform value the compiler may not see through: a running sum taken
// through it is formed row by row (one scalar add each) instead of being
// rewritten as row * step and hoisted into one scalar register per row.
__device__ __forceinline__ uint32_t opaque_s(uint32_t x) {
  asm volatile("" : "+s"(x));
  return x;
}

// One strip of R read rows swept over every window column.  FIRST: the strip
// starts at read row 0 (top boundary H = 0); LAST: no strip follows (nothing
// is written to the scratch rows).  FR: final-row mode (only row L-1 may hold
// the best cell); a template parameter so that the local mode keeps its
// register budget.  TRACK: keep the per-row maxima; a final-row strip that holds
// no lane's last row skips them (one packed op per row of ten).
template <int R, bool FIRST, bool LAST, bool FR, bool TRACK = true>
__device__ __forceinline__ void strip16(const DpConst &K, const uint32_t *win, const uint32_t *rdw, uint2 *scr,
                                        int lane, int r0, int L, int W, int Wmin, int Wmax,
                                        volatile uint64_t *best) {
  static_assert(R <= kInt16StripRowsMax, "the int16 layout holds row offsets of at most kInt16StripRowsMax rows");
  const v2s GOE_E = pair(K.goe_e16), GE_E = pair(K.ge_e16);
  // Row r of the strip carries + r * GF (GF = gap_extend * 2^K): F then moves down
  // a row with no gap-extend step, F = max(F, H - gap_open).  The rows above and
  // below the strip are handed over at offset 0 (H as H - GF, for the diagonal
  // step's + GF).
  const uint32_t GFu = K.ge_f16;
  const v2s GOE_F = pair(K.goe_f16), GO_F = pair(K.goe_f16 - GFu), GF = pair(GFu);
  const v2s RGF = pair((uint32_t)R * GFu);
  const v2s TAGU = pair(K.tag16), BIAS = pair(K.bias16);
  const int U = 1 << K.kbits16;
  uint32_t sel[R];
  v2s Hl[R], E[R], M[R];
  // column -1 (H = 0, tag 2^K) on row r, formed row by row in this strip (hoisted,
  // the 2R starting values would stay live across the whole kernel)
  uint32_t h0 = K.tag16 + K.bias16;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = r0 + r;
    if (i < L) {
      const uint32_t qf = base_at(rdw, lane, i);
      const uint32_t qr = 3u - base_at(rdw, lane, L - 1 - i);
      sel[r] = qf | ((qf | 4u) << 8) | (qr << 16) | ((qr | 4u) << 24);
    } else {
      sel[r] = 0x0D0C0D0Cu;
    }
    Hl[r] = pair(h0);
    // E is kept clamped at zero (see below): column 0 starts at its zero
    E[r] = pair(h0 - 0x00010001u);
    M[r] = pair(0u);
    h0 = opaque_s(h0 + GFu);
  }
  v2s hup_prev = TAGU + BIAS - GF;
  // the hand-over row of the next column, loaded one column ahead
  uint2 pf = make_uint2(0, 0);
  if (!FIRST) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    pf = scr[lane];
  }
  for (int tb = 0; tb < Wmax; tb += U) {
    const int tend = min(tb + U, Wmax);
    uint32_t wd = 0;
    for (int c = tb; c < tend; ++c) {
      const int cc = c - tb;
      // the zero of column c: V = 0 with the column's tag
      const uint32_t zt = (uint32_t)(U - 1 - cc) * 0x00010001u + K.bias16;
      if ((c & 15) == 0) wd = win[(c >> 4) * 64 + lane];
      const uint32_t sh8 = ((wd >> (2 * (c & 15))) & 3u) << 3;
      uint32_t tlo = K.xlo ^ (K.dlo << sh8);
      uint32_t thi = K.xhi ^ (K.dhi << sh8);
      if (c >= Wmin) {
        if (c >= W) {
          tlo = 0u;
          thi = 0x80808080u;
        }
      }
      v2s hup, F;
      if (FIRST) {
        hup = pair(zt) - GF;
        F = pair(zt) - GOE_F;
      } else {
        hup = pair(pf.x);
        F = pair(pf.y);
        if (c + 1 < Wmax) pf = (scr + (size_t)(c + 1) * 64)[lane];
      }
      // the zero of the next column (the tag one lower), where E is clamped
      const uint32_t ztn = zt - 0x00010001u;
      // E is carried as max(E, 0): then H = max(diagonal, E, F) needs no zero
      // operand, and the clamped E obeys the same recurrence clamped at zero
      // (max(max(E, 0) - ge, H - go - ge, 0) = max(E - ge, H - go - ge, 0)).
      // Per row: H in one three-way maximum, E in three ops (its zero, with the
      // row's offset, is wave-uniform), F in two, the diagonal operand of the
      // next row in two, the running maximum in one.
      v2s t = hup_prev + pair(__builtin_amdgcn_perm(thi, tlo, sel[0]));
      hup_prev = hup;
      uint32_t zr = ztn;  // the zero of the next column on row r
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // the diagonal of row r+1 is row r's previous H: consume it before row r's
        // new H takes its register
        v2s tn;
        if (r + 1 < R) tn = Hl[r] + pair(__builtin_amdgcn_perm(thi, tlo, sel[r + 1]));
        const v2s H = vmax3h(t, E[r], F);
        if (r + 1 < R) t = tn;
        const v2s e2 = E[r] - GE_E;
        const v2s v = H - GO_F;
        const v2s u = H - GOE_E;
        F = vmax(F, v);
        E[r] = vmax3h(e2, u, pair(zr));
        zr = opaque_s(zr + GFu);
        if (!FR || TRACK) M[r] = vmax(M[r], H);
        Hl[r] = H;
      }
      // the column's scratch row: a wave-uniform base plus the lane
      if (!LAST) (scr + (size_t)c * 64)[lane] = make_uint2(bits(Hl[R - 1] - RGF), bits(F - RGF));
    }
    if (FR && TRACK) {
      // read-end-anchored scoring: only row L-1 may hold the best cell
      const int rr = L - 1 - r0;
      v2s m = pair(0u);
#pragma unroll
      for (int r = 0; r < R; ++r) m = r == rr ? M[r] : m;
      if (rr > 0 && rr < R) m = m - pair((uint32_t)rr * GFu);  // the row's offset
      fold16_row(K, m, L - 1, tb, best);
    } else if (!FR) {
      // the rows' offsets off, so that maxima compare across rows
      uint32_t off = 0;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        off = opaque_s(off + GFu);
        M[r] = M[r] - pair(off);
      }
      fold16<R>(K, M, r0, tb, best);
    }
    if (tend < Wmax) {
      // next tile: restart the row maxima and re-base the carried tags by +2^K
#pragma unroll
      for (int r = 0; r < R; ++r) {
        M[r] = pair(0u);
        Hl[r] = Hl[r] + TAGU;
        E[r] = E[r] + TAGU;
      }
      hup_prev = hup_prev + TAGU;
    }
  }
  if (!LAST) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

// One strip of a tile: in final-row mode the row maxima are kept only if some
// lane's last read row lies in the strip (a wave-uniform choice).
template <int R, bool FIRST, bool LAST, bool FR>
__device__ __forceinline__ void strip16_sel(const DpConst &K, const uint32_t *win, const uint32_t *rdw, uint2 *scr,
                                            int lane, int r0, int L, int W, int Wmin, int Wmax,
                                            volatile uint64_t *best) {
  if (FR && __ballot(L > 0 && L - 1 >= r0 && L - 1 < r0 + R) == 0ull) {
    strip16<R, FIRST, LAST, FR, false>(K, win, rdw, scr, lane, r0, L, W, Wmin, Wmax, best);
    return;
  }
  strip16<R, FIRST, LAST, FR, true>(K, win, rdw, scr, lane, r0, L, W, Wmin, Wmax, best);
}

// One tile of up to 64 CALs (task positions [first, first + count)).
template <int R, bool FR>
__device__ __forceinline__ void tile16(const AlignArgs &A, const int64_t *rt_off, const int64_t *rt_len,
                                       uint32_t *win, uint32_t *rdw, uint2 *scr, uint64_t *lrec, int lane,
                                       int64_t first, int count) {
  LaneTask t{};
  if (lane < count) {
    const int64_t pos = first + lane;
    const int64_t c = A.order ? (int64_t)A.order[pos] : pos;
    t = load_task(A, rt_len, c, 3);
  }
  const int L = t.L, W = t.W;
  const int Lmax = wave_max(L);
  if (Lmax == 0) return;
  const int Wmax = wave_max(W);
  const int Wmin = wave_min(L > 0 ? W : 0x7fffffff);
  stage(A, rt_off, rt_len, t, (Lmax + 15) >> 4, (Wmax + 15) >> 4, rdw, win, lane);

  // the tile's longest read may allow a wider tag than the call's bound
  DpConst K = A.k;
  if (K.kbits16 < 6) set_int16_layout(K, (int64_t)K.match * Lmax);
  // The lane's record stays in LDS during the sweep, which needs every register
  // it can get: best keys (forward at [0], reverse at [64]), the CAL index at
  // [128] and the window start with the strand mask at [192].
  volatile uint64_t *best = lrec + lane;
  best[0] = 0;
  best[64] = 0;
  best[128] = (uint64_t)t.c;
  best[192] = ((uint64_t)t.ws << 2) | (uint64_t)(t.mask & 3);
  const int nstrips = (Lmax + R - 1) / R;
  if (nstrips == 1) {
    strip16_sel<R, true, true, FR>(K, win, rdw, scr, lane, 0, L, W, Wmin, Wmax, best);
  } else {
    strip16_sel<R, true, false, FR>(K, win, rdw, scr, lane, 0, L, W, Wmin, Wmax, best);
    for (int s = 1; s + 1 < nstrips; ++s)
      strip16_sel<R, false, false, FR>(K, win, rdw, scr, lane, s * R, L, W, Wmin, Wmax, best);
    strip16_sel<R, false, true, FR>(K, win, rdw, scr, lane, (nstrips - 1) * R, L, W, Wmin, Wmax, best);
  }
  if (L > 0) {
    const int64_t c = (int64_t)best[128];
    const uint64_t wm = best[192];
    const int64_t ws = (int64_t)(wm >> 2);
    if (wm & 1) write_result(A, 2 * c, best[0], ws);
    if (wm & 2) write_result(A, 2 * c + 1, best[64], ws);
  }
}

// Plain launch: fixed 64-CAL tiles, static striding over a persistent grid.
template <int R, bool FR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_inter16(const AlignArgs A, const RefTable T) {
  extern __shared__ uint32_t smem[];
  __shared__ int64_t rt_off[SW_MAX_REFS], rt_len[SW_MAX_REFS];
  __shared__ uint64_t lrec[256];
  const int lane = threadIdx.x;
  load_ref_table(T, A.n_refs, rt_off, rt_len, lane);
  uint32_t *win = smem;
  uint32_t *rdw = smem + A.wwords * 64;
  uint2 *scr = A.scratch + (size_t)blockIdx.x * (size_t)A.wcap * 64;
  TileIter it{(int64_t)blockIdx.x, (A.n_tasks + 63) / 64};
  int64_t first, ti;
  int count;
  while (next_tile(A, it, first, count, ti))
    tile16<R, FR>(A, rt_off, rt_len, win, rdw, scr, lrec, lane, first, count);
}

// Batched launch: tiles (each with its own strip height) popped from a device
// work queue, longest reads first.
template <bool FR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_inter16_queue(const AlignArgs A, const RefTable T) {
  extern __shared__ uint32_t smem[];
  __shared__ int64_t rt_off[SW_MAX_REFS], rt_len[SW_MAX_REFS];
  __shared__ uint64_t lrec[256];
  const int lane = threadIdx.x;
  load_ref_table(T, A.n_refs, rt_off, rt_len, lane);
  uint32_t *win = smem;
  uint32_t *rdw = smem + A.wwords * 64;
  uint2 *scr = A.scratch + (size_t)blockIdx.x * (size_t)A.wcap * 64;
  TileIter it{(int64_t)blockIdx.x, (int64_t)*A.n_tiles_dev};
  int64_t first, ti;
  int count;
  while (next_tile(A, it, first, count, ti)) {
    switch (A.tile_strips[ti]) {
#define SW_Q16_CASE(RR)                                                     \
  case RR:                                                                  \
    tile16<RR, FR>(A, rt_off, rt_len, win, rdw, scr, lrec, lane, first, count); \
    break;
      SW_QUEUE16_STRIPS(SW_Q16_CASE)
#undef SW_Q16_CASE
      default:
        break;
    }
  }
}

// --------------------------------------------------------------------------- int32 kernel
//
// Same sweep with one task (one strand of one CAL) per lane and 32-bit values
// tagged with K = 12 bits (tiles of 4096 columns, wider than any window the
// library accepts, so no tile change happens inside a sweep).

// P: substitution by byte permutation (DpConst::perm32), else compare and select.
template <int R, bool P>
__device__ __forceinline__ void tile32(const AlignArgs &A, const int64_t *rt_off, const int64_t *rt_len,
                                       uint32_t *win, uint32_t *rdw, uint2 *scr, int lane, int64_t first,
                                       int count) {
  const DpConst &K = A.k;
  LaneTask t{};
  int h = 0;
  if (lane < count) {
    const int64_t pos = first + lane;
    const int64_t tk = A.order ? (int64_t)A.order[pos] : pos;
    h = (int)(tk & 1);
    t = load_task(A, rt_len, tk >> 1, 1 << h);
  }
  const int L = t.L, W = t.W;
  const int Lmax = wave_max(L);
  if (Lmax == 0) return;
  const int Wmax = wave_max(W);
  stage(A, rt_off, rt_len, t, (Lmax + 15) >> 4, (Wmax + 15) >> 4, rdw, win, lane);

  uint64_t best = 0;
  // Row r of a strip carries + r * GF, as in strip16: F moves down a row with no
  // gap-extend step, a diagonal move carries + GF in its substitution (in the
  // byte tables with P), and the rows above and below a strip are handed over at
  // offset 0 (H as H - GF).
  const int32_t GF = K.ge_f32, GO_F = K.goe_f32 - K.ge_f32;
  const int32_t SMR = K.sm32 + GF, SXR = K.sx32 + GF;
  const int nstrips = (Lmax + R - 1) / R;
  for (int s = 0; s < nstrips; ++s) {
    const int r0 = s * R;
    // per row the read code (compare and select), or with P the byte selector
    // (0xFF, table byte q, sign byte q, sign byte q); past the read end a code
    // that never equals a window code, or the selector of 0xFFFF00FF (about -16 per row)
    int32_t q[R], Hl[R], E[R], M[R];
    // column -1 (H = 0, tag 4096) on row r, formed row by row (see strip16)
    uint32_t h0 = 4096;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = r0 + r;
      if (i < L) {
        q[r] = h == 0 ? (int32_t)base_at(rdw, lane, i) : (int32_t)(3u - base_at(rdw, lane, L - 1 - i));
        if (P) q[r] = 0x0D | (q[r] << 8) | ((q[r] | 4) << 16) | ((q[r] | 4) << 24);
      } else {
        q[r] = P ? 0x0D0D0C0D : 4;
      }
      Hl[r] = (int32_t)h0;
      E[r] = (int32_t)h0 - 1;  // E is kept clamped at zero: column 0 starts at its zero
      M[r] = 0;
      h0 = opaque_s(h0 + (uint32_t)GF);
    }
    int32_t hup_prev = 4096 - GF;
    uint2 pf0 = make_uint2(0, 0), pf1 = make_uint2(0, 0);
    if (s > 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      pf0 = scr[lane];
      if (Wmax > 1) pf1 = scr[64 + lane];
    }
    uint32_t wd = 0;
    for (int c = 0; c < Wmax; ++c) {
      const int32_t zt = 4095 - c;
      if ((c & 15) == 0) wd = win[(c >> 4) * 64 + lane];
      int32_t w = (int32_t)((wd >> (2 * (c & 15))) & 3u);
      // past the lane's window: a wall (no diagonal move enters these columns, so
      // no cell there can beat a real cell of its row, which the final-row mode needs)
      int32_t sx = SXR;
      uint32_t tlo = 0, thi = 0;
      if (P) {
        const uint32_t sh8 = (uint32_t)w << 3;
        tlo = K.xlo32 ^ (K.dlo32 << sh8);
        thi = K.xhi32 ^ (K.dhi32 << sh8);
        if (c >= W) {
          tlo = 0u;           // 0x808000FF: about -2^31
          thi = 0x80808080u;
        }
      } else if (c >= W) {
        w = 5;
        sx = -(1 << 30);
      }
      int32_t hup, F;
      if (s == 0) {
        hup = zt - GF;
        F = zt - K.goe_f32;
      } else {
        const uint2 cur = pf0;
        pf0 = pf1;
        if (c + 2 < Wmax) pf1 = scr[(c + 2) * 64 + lane];
        hup = (int32_t)cur.x;
        F = (int32_t)cur.y;
      }
      // E is carried as max(E, 0), so H = max(diagonal, E, F) is one v_max3_i32
      // and the clamp moves into E's own three-way maximum (with the next
      // column's zero, tag one lower)
      auto subst = [&](int32_t qr) {
        return P ? (int32_t)__builtin_amdgcn_perm(thi, tlo, (uint32_t)qr) : (qr == w ? SMR : sx);
      };
      int32_t t = hup_prev + subst(q[0]);
      hup_prev = hup;
      uint32_t zr = (uint32_t)(zt - 1);  // the zero of the next column on row r
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // the diagonal of row r+1 is row r's previous H: consume it before row r's
        // new H takes its register
        int32_t tn = 0;
        if (r + 1 < R) tn = Hl[r] + subst(q[r + 1]);
        const int32_t H = max(max(t, E[r]), F);
        t = tn;
        M[r] = max(M[r], H);
        E[r] = max(max(E[r] - K.ge_e32, H - K.goe_e32), (int32_t)zr);
        zr = opaque_s(zr + (uint32_t)GF);
        F = max(F, H - GO_F);
        Hl[r] = H;
      }
      if (s + 1 < nstrips)
        scr[c * 64 + lane] = make_uint2((uint32_t)(Hl[R - 1] - R * GF), (uint32_t)(F - R * GF));
    }
    uint32_t off = 0;  // row r's offset
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = r0 + r;
      const int32_t m = M[r] - (int32_t)off;
      off = opaque_s(off + (uint32_t)GF);
      int32_t v = m >> 12;
      if (i < L && v > 0 && (!K.final_row || i == L - 1)) {
        uint64_t kk = cell_key(v, 4095 - (m & 4095), i);
        best = kk > best ? kk : best;
      }
    }
    if (s + 1 < nstrips) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  }
  if (L > 0) write_result(A, 2 * t.c + h, best, t.ws);
}

template <int R, bool P>
__global__ __launch_bounds__(64) void k_inter32(const AlignArgs A, const RefTable T) {
  extern __shared__ uint32_t smem[];
  __shared__ int64_t rt_off[SW_MAX_REFS], rt_len[SW_MAX_REFS];
  const int lane = threadIdx.x;
  load_ref_table(T, A.n_refs, rt_off, rt_len, lane);
  uint32_t *win = smem;
  uint32_t *rdw = smem + A.wwords * 64;
  uint2 *scr = A.scratch + (size_t)blockIdx.x * (size_t)A.wcap * 64;
  TileIter it{(int64_t)blockIdx.x, (A.n_tasks + 63) / 64};
  int64_t first, ti;
  int count;
  while (next_tile(A, it, first, count, ti)) tile32<R, P>(A, rt_off, rt_len, win, rdw, scr, lane, first, count);
}

template <bool P>
__global__ __launch_bounds__(64) void k_inter32_queue(const AlignArgs A, const RefTable T) {
  extern __shared__ uint32_t smem[];
  __shared__ int64_t rt_off[SW_MAX_REFS], rt_len[SW_MAX_REFS];
  const int lane = threadIdx.x;
  load_ref_table(T, A.n_refs, rt_off, rt_len, lane);
  uint32_t *win = smem;
  uint32_t *rdw = smem + A.wwords * 64;
  uint2 *scr = A.scratch + (size_t)blockIdx.x * (size_t)A.wcap * 64;
  TileIter it{(int64_t)blockIdx.x, (int64_t)*A.n_tiles_dev};
  int64_t first, ti;
  int count;
  while (next_tile(A, it, first, count, ti)) {
    switch (A.tile_strips[ti]) {
#define SW_Q32_CASE(RR)                                                  \
  case RR:                                                               \
    tile32<RR, P>(A, rt_off, rt_len, win, rdw, scr, lane, first, count); \
    break;
      SW_QUEUE32_STRIPS(SW_Q32_CASE)
#undef SW_Q32_CASE
      default:
        break;
    }
  }
}

// --------------------------------------------------------------------------- intra-task kernel
//
// One wavefront per task (one strand of one CAL).  Lane j holds window column
// 64*s + j of strip s; the strip is swept along anti-diagonals: at step t lane
// j computes row i = t - j.  Every dependency on column j-1 is a one-lane
// shift of a value computed one step earlier (wave_shr:1 DPP): E(i, j) is
// computed by lane j-1 for lane j, the diagonal H(i-1, j-1) is lane j-1's H
// from two steps earlier, and the read base of row i travels with the
// anti-diagonal.  Lane 0 receives its left boundary through the `old` operand
// of the shift: column -1 values for the first strip, and for later strips the
// values lane 63 of the previous strip left in LDS, one entry per row.
//
// Values are V*4096 + tag(t), tag(t) = 4095 - t (t < 4096 within a strip), so
// the zero term is the wave-uniform tag, every move carries its tag change in
// its constant (E and F: -1, diagonal: -2), and a per-lane running max orders a
// column's cells by (V, then smallest row).  The strip hand-over through LDS
// crosses 64 steps of the timeline, so lane 0 adds 64 to what it reads.

__device__ __forceinline__ int32_t shr1(int32_t old, int32_t src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xf, 0xf, false);  // wave_shr:1
}

__global__ __launch_bounds__(64) void k_intra32(const AlignArgs A, const RefTable T) {
  extern __shared__ uint32_t smem[];
  __shared__ int64_t rt_off[SW_MAX_REFS], rt_len[SW_MAX_REFS];
  const int lane = threadIdx.x;
  load_ref_table(T, A.n_refs, rt_off, rt_len, lane);
  int4 *rows = reinterpret_cast<int4 *>(smem);                   // [max_read_len]: q, E, H of lane 63
  uint32_t *win = smem + 4 * A.max_read_len;                      // [wwords]
  const DpConst &K = A.k;
  const int32_t SM = K.sm32 - 1, SX = K.sx32 - 1;                 // diagonal: tag -2
  const int32_t GOE = K.goe_e32, GE = K.ge_e32;                   // E and F moves: tag -1

  for (int64_t tk = blockIdx.x; tk < A.n_tasks; tk += gridDim.x) {
    const int64_t c = tk >> 1;
    const int h = (int)(tk & 1);
    LaneTask t{};
    if (lane == 0) t = load_task(A, rt_len, c, 1 << h);
    const int L = __shfl(t.L, 0, 64);
    if (L == 0) continue;
    const int W = __shfl(t.W, 0, 64);
    const int k = __shfl(t.k, 0, 64);
    const int r = __shfl(t.r, 0, 64);
    const int64_t ws = shfl_i64([](int v, int src) { return __shfl(v, src, 64); }, t.ws, 0);
    __syncthreads();
    // stage the oriented read (one code per row) and the window words
    const uint32_t *rp = A.reads + A.read_word_off[r];
    for (int i = lane; i < L; i += 64) {
      const int src = h == 0 ? i : L - 1 - i;
      const uint32_t b = (rp[src >> 4] >> (2 * (src & 15))) & 3u;
      rows[i].x = (int32_t)(h == 0 ? b : 3u - b);
    }
    const int64_t first = rt_off[k] + (ws >> 4);
    const int64_t last = rt_off[k] + ((rt_len[k] - 1) >> 4);
    const uint32_t sh = 2u * (uint32_t)(ws & 15);
    const int nww = (W + 15) >> 4;
    for (int q = lane; q < nww; q += 64) {
      const uint32_t lo = A.ref_words[first + q];
      const uint32_t hi = (first + q + 1 <= last) ? A.ref_words[first + q + 1] : 0u;
      win[q] = (uint32_t)((((uint64_t)hi << 32) | lo) >> sh);
    }
    __syncthreads();

    uint64_t best = 0;
    const int row_lo = K.final_row ? L - 1 : 0;  // first row that may hold the best cell
    const int nstrips = (W + 63) >> 6;
    for (int s = 0; s < nstrips; ++s) {
      const int col = 64 * s + lane;
      const int32_t w = col < W ? (int32_t)((win[col >> 4] >> (2 * (col & 15))) & 3u) : 5;
      const int width = min(64, W - 64 * s);
      const int nsteps = L + width - 1;
      // registers of lane j before its row 0 (boundary row -1 and the F entering row 0)
      int32_t H = 4096 - lane;               // H(-1, j): lane j+1's first diagonal (tag(j + 1) + 2)
      int32_t Hd1 = 4097 - lane;              // lane 0: H(-1, -1), its diagonal at step 0
      int32_t F = 4095 - lane - (GOE - 1);    // F(0, j) = H(-1, j) - go - ge at step j
      int32_t Eout = 0, Ein = 0;
      int32_t q = 0;
      int32_t M = 0;
      for (int st = 0; st < nsteps; ++st) {
        const int32_t zt = 4095 - st;
        // lane 0 boundary for this step: row st at column 64s - 1
        int32_t e_b, h_b, q_b;
        if (st < L) {
          const int4 rb = rows[st];
          q_b = rb.x;
          if (s == 0) {
            e_b = zt - (GOE - 1);             // E(st, 0) = 0 - go - ge
          } else {
            e_b = rb.y + 64;
          }
        } else {
          q_b = 4;
          e_b = zt - (GOE - 1);
        }
        // H(st, 64s - 1): lane 0 uses it as its diagonal at step st + 1 (tag + 2)
        if (s == 0 || st >= L) {
          h_b = zt + 1;                        // column -1: H = 0
        } else {
          h_b = rows[st].z + 64;
        }
        // shifts from lane j-1 (full exec)
        q = shr1(q_b, q);
        Ein = shr1(e_b, Eout);
        const int32_t Hs = shr1(h_b, H);      // lane j-1's H of the previous step
        const int i = st - lane;
        if (i >= 0 && i < L) {
          const int32_t Hdiag = Hd1;          // lane j-1's H two steps back
          const int32_t sub = q == w ? SM : SX;
          int32_t Hn = max(max(Hdiag + sub, Ein), F);
          Hn = max(Hn, zt);
          M = max(M, i >= row_lo ? Hn : 0);
          const int32_t U = Hn - GOE;
          Eout = max(Ein - GE, U);
          F = max(F - GE, U);
          H = Hn;
          if (lane == 63) {
            rows[i].y = Eout;
            rows[i].z = Hn;
          }
        }
        Hd1 = Hs;
      }
      const int32_t v = M >> 12;
      if (v > 0 && col < W) {
        const int32_t row = (4095 - (M & 4095)) - lane;
        const uint64_t kk = cell_key(v, col, row);
        best = kk > best ? kk : best;
      }
      __syncthreads();
    }
    // wave max of the 64-bit keys
    for (int m = 32; m; m >>= 1) {
      const uint64_t o = ((uint64_t)(uint32_t)__shfl_xor((int)(best >> 32), m, 64) << 32) |
                         (uint32_t)__shfl_xor((int)(best & 0xffffffffu), m, 64);
      best = o > best ? o : best;
    }
    if (lane == 0) write_result(A, 2 * c + h, best, ws);
    __syncthreads();
  }
}

// --------------------------------------------------------------------------- intra-task kernel, int16 pairs
//
// One wavefront per CAL with both strands in the 16-bit halves of every
// register (low: forward, high: reverse complement of the read), swept along
// anti-diagonals as in k_intra32: lane j holds window column 64*s + j of strip
// s and computes row i = t - j at step t; the selector of row i's read base, E
// and H move one lane per step through wave_shr:1.
//
// Values carry a bias beta (>= |mismatch|, gap_open + gap_extend, gap_extend) so
// that every operand of the three-way maxima is a non-negative int16 below
// 0x7C00, where the packed half-precision maximum orders as the integer one:
// H = max(diagonal, E, F) and the clamped gap terms max(E - ge, H - go - ge, 0)
// and max(F - ge, H - go - ge, 0) are one v_pk_maximum3_f16 each (clamping E
// and F at zero leaves H unchanged, and the clamped terms follow the same
// recurrence).  The zero of H is the bias itself.
//
// No position tags ride on the values: each lane keeps, per half, a running
// 32-bit maximum of (H << 16 | 0xFFFF - t).  A lane meets its column's rows in
// increasing order, so among equal values the largest key is the earliest step,
// i.e. the smallest row.
//
// The substitution comes from one v_perm_b32 per cell: the lane's column base
// fixes a table of the score's low and high bytes per read base, and each row's
// selector word holds (q_fwd, q_fwd + 4, q_rev, q_rev + 4).

template <bool FR>
__global__ __launch_bounds__(64) void k_intra16(const AlignArgs A, const RefTable T) {
  extern __shared__ uint32_t smem[];
  __shared__ int64_t rt_off[SW_MAX_REFS], rt_len[SW_MAX_REFS];
  const int lane = threadIdx.x;
  load_ref_table(T, A.n_refs, rt_off, rt_len, lane);
  uint4 *rows = reinterpret_cast<uint4 *>(smem);  // [max_read_len]: selector, E and H of lane 63
  uint32_t *win = smem + 4 * A.max_read_len;       // [wwords]
  const DpConst &K = A.k;
  const uint32_t beta = (uint32_t)K.beta16 * 0x00010001u;
  const uint32_t goe2 = (uint32_t)K.goe * 0x00010001u, ge2 = (uint32_t)K.ge * 0x00010001u;
  const uint32_t xlo = (uint32_t)K.mismatch & 0xFFu, mlo = (uint32_t)K.match & 0xFFu;
  const uint32_t xhi = ((uint32_t)K.mismatch >> 8) & 0xFFu, mhi = ((uint32_t)K.match >> 8) & 0xFFu;

  for (int64_t c = blockIdx.x; c < A.n_cals; c += gridDim.x) {
    LaneTask t{};
    if (lane == 0) t = load_task(A, rt_len, c, 3);
    const int L = __shfl(t.L, 0, 64);
    if (L == 0) continue;
    const int W = __shfl(t.W, 0, 64);
    const int k = __shfl(t.k, 0, 64);
    const int r = __shfl(t.r, 0, 64);
    const int mask = __shfl(t.mask, 0, 64);
    const int64_t ws = shfl_i64([](int v, int src) { return __shfl(v, src, 64); }, t.ws, 0);
    __syncthreads();
    // stage the selectors of the oriented read rows and the window words
    const uint32_t *rp = A.reads + A.read_word_off[r];
    for (int i = lane; i < L; i += 64) {
      const uint32_t bf = (rp[i >> 4] >> (2 * (i & 15))) & 3u;
      const int ir = L - 1 - i;
      const uint32_t br = 3u - ((rp[ir >> 4] >> (2 * (ir & 15))) & 3u);
      // the first strip's left boundary: E(i, 0) and H(i, -1) are zero
      rows[i] = make_uint4(bf | ((bf + 4u) << 8) | (br << 16) | ((br + 4u) << 24), beta, beta, 0u);
    }
    const int64_t first = rt_off[k] + (ws >> 4);
    const int64_t last = rt_off[k] + ((rt_len[k] - 1) >> 4);
    const uint32_t sh = 2u * (uint32_t)(ws & 15);
    const int nww = (W + 15) >> 4;
    for (int q = lane; q < nww; q += 64) {
      const uint32_t lo = A.ref_words[first + q];
      const uint32_t hi = (first + q + 1 <= last) ? A.ref_words[first + q + 1] : 0u;
      win[q] = (uint32_t)((((uint64_t)hi << 32) | lo) >> sh);
    }
    __syncthreads();

    uint64_t best_f = 0, best_r = 0;
    const int nstrips = (W + 63) >> 6;
    for (int s = 0; s < nstrips; ++s) {
      const int col = 64 * s + lane;
      // the lane's substitution table: every read base against its column's base
      // (columns past the window score mismatches; nothing reported comes from them)
      uint32_t tlo = xlo * 0x01010101u, thi = xhi * 0x01010101u;
      if (col < W) {
        const uint32_t w = (win[col >> 4] >> (2 * (col & 15))) & 3u;
        tlo ^= (xlo ^ mlo) << (8 * w);
        thi ^= (xhi ^ mhi) << (8 * w);
      }
      const int width = min(64, W - 64 * s);
      const int nsteps = L + width - 1;
      uint32_t H = beta, Hd1 = beta, F = beta, Eout = beta, q = 0;
      uint32_t M_f = 0, M_r = 0;
      // lane 0's left boundary for row st (its selector, E(st, 64s) and H(st, 64s - 1)),
      // read one step ahead; past the last row the entry of row L - 1 stands in (lane 0
      // and every lane it feeds are past the read's end there, so it is never used)
      uint4 nb = rows[0];
      for (int st = 0; st < nsteps; ++st) {
        const uint4 rb = nb;
        nb = rows[min(st + 1, L - 1)];
        q = (uint32_t)shr1((int32_t)rb.x, (int32_t)q);
        const uint32_t Ein = (uint32_t)shr1((int32_t)rb.y, (int32_t)Eout);
        const uint32_t Hs = (uint32_t)shr1((int32_t)rb.z, (int32_t)H);
        const int i = st - lane;
        if (i >= 0 && i < L) {
          const uint32_t sub = __builtin_amdgcn_perm(thi, tlo, q);
          const uint32_t diag = bits(pair(Hd1) + pair(sub));
          const uint32_t Hn = half_max3(diag, Ein, F);
          if (!FR || i == L - 1) {
            const uint32_t tag = 0xFFFFu - (uint32_t)st;
            M_f = max(M_f, (Hn << 16) | tag);
            M_r = max(M_r, (Hn & 0xFFFF0000u) | tag);
          }
          const uint32_t U = bits(pair(Hn) - pair(goe2));
          Eout = half_max3(bits(pair(Ein) - pair(ge2)), U, beta);
          F = half_max3(bits(pair(F) - pair(ge2)), U, beta);
          H = Hn;
          if (lane == 63) {
            rows[i].y = Eout;
            rows[i].z = Hn;
          }
        }
        Hd1 = Hs;
      }
      if (col < W) {
        const int32_t vf = (int32_t)(M_f >> 16) - K.beta16, vr = (int32_t)(M_r >> 16) - K.beta16;
        if (vf > 0) {
          const uint64_t kk = cell_key(vf, col, (int32_t)(0xFFFFu - (M_f & 0xFFFFu)) - lane);
          best_f = kk > best_f ? kk : best_f;
        }
        if (vr > 0) {
          const uint64_t kk = cell_key(vr, col, (int32_t)(0xFFFFu - (M_r & 0xFFFFu)) - lane);
          best_r = kk > best_r ? kk : best_r;
        }
      }
      __syncthreads();
    }
    // wave maxima of the 64-bit keys
    for (int m = 32; m; m >>= 1) {
      const uint64_t of = ((uint64_t)(uint32_t)__shfl_xor((int)(best_f >> 32), m, 64) << 32) |
                          (uint32_t)__shfl_xor((int)(best_f & 0xffffffffu), m, 64);
      const uint64_t orr = ((uint64_t)(uint32_t)__shfl_xor((int)(best_r >> 32), m, 64) << 32) |
                           (uint32_t)__shfl_xor((int)(best_r & 0xffffffffu), m, 64);
      best_f = of > best_f ? of : best_f;
      best_r = orr > best_r ? orr : best_r;
    }
    if (lane == 0) {
      if (mask & 1) write_result(A, 2 * c, best_f, ws);
      if (mask & 2) write_result(A, 2 * c + 1, best_r, ws);
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------------- batched planning
//
// Tasks are binned by read length so that the lanes of a tile share their
// strip count; bins are laid out longest first (largest work first onto the
// queue) and cut into tiles of at most 64 tasks.  Every step runs on the
// device, so the whole batched call needs no host synchronisation and can be
// captured into a HIP graph.

__device__ __forceinline__ int task_bin(const int32_t *cal_read, const int32_t *read_len, int32_t n_reads,
                                        int64_t c, const BinParams &P) {
  const int32_t r = cal_read[c];
  if (r < 0 || r >= n_reads) return P.nb;
  const int32_t L = read_len[r];
  if (L < 1 || L > P.max_read_len) return P.nb;
  return (L - 1) / P.bin_width;
}

__global__ void k_bin_count(const int32_t *__restrict__ cal_read, const int32_t *__restrict__ read_len,
                            int32_t n_reads, int64_t n_tasks, int32_t *__restrict__ bin_count, const BinParams P) {
  extern __shared__ int32_t hist[];
  for (int i = threadIdx.x; i <= P.nb; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_tasks;
       k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&hist[task_bin(cal_read, read_len, n_reads, k / P.per_cal, P)], 1);
  __syncthreads();
  for (int i = threadIdx.x; i <= P.nb; i += blockDim.x)
    if (hist[i]) atomicAdd(&bin_count[i], hist[i]);
}

// Bin order, bin offsets, tile offsets, strip height per bin, and the queue
// reset.  The block stages the bin counts in LDS and computes each bin's strip
// height in parallel; one thread then runs the prefix sums over LDS (a serial
// loop over global loads would pay a load latency per bin).
__global__ void k_bin_plan(const int32_t *__restrict__ bin_count, int32_t *__restrict__ bin_off,
                           int32_t *__restrict__ bin_cursor, int32_t *__restrict__ tile_off,
                           int32_t *__restrict__ tile_bin, int32_t *__restrict__ strip_of_bin,
                           int32_t *__restrict__ n_tiles, int32_t *__restrict__ queue, const BinParams P) {
  extern __shared__ int32_t cnt[];  // [nb + 1]
  if (blockIdx.x != 0) return;
  for (int b = threadIdx.x; b <= P.nb; b += blockDim.x) {
    cnt[b] = bin_count[b];
    strip_of_bin[b] = b < P.nb ? bin_strip_height(P, min((b + 1) * P.bin_width, P.max_read_len)) : P.strips[0];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  int32_t pos = 0, tiles = 0;
  for (int k = 0; k <= P.nb; ++k) {
    const int b = k == P.nb ? P.nb : (P.descending ? P.nb - 1 - k : k);
    bin_off[b] = pos;
    bin_cursor[b] = pos;
    tile_off[k] = tiles;
    tile_bin[k] = b;
    const int32_t c = cnt[b];
    pos += c;
    tiles += (c + 63) / 64;
  }
  tile_off[P.nb + 1] = tiles;
  *n_tiles = tiles;
  *queue = 0;
}

__global__ void k_bin_scatter(const int32_t *__restrict__ cal_read, const int32_t *__restrict__ read_len,
                              int32_t n_reads, int64_t n_tasks, int32_t *__restrict__ bin_cursor,
                              int32_t *__restrict__ order, const BinParams P) {
  extern __shared__ int32_t sh[];
  int32_t *cnt = sh;                // [nb+1]
  int32_t *base = sh + (P.nb + 1);  // [nb+1]
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // the block handles the tasks k = k0 + j*stride, one pass per j
  for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x; k0 < n_tasks; k0 += stride) {
    for (int i = threadIdx.x; i <= P.nb; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const int64_t k = k0 + threadIdx.x;
    int b = -1;
    if (k < n_tasks) {
      b = task_bin(cal_read, read_len, n_reads, k / P.per_cal, P);
      atomicAdd(&cnt[b], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= P.nb; i += blockDim.x) {
      base[i] = cnt[i] ? atomicAdd(&bin_cursor[i], cnt[i]) : 0;
      cnt[i] = 0;
    }
    __syncthreads();
    if (b >= 0) {
      const int local = atomicAdd(&cnt[b], 1);
      order[base[b] + local] = (int32_t)k;
    }
    __syncthreads();
  }
}

__global__ void k_tile_fill(const int32_t *__restrict__ bin_count, const int32_t *__restrict__ bin_off,
                            const int32_t *__restrict__ tile_off, const int32_t *__restrict__ tile_bin,
                            const int32_t *__restrict__ strip_of_bin, const int32_t *__restrict__ n_tiles,
                            int32_t *__restrict__ tiles, int32_t *__restrict__ tile_len,
                            int32_t *__restrict__ tile_strips, int32_t max_tiles, const BinParams P) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= *n_tiles || t >= max_tiles) return;
  int lo = 0, hi = P.nb;  // find k with tile_off[k] <= t < tile_off[k+1]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_off[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  const int b = tile_bin[lo];
  const int32_t j = t - tile_off[lo];
  tiles[t] = bin_off[b] + 64 * j;
  tile_len[t] = min(64, bin_count[b] - 64 * j);
  tile_strips[t] = strip_of_bin[b];
}

// --------------------------------------------------------------------------- launchers

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_pack(const uint8_t *codes, int64_t n, uint32_t *words, hipStream_t st) {
  int64_t nw = (n + 15) / 16;
  if (nw == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_2bit, dim3(blocks_for(nw, 256)), dim3(256), 0, st, codes, n, words, nw);
  return hipGetLastError();
}

hipError_t launch_expand(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, int32_t *cal_read,
                         hipStream_t st) {
  if (n_cals > 0)
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n_cals, 256)), dim3(256), 0, st, cal_read, n_cals, -1);
  if (n_reads > 0)
    hipLaunchKernelGGL(k_cal_owner, dim3(blocks_for(n_reads, 256)), dim3(256), 0, st, cal_ptr, n_reads,
                       n_cals, cal_read);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

template <int R>
static hipError_t launch_inter16_r(const AlignArgs &A, const RefTable &T, int grid, size_t lds,
                                   hipStream_t st) {
  if (A.k.final_row)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inter16<R, true>), dim3(grid), dim3(64), lds, st, A, T);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inter16<R, false>), dim3(grid), dim3(64), lds, st, A, T);
  return hipGetLastError();
}
template <int R>
static hipError_t launch_inter32_r(const AlignArgs &A, const RefTable &T, int grid, size_t lds,
                                   hipStream_t st) {
  if (A.k.perm32)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inter32<R, true>), dim3(grid), dim3(64), lds, st, A, T);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inter32<R, false>), dim3(grid), dim3(64), lds, st, A, T);
  return hipGetLastError();
}

#define SW_INTER16_CASE(RR) \
  case RR:                  \
    return launch_inter16_r<RR>(A, T, grid, lds, st);
#define SW_INTER32_CASE(RR) \
  case RR:                  \
    return launch_inter32_r<RR>(A, T, grid, lds, st);

hipError_t launch_inter(bool int16, const AlignArgs &A, const RefTable &T, int grid, hipStream_t st) {
  size_t lds = (size_t)(A.wwords + A.rwords) * 64 * sizeof(uint32_t);
  if (int16) {
    switch (A.strip_rows) { SW_INTER16_STRIPS(SW_INTER16_CASE) default: return hipErrorInvalidValue; }
  } else {
    switch (A.strip_rows) { SW_INTER32_STRIPS(SW_INTER32_CASE) default: return hipErrorInvalidValue; }
  }
}

hipError_t launch_batch_plan(const BatchBufs &B, const int32_t *read_len, int32_t n_reads, int64_t n_tasks,
                             const BinParams &P, hipStream_t st) {
  if (n_tasks == 0) return hipSuccess;
  const int nbins = P.nb + 1;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(nbins, 256)), dim3(256), 0, st, B.bin_count, (int64_t)nbins, 0);
  const int grid = (int)std::min<int64_t>(1024, blocks_for(n_tasks, 256));
  hipLaunchKernelGGL(k_bin_count, dim3(grid), dim3(256), nbins * sizeof(int32_t), st, B.cal_read, read_len,
                     n_reads, n_tasks, B.bin_count, P);
  hipLaunchKernelGGL(k_bin_plan, dim3(1), dim3(256), nbins * sizeof(int32_t), st, B.bin_count, B.bin_off,
                     B.bin_cursor, B.tile_off, B.tile_bin, B.strip_of_bin, B.n_tiles, B.queue, P);
  hipLaunchKernelGGL(k_bin_scatter, dim3(grid), dim3(256), 2 * nbins * sizeof(int32_t), st, B.cal_read, read_len,
                     n_reads, n_tasks, B.bin_cursor, B.order, P);
  const int64_t max_tiles = (n_tasks + 63) / 64 + nbins;
  hipLaunchKernelGGL(k_tile_fill, dim3(blocks_for(max_tiles, 256)), dim3(256), 0, st, B.bin_count, B.bin_off,
                     B.tile_off, B.tile_bin, B.strip_of_bin, B.n_tiles, B.tiles, B.tile_len, B.tile_strips,
                     (int32_t)max_tiles, P);
  return hipGetLastError();
}

hipError_t launch_inter_queue(bool int16, const AlignArgs &A, const RefTable &T, int grid, hipStream_t st) {
  size_t lds = (size_t)(A.wwords + A.rwords) * 64 * sizeof(uint32_t);
  if (int16 && A.k.final_row)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inter16_queue<true>), dim3(grid), dim3(64), lds, st, A, T);
  else if (int16)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inter16_queue<false>), dim3(grid), dim3(64), lds, st, A, T);
  else if (A.k.perm32)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inter32_queue<true>), dim3(grid), dim3(64), lds, st, A, T);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inter32_queue<false>), dim3(grid), dim3(64), lds, st, A, T);
  return hipGetLastError();
}

int queue_blocks_per_cu(bool int16) {
  int n = 0;
  const void *f = int16 ? reinterpret_cast<const void *>(&k_inter16_queue<false>)
                        : reinterpret_cast<const void *>(&k_inter32_queue<false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64, 8192) != hipSuccess) return 0;
  return n;
}

hipError_t launch_intra(bool int16, const AlignArgs &A, const RefTable &T, int grid, hipStream_t st) {
  const size_t lds = (size_t)A.max_read_len * sizeof(int4) + (size_t)A.wwords * sizeof(uint32_t);
  if (!int16)
    hipLaunchKernelGGL(k_intra32, dim3(grid), dim3(64), lds, st, A, T);
  else if (A.k.final_row)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_intra16<true>), dim3(grid), dim3(64), lds, st, A, T);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_intra16<false>), dim3(grid), dim3(64), lds, st, A, T);
  return hipGetLastError();
}

int intra_blocks_per_cu(bool int16, size_t lds) {
  int n = 0;
  const void *f = int16 ? reinterpret_cast<const void *>(&k_intra16<false>) : reinterpret_cast<const void *>(&k_intra32);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64, lds) != hipSuccess) return 0;
  return n;
}


// --------------------------------------------------------------------------- queries

__device__ unsigned long long g_invalid_tasks;

unsigned long long *error_counter() {
  static void *addr[64] = {nullptr};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  if (!addr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_invalid_tasks)) != hipSuccess) return nullptr;
    addr[dev] = p;
  }
  return (unsigned long long *)addr[dev];
}

template <int R>
static int occ16(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_inter16<R, false>), 64,
                                                  lds) != hipSuccess)
    return 0;
  return n;
}
template <int R>
static int occ32(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_inter32<R, false>), 64,
                                                  lds) != hipSuccess)
    return 0;
  return n;
}

#define SW_OCC16_CASE(RR) \
  case RR:                \
    return occ16<RR>(8192);
#define SW_OCC32_CASE(RR) \
  case RR:                \
    return occ32<RR>(8192);

int inter_blocks_per_cu(bool int16, int strip_rows) {
  if (int16) {
    switch (strip_rows) { SW_INTER16_STRIPS(SW_OCC16_CASE) default: return 0; }
  } else {
    switch (strip_rows) { SW_INTER32_STRIPS(SW_OCC32_CASE) default: return 0; }
  }
}

}  // namespace swk
