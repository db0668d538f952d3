/*
 * CPU oracle for affine-gap Smith-Waterman (Gotoh) scoring of short reads
 * against candidate-alignment-location (CAL) windows.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU library and must never be called by the product path.
 *
 * What it computes (McVicar et al., "FPGA Acceleration of Short Read
 * Alignment"):
 *   - Each read is scored against the reference around each of its CALs with
 *     Smith-Waterman under the affine gap model (section 3.5).  The paper
 *     defers the recurrences to an external reference; the ones used here are
 *     Gotoh's three-state local-alignment recurrences, written in the plain
 *     full-matrix form:
 *         E(i,j) = max(E(i,j-1) - ge, H(i,j-1) - go - ge)   gap consuming window base j
 *         F(i,j) = max(F(i-1,j) - ge, H(i-1,j) - go - ge)   gap consuming read base i
 *         H(i,j) = max(0, H(i-1,j-1) + s(q_i, w_j), E(i,j), F(i,j))
 *     with H = 0 and E = F = -infinity on the boundary, so a gap of k bases
 *     costs go + k*ge.
 *   - The read is aligned in the direction given by the strand bit kept with
 *     each CAL (section 3.1): the reverse strand aligns the reverse complement
 *     of the read (complement = 3 - code with A,C,G,T = 0,1,2,3, Fig. 3)
 *     against the forward reference window.
 *   - The Score Tracker keeps the best-scoring CAL per read (sections 3.6, 4.2),
 *     or some number of the best CALs, or all CALs tied for the best score
 *     (the variants section 4.2 lists).
 *
 * Readings of points the paper leaves open (each is also listed in the design
 * notes of the repository):
 *   - score = the maximum over every cell of H (a full local maximum) by
 *     default; the final-row mode keeps only the last read row, which is the
 *     paper's own V1 output (the best cell of the final row, sections 3.5 and
 *     3.6), so the alignment ends at the read's last base;
 *   - window = [p - band, p + L + band) clipped to the reference;
 *   - ties inside a task: highest score, then smallest reference end, then
 *     smallest read end; score 0 reports both ends as -1;
 *   - ties across the CALs of a read: lowest slot index (slot 2c forward,
 *     2c+1 reverse) and the number of tied slots is reported.
 *
 * Arithmetic is int64 throughout; the matrices are allocated in full.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORACLE_NEG_INF (INT64_MIN / 4)

typedef struct {
  int32_t match, mismatch, gap_open, gap_extend, band;
  /* 0: best cell anywhere (full local maximum); 1: best cell of the final row
   * only, i.e. the alignment must end at the last read base (the V1 array's
   * output, sections 3.5 and 3.6) */
  int32_t final_row;
} oracle_scoring_t;

/* Result of one task. */
typedef struct {
  int64_t score, ref_end, read_end;
} oracle_hit_t;

static inline int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

/*
 * Gotoh local alignment of q[0..L) against w[0..W) with full matrices.
 * buf must hold 3*(L+1)*(W+1) int64 values.  Ends are 0-based; (-1, -1) when
 * the best score is 0.
 */
static oracle_hit_t gotoh_full(const uint8_t *q, int64_t L, const uint8_t *w, int64_t W,
                               const oracle_scoring_t *sc, int64_t *buf) {
  const int64_t cols = W + 1;
  int64_t *H = buf;
  int64_t *E = buf + (L + 1) * cols;
  int64_t *F = buf + 2 * (L + 1) * cols;
  const int64_t go = sc->gap_open, ge = sc->gap_extend;
#define AT(M, i, j) M[(i) * cols + (j)]
  for (int64_t j = 0; j <= W; ++j) {
    AT(H, 0, j) = 0;
    AT(E, 0, j) = ORACLE_NEG_INF;
    AT(F, 0, j) = ORACLE_NEG_INF;
  }
  for (int64_t i = 1; i <= L; ++i) {
    AT(H, i, 0) = 0;
    AT(E, i, 0) = ORACLE_NEG_INF;
    AT(F, i, 0) = ORACLE_NEG_INF;
    for (int64_t j = 1; j <= W; ++j) {
      int64_t s = (q[i - 1] == w[j - 1]) ? sc->match : sc->mismatch;
      AT(E, i, j) = max2(AT(E, i, j - 1) - ge, AT(H, i, j - 1) - go - ge);
      AT(F, i, j) = max2(AT(F, i - 1, j) - ge, AT(H, i - 1, j) - go - ge);
      int64_t h = AT(H, i - 1, j - 1) + s;
      h = max2(h, AT(E, i, j));
      h = max2(h, AT(F, i, j));
      AT(H, i, j) = max2(h, 0);
    }
  }
  /* best cell: highest score, then smallest window column, then smallest read row */
  oracle_hit_t best = {0, -1, -1};
  const int64_t i_first = sc->final_row ? L : 1;
  for (int64_t j = 1; j <= W; ++j) {
    for (int64_t i = i_first; i <= L; ++i) {
      int64_t v = AT(H, i, j);
      if (v > best.score) {
        best.score = v;
        best.ref_end = j - 1;
        best.read_end = i - 1;
      }
    }
  }
#undef AT
  return best;
}

/* Single pair, exposed for the brute-force and invariant tests. */
void oracle_gotoh_many(const uint8_t *q_codes, const int64_t *q_off, const int64_t *q_len,
                       const uint8_t *w_codes, const int64_t *w_off, const int64_t *w_len,
                       int64_t n, const oracle_scoring_t *sc, int64_t *score, int64_t *ref_end,
                       int64_t *read_end) {
  int64_t cap = 0;
  int64_t *buf = NULL;
  for (int64_t k = 0; k < n; ++k) {
    int64_t need = 3 * (q_len[k] + 1) * (w_len[k] + 1);
    if (need > cap) {
      free(buf);
      cap = need;
      buf = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    }
    oracle_hit_t h = gotoh_full(q_codes + q_off[k], q_len[k], w_codes + w_off[k], w_len[k], sc, buf);
    score[k] = h.score;
    ref_end[k] = h.ref_end;
    read_end[k] = h.read_end;
  }
  free(buf);
}

/* ---------------------------------------------------------------- batch */

typedef struct {
  const uint8_t *read_codes;
  const int64_t *read_off;
  const int32_t *read_len;
  int32_t n_reads;
  const uint8_t *ref_codes;
  const int64_t *ref_off;
  const int64_t *ref_len;
  int32_t n_refs;
  const int64_t *cal_ptr;
  const int64_t *cal_read; /* owning read of each CAL */
  const int64_t *cal_pos;
  const int16_t *cal_ref;
  const uint8_t *strand;
  int64_t n_cals;
  oracle_scoring_t sc;
  int32_t max_read_len;
  int32_t *score;
  int64_t *ref_end;
  int16_t *read_end;
  int64_t begin, end; /* CAL range of this worker */
  int64_t errors;
} batch_job_t;

static void *batch_worker(void *arg) {
  batch_job_t *jb = (batch_job_t *)arg;
  int64_t cap = 0;
  int64_t *buf = NULL;
  uint8_t *qbuf = (uint8_t *)malloc((size_t)jb->max_read_len + 1);
  for (int64_t c = jb->begin; c < jb->end; ++c) {
    int64_t r = jb->cal_read[c];
    int64_t L = jb->read_len[r];
    int64_t k = jb->cal_ref[c];
    int64_t p = jb->cal_pos[c];
    uint8_t mask = jb->strand[c];
    int valid = (k >= 0 && k < jb->n_refs && L >= 1 && L <= jb->max_read_len);
    if (valid) valid = (p >= 0 && p < jb->ref_len[k]);
    for (int h = 0; h < 2; ++h) {
      int64_t slot = 2 * c + h;
      jb->score[slot] = -1;
      jb->ref_end[slot] = -1;
      jb->read_end[slot] = -1;
      if (!(mask & (1 << h))) continue;
      if (!valid) {
        jb->score[slot] = INT32_MIN;
        jb->errors++;
        continue;
      }
      const uint8_t *read = jb->read_codes + jb->read_off[r];
      /* oriented read: forward as given, reverse = reverse complement */
      for (int64_t i = 0; i < L; ++i) qbuf[i] = h == 0 ? read[i] : (uint8_t)(3 - read[L - 1 - i]);
      int64_t ws = p - jb->sc.band;
      if (ws < 0) ws = 0;
      int64_t we = p + L + jb->sc.band;
      if (we > jb->ref_len[k]) we = jb->ref_len[k];
      int64_t W = we - ws;
      int64_t need = 3 * (L + 1) * (W + 1);
      if (need > cap) {
        free(buf);
        cap = need;
        buf = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
      }
      oracle_hit_t hit = gotoh_full(qbuf, L, jb->ref_codes + jb->ref_off[k] + ws, W, &jb->sc, buf);
      jb->score[slot] = (int32_t)hit.score;
      if (hit.score > 0) {
        jb->ref_end[slot] = ws + hit.ref_end;
        jb->read_end[slot] = (int16_t)hit.read_end;
      }
    }
  }
  free(buf);
  free(qbuf);
  return NULL;
}

/*
 * Score every requested (CAL, strand) slot.  Outputs have 2*n_cals entries:
 * slot 2c forward, 2c+1 reverse.  Unrequested slots: score -1; invalid tasks
 * (reference id, position or read length out of range): score INT32_MIN.
 * Returns the number of invalid task slots.
 */
int64_t oracle_align_batch(const uint8_t *read_codes, const int64_t *read_off, const int32_t *read_len,
                           int32_t n_reads, const uint8_t *ref_codes, const int64_t *ref_off,
                           const int64_t *ref_len, int32_t n_refs, const int64_t *cal_ptr,
                           const int64_t *cal_pos, const int16_t *cal_ref, const uint8_t *strand,
                           int64_t n_cals, const oracle_scoring_t *sc, int32_t max_read_len,
                           int32_t *score, int64_t *ref_end, int16_t *read_end, int32_t n_threads) {
  int64_t *cal_read = (int64_t *)malloc((size_t)(n_cals > 0 ? n_cals : 1) * sizeof(int64_t));
  for (int64_t r = 0; r < n_reads; ++r)
    for (int64_t c = cal_ptr[r]; c < cal_ptr[r + 1]; ++c) cal_read[c] = r;
  if (n_threads < 1) n_threads = 1;
  batch_job_t *jobs = (batch_job_t *)calloc((size_t)n_threads, sizeof(batch_job_t));
  pthread_t *tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  for (int t = 0; t < n_threads; ++t) {
    batch_job_t *jb = &jobs[t];
    jb->read_codes = read_codes; jb->read_off = read_off; jb->read_len = read_len;
    jb->n_reads = n_reads; jb->ref_codes = ref_codes; jb->ref_off = ref_off;
    jb->ref_len = ref_len; jb->n_refs = n_refs; jb->cal_ptr = cal_ptr; jb->cal_read = cal_read;
    jb->cal_pos = cal_pos; jb->cal_ref = cal_ref; jb->strand = strand; jb->n_cals = n_cals;
    jb->sc = *sc; jb->max_read_len = max_read_len; jb->score = score; jb->ref_end = ref_end;
    jb->read_end = read_end;
    jb->begin = n_cals * t / n_threads;
    jb->end = n_cals * (t + 1) / n_threads;
  }
  if (n_threads == 1) {
    batch_worker(&jobs[0]);
  } else {
    for (int t = 0; t < n_threads; ++t) pthread_create(&tids[t], NULL, batch_worker, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(tids[t], NULL);
  }
  int64_t errors = 0;
  for (int t = 0; t < n_threads; ++t) errors += jobs[t].errors;
  free(jobs);
  free(tids);
  free(cal_read);
  return errors;
}

/*
 * Best slot per (read, reference): highest score, lowest slot index among ties,
 * and the number of slots tied at that score.  Unrequested and invalid slots
 * (negative scores) are skipped.  A pair with no valid slot reports
 * (-1, -1, 0).  Outputs are [n_reads * n_refs], row-major by read.
 */
void oracle_reduce_best(const int64_t *cal_ptr, const int16_t *cal_ref, int32_t n_reads, int32_t n_refs,
                        const int32_t *score, int32_t *best_score, int64_t *best_slot, int32_t *n_tied) {
  for (int64_t r = 0; r < n_reads; ++r) {
    for (int64_t k = 0; k < n_refs; ++k) {
      best_score[r * n_refs + k] = -1;
      best_slot[r * n_refs + k] = -1;
      n_tied[r * n_refs + k] = 0;
    }
    for (int64_t c = cal_ptr[r]; c < cal_ptr[r + 1]; ++c) {
      int64_t k = cal_ref[c];
      if (k < 0 || k >= n_refs) continue;
      for (int h = 0; h < 2; ++h) {
        int64_t slot = 2 * c + h;
        int32_t s = score[slot];
        if (s < 0) continue;
        int64_t o = r * n_refs + k;
        if (s > best_score[o]) {
          best_score[o] = s;
          best_slot[o] = slot;
          n_tied[o] = 1;
        } else if (s == best_score[o]) {
          n_tied[o] += 1;
        }
      }
    }
  }
}

/*
 * Score Tracker variants (section 4.2): best CAL, top-k CALs, or all tied CALs.
 * Top k slots of each read over all its CALs and strands: highest score first,
 * lower slot index first among equal scores; negative scores are skipped and
 * missing entries are (-1, -1).  Outputs [n_reads * k].
 */
void oracle_topk(const int64_t *cal_ptr, int32_t n_reads, const int32_t *score, int32_t k, int32_t *top_score,
                 int64_t *top_slot) {
  for (int64_t r = 0; r < n_reads; ++r) {
    for (int32_t t = 0; t < k; ++t) {
      top_score[r * k + t] = -1;
      top_slot[r * k + t] = -1;
    }
    for (int64_t slot = 2 * cal_ptr[r]; slot < 2 * cal_ptr[r + 1]; ++slot) {
      int32_t s = score[slot];
      if (s < 0) continue;
      /* insert into the sorted list if it beats the last entry */
      int32_t pos = k;
      while (pos > 0) {
        int32_t ps = top_score[r * k + pos - 1];
        int64_t pl = top_slot[r * k + pos - 1];
        int beats = pl < 0 || s > ps || (s == ps && slot < pl);
        if (!beats) break;
        pos--;
      }
      if (pos >= k) continue;
      for (int32_t t = k - 1; t > pos; --t) {
        top_score[r * k + t] = top_score[r * k + t - 1];
        top_slot[r * k + t] = top_slot[r * k + t - 1];
      }
      top_score[r * k + pos] = s;
      top_slot[r * k + pos] = slot;
    }
  }
}

/* Slots whose score equals the best score of their read over all references
 * (and is non-negative): flag 1, else 0.  Output [2 * n_cals]. */
void oracle_tied_flags(const int64_t *cal_ptr, int32_t n_reads, const int32_t *score, uint8_t *flags) {
  for (int64_t r = 0; r < n_reads; ++r) {
    int32_t best = -1;
    for (int64_t slot = 2 * cal_ptr[r]; slot < 2 * cal_ptr[r + 1]; ++slot)
      if (score[slot] > best) best = score[slot];
    for (int64_t slot = 2 * cal_ptr[r]; slot < 2 * cal_ptr[r + 1]; ++slot)
      flags[slot] = (best >= 0 && score[slot] == best) ? 1 : 0;
  }
}

/*
 * Two-or-more-reference classification (section 6.2): a read belongs to the
 * reference with the strictly highest best score if that score reaches the
 * threshold; -2 when two or more references share a top score that reaches
 * it (tie); -1 when no reference reaches it (unaligned).
 */
void oracle_classify(const int32_t *best_score, int32_t n_reads, int32_t n_refs, int32_t threshold,
                     int32_t *cls) {
  for (int64_t r = 0; r < n_reads; ++r) {
    int32_t top = -1, arg = -1, count = 0;
    for (int32_t k = 0; k < n_refs; ++k) {
      int32_t v = best_score[r * n_refs + k];
      if (v > top) {
        top = v;
        arg = k;
        count = 1;
      } else if (v == top) {
        count++;
      }
    }
    if (top < threshold) cls[r] = -1;
    else if (count > 1) cls[r] = -2;
    else cls[r] = arg;
  }
}

/*
 * Start position and CIGAR of selected slots (the alignment behind a score;
 * section 6.4 finds CIGAR string generation the next bottleneck once CALs per
 * seed are limited, Table 5).
 *
 * For slot 2c+h with a positive score, the full H, E, F matrices of the task
 * are rebuilt and walked backwards from the reported end cell.  Several
 * alignments can reach the same score; this walk fixes one by taking, at every
 * cell, the first move that explains its value:
 *   - in H: the diagonal first, then the gap consuming a read base (F), then
 *     the gap consuming a window base (E); a diagonal step that lands on a
 *     cell with H = 0 (or on the boundary) ends the walk: the alignment starts
 *     at the cell it left;
 *   - in F or E: leave the gap (it was opened from H) whenever that explains
 *     the value, otherwise extend it.
 * Operations use the BAM numbering: 1 = I (read base, no window base),
 * 2 = D (window base, no read base), 4 = S (soft clip), 7 = '=' (match),
 * 8 = X (mismatch); each entry is (length << 4) | op, in forward reference
 * order, with the read's unaligned head and tail as soft clips.
 * Outputs per entry t of `slots`: ref_start (absolute forward position),
 * read_start (in the oriented read), n_ops and cigar[t*cap .. t*cap+n_ops).
 * n_ops = 0 with starts -1 when the slot is -1 or its score is not positive;
 * n_ops = -1 (row cleared to 0) when more than `cap` operations are needed;
 * n_ops = -2 when the
 * slot, its task or its reported end is invalid (the end cell's H differs from
 * the reported score).
 */
typedef struct {
  uint32_t op, len;
} oracle_run_t;

static void push_op(oracle_run_t *runs, int64_t *n, uint32_t op) {
  if (*n > 0 && runs[*n - 1].op == op) {
    runs[*n - 1].len++;
  } else {
    runs[*n].op = op;
    runs[*n].len = 1;
    (*n)++;
  }
}

void oracle_traceback(const uint8_t *read_codes, const int64_t *read_off, const int32_t *read_len, int32_t n_reads,
                      const uint8_t *ref_codes, const int64_t *ref_off, const int64_t *ref_len, int32_t n_refs,
                      const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref, int64_t n_cals,
                      const oracle_scoring_t *sc, int32_t max_read_len, const int32_t *score, const int64_t *ref_end,
                      const int16_t *read_end, const int64_t *slots, int64_t n_slots, int32_t cap,
                      int64_t *out_ref_start, int16_t *out_read_start, int32_t *out_n_ops, uint32_t *cigar) {
  const int64_t go = sc->gap_open, ge = sc->gap_extend;
  for (int64_t t = 0; t < n_slots; ++t) {
    out_ref_start[t] = -1;
    out_read_start[t] = -1;
    out_n_ops[t] = 0;
    const int64_t slot = slots[t];
    if (slot == -1) continue;
    if (slot < 0 || slot >= 2 * n_cals) {
      out_n_ops[t] = -2;
      continue;
    }
    const int64_t c = slot >> 1;
    const int h = (int)(slot & 1);
    if (score[slot] <= 0) continue;
    /* owning read: the r with cal_ptr[r] <= c < cal_ptr[r+1] (bisection over
     * the non-decreasing row pointer) */
    int64_t r = -1;
    if (n_reads > 0 && cal_ptr[0] <= c && c < cal_ptr[n_reads]) {
      int64_t lo = 0, hi = n_reads; /* cal_ptr[lo] <= c < cal_ptr[hi] */
      while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (cal_ptr[mid] <= c) lo = mid; else hi = mid;
      }
      r = lo;
    }
    const int64_t k = cal_ref[c];
    const int64_t p = cal_pos[c];
    const int64_t L = r >= 0 ? read_len[r] : 0;
    if (r < 0 || k < 0 || k >= n_refs || L < 1 || L > max_read_len || p < 0 || p >= ref_len[k]) {
      out_n_ops[t] = -2;
      continue;
    }
    int64_t ws = p - sc->band;
    if (ws < 0) ws = 0;
    int64_t we = p + L + sc->band;
    if (we > ref_len[k]) we = ref_len[k];
    const int64_t W = we - ws;
    const int64_t ie = read_end[slot], je = ref_end[slot] - ws; /* 0-based end cell */
    if (ie < 0 || ie >= L || je < 0 || je >= W) {
      out_n_ops[t] = -2;
      continue;
    }
    uint8_t *q = (uint8_t *)malloc((size_t)L);
    const uint8_t *read = read_codes + read_off[r];
    for (int64_t i = 0; i < L; ++i) q[i] = h == 0 ? read[i] : (uint8_t)(3 - read[L - 1 - i]);
    const uint8_t *w = ref_codes + ref_off[k] + ws;
    const int64_t cols = W + 1;
    int64_t *H = (int64_t *)malloc((size_t)(3 * (L + 1) * cols) * sizeof(int64_t));
    int64_t *E = H + (L + 1) * cols;
    int64_t *F = E + (L + 1) * cols;
#define AT(M, i, j) M[(i) * cols + (j)]
    for (int64_t j = 0; j <= W; ++j) {
      AT(H, 0, j) = 0;
      AT(E, 0, j) = ORACLE_NEG_INF;
      AT(F, 0, j) = ORACLE_NEG_INF;
    }
    for (int64_t i = 1; i <= L; ++i) {
      AT(H, i, 0) = 0;
      AT(E, i, 0) = ORACLE_NEG_INF;
      AT(F, i, 0) = ORACLE_NEG_INF;
      for (int64_t j = 1; j <= W; ++j) {
        const int64_t s = q[i - 1] == w[j - 1] ? sc->match : sc->mismatch;
        AT(E, i, j) = max2(AT(E, i, j - 1) - ge, AT(H, i, j - 1) - go - ge);
        AT(F, i, j) = max2(AT(F, i - 1, j) - ge, AT(H, i - 1, j) - go - ge);
        AT(H, i, j) = max2(max2(AT(H, i - 1, j - 1) + s, AT(E, i, j)), max2(AT(F, i, j), 0));
      }
    }
    /* 1-based walk from the end cell; runs are collected end first */
    int64_t i = ie + 1, j = je + 1;
    if (AT(H, i, j) != score[slot]) {
      out_n_ops[t] = -2;
      free(H);
      free(q);
      continue;
    }
    oracle_run_t *runs = (oracle_run_t *)malloc((size_t)(L + W + 2) * sizeof(oracle_run_t));
    int64_t n = 0;
    if (L - i > 0) {
      runs[0].op = 4;
      runs[0].len = (uint32_t)(L - i);
      n = 1;
    }
    enum { ST_H, ST_E, ST_F } st = ST_H;
    for (;;) {
      if (st == ST_H) {
        if (i == 0 || j == 0 || AT(H, i, j) == 0) break; /* the previous diagonal step was the first pair */
        const int64_t s = q[i - 1] == w[j - 1] ? sc->match : sc->mismatch;
        if (AT(H, i, j) == AT(H, i - 1, j - 1) + s) {
          push_op(runs, &n, q[i - 1] == w[j - 1] ? 7u : 8u);
          --i;
          --j;
        } else if (AT(H, i, j) == AT(F, i, j)) {
          st = ST_F;
        } else {
          st = ST_E;
        }
      } else if (st == ST_F) {
        push_op(runs, &n, 1u);
        if (AT(F, i, j) == AT(H, i - 1, j) - go - ge) st = ST_H;
        --i;
      } else {
        push_op(runs, &n, 2u);
        if (AT(E, i, j) == AT(H, i, j - 1) - go - ge) st = ST_H;
        --j;
      }
    }
#undef AT
    /* (i, j) is now the 1-based predecessor of the first aligned pair */
    if (i > 0) {
      runs[n].op = 4;
      runs[n].len = (uint32_t)i;
      n++;
    }
    if (n > cap) {
      out_n_ops[t] = -1;
      for (int64_t x = 0; x < cap; ++x) cigar[t * cap + x] = 0;
    } else {
      out_ref_start[t] = ws + j;
      out_read_start[t] = (int16_t)i;
      out_n_ops[t] = (int32_t)n;
      for (int64_t x = 0; x < n; ++x) cigar[t * cap + x] = (runs[n - 1 - x].len << 4) | runs[n - 1 - x].op;
    }
    free(runs);
    free(H);
    free(q);
  }
}

/*
 * CAL Filter (section 3.3): duplicate CALs of a read are combined into one
 * reference lookup.  Two CALs of the same read are duplicates when they name
 * the same reference and their positions fall in the same bucket of
 * 2^bucket_bits bases (bucket_bits = 0: identical positions).  Each read keeps
 * the first CAL of every bucket, in input order, with the union of the strand
 * masks of its duplicates; cal_map[c] is the output CAL that input CAL c was
 * folded into.  Outputs: out_ptr [n_reads+1], out_pos/out_ref/out_strand
 * [out_ptr[n_reads]], cal_map [n_cals].  Returns the number of output CALs.
 */
int64_t oracle_cal_filter(const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref,
                          const uint8_t *strand, int32_t n_reads, int32_t bucket_bits, int64_t *out_ptr,
                          int64_t *out_pos, int16_t *out_ref, uint8_t *out_strand, int64_t *cal_map) {
  int64_t n = 0;
  out_ptr[0] = 0;
  for (int64_t r = 0; r < n_reads; ++r) {
    const int64_t first_out = n;
    for (int64_t c = cal_ptr[r]; c < cal_ptr[r + 1]; ++c) {
      int64_t hit = -1;
      for (int64_t o = first_out; o < n && hit < 0; ++o)
        if (out_ref[o] == cal_ref[c] && (out_pos[o] >> bucket_bits) == (cal_pos[c] >> bucket_bits)) hit = o;
      if (hit < 0) {
        hit = n++;
        out_pos[hit] = cal_pos[c];
        out_ref[hit] = cal_ref[c];
        out_strand[hit] = 0;
      }
      out_strand[hit] |= strand[c];
      cal_map[c] = hit;
    }
    out_ptr[r + 1] = n;
  }
  return n;
}

/*
 * Seeding and CAL finding (sections 3.1 and 3.2).
 *
 * A seed is a string of seed_len consecutive bases (seed_len <= 32).  The
 * reference is cut into every overlapping seed; a read is cut into seeds
 * starting at offsets 0, stride, 2*stride, ... that fit in the read (stride 1:
 * overlapping seeds, stride = seed_len: non-overlapping ones).  A read seed s
 * matches reference position x of reference k in the forward orientation when
 * the reference seed there equals s, and in the reverse orientation when it
 * equals the reverse complement of s (the index keeps one canonical form per
 * seed and a strand bit, section 3.1; matching both orientations is what that
 * construction achieves).  A palindromic seed matches both ways.
 *
 * A read seed with more than max_cals_per_seed matches (0: no limit)
 * contributes nothing (the per-seed CAL limit of the index).  Otherwise each
 * match becomes one CAL:
 *   forward: strand 1, position x - o (where read base 0 falls);
 *   reverse: strand 2, position x - (L - o - seed_len) (where base 0 of the
 *            read's reverse complement falls);
 * clipped to [0, length of reference k).  A read's CALs are listed seed by
 * seed, each seed's matches by (reference, position), the forward match of a
 * palindrome before the reverse one.
 *
 * The reference seeds are found through a sorted array of (seed, reference,
 * position) triples and binary search, the plainest exact lookup; the hashed
 * pointer and CAL tables of the paper are a storage layout with the same
 * answers.  Returns the total number of CALs; only `capacity` are written.
 */
typedef struct {
  uint64_t seed;
  int32_t ref;
  int64_t pos;
} oracle_occ_t;

static uint64_t seed_at(const uint8_t *s, int S) {
  uint64_t v = 0;
  for (int i = 0; i < S; ++i) v = (v << 2) | (uint64_t)(s[i] & 3);
  return v;
}

static uint64_t seed_revcomp(uint64_t v, int S) {
  uint64_t r = 0;
  for (int i = 0; i < S; ++i) {
    r = (r << 2) | (3 - (v & 3));
    v >>= 2;
  }
  return r;
}

static int occ_cmp(const void *a, const void *b) {
  const oracle_occ_t *x = (const oracle_occ_t *)a, *y = (const oracle_occ_t *)b;
  if (x->seed != y->seed) return x->seed < y->seed ? -1 : 1;
  if (x->ref != y->ref) return x->ref < y->ref ? -1 : 1;
  if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
  return 0;
}

/* first index whose seed is >= v */
static int64_t occ_lower(const oracle_occ_t *o, int64_t n, uint64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (o[mid].seed < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

int64_t oracle_find_cals(const uint8_t *ref_codes, const int64_t *ref_off, const int64_t *ref_len, int32_t n_refs,
                         const uint8_t *read_codes, const int64_t *read_off, const int32_t *read_len, int32_t n_reads,
                         int32_t seed_len, int32_t stride, int32_t max_cals_per_seed, int64_t *cal_ptr,
                         int64_t *cal_pos, int16_t *cal_ref, uint8_t *strand, int64_t capacity) {
  const int S = seed_len;
  int64_t n_occ = 0;
  for (int k = 0; k < n_refs; ++k)
    if (ref_len[k] >= S) n_occ += ref_len[k] - S + 1;
  oracle_occ_t *occ = (oracle_occ_t *)malloc((size_t)(n_occ > 0 ? n_occ : 1) * sizeof(oracle_occ_t));
  int64_t m = 0;
  for (int k = 0; k < n_refs; ++k)
    for (int64_t x = 0; x + S <= ref_len[k]; ++x) {
      occ[m].seed = seed_at(ref_codes + ref_off[k] + x, S);
      occ[m].ref = k;
      occ[m].pos = x;
      ++m;
    }
  qsort(occ, (size_t)n_occ, sizeof(oracle_occ_t), occ_cmp);
  int64_t n = 0;
  cal_ptr[0] = 0;
  for (int64_t r = 0; r < n_reads; ++r) {
    const int64_t L = read_len[r];
    for (int64_t o = 0; o + S <= L; o += stride) {
      const uint64_t s = seed_at(read_codes + read_off[r] + o, S);
      const uint64_t rs = seed_revcomp(s, S);
      const int64_t f0 = occ_lower(occ, n_occ, s), f1 = occ_lower(occ, n_occ, s + 1);
      const int64_t r0 = occ_lower(occ, n_occ, rs), r1 = occ_lower(occ, n_occ, rs + 1);
      const int64_t total = (f1 - f0) + (r1 - r0); /* a palindrome counts twice */
      if (total == 0 || (max_cals_per_seed > 0 && total > max_cals_per_seed)) continue;
      int64_t i = f0, j = r0;
      while (i < f1 || j < r1) {
        /* next match in (reference, position) order; the forward one first on a tie */
        int take_fwd;
        if (i >= f1) take_fwd = 0;
        else if (j >= r1) take_fwd = 1;
        else take_fwd = (occ[i].ref < occ[j].ref || (occ[i].ref == occ[j].ref && occ[i].pos <= occ[j].pos));
        const oracle_occ_t *h = take_fwd ? &occ[i++] : &occ[j++];
        int64_t p = take_fwd ? h->pos - o : h->pos - (L - o - S);
        if (p < 0) p = 0;
        if (p >= ref_len[h->ref]) p = ref_len[h->ref] - 1;
        if (n < capacity) {
          cal_pos[n] = p;
          cal_ref[n] = (int16_t)h->ref;
          strand[n] = take_fwd ? 1 : 2;
        }
        ++n;
      }
    }
    cal_ptr[r + 1] = n;
  }
  free(occ);
  return n;
}
