// CPU stand-ins for the library calls that the served path makes besides its
// own gather/scatter kernels: the scoring entry points run stub_slot on the
// step batch they are given (reading the packed words through the step's word
// offsets, as the kernels do), the reduction is the Score Tracker definition,
// and the validation helpers keep only what the server relies on.  Like the
// library calls, the stand-ins only queue their work on the caller's stream;
// the stream's worker runs it later, so every buffer they touch must still be
// live and hold the step's data when the worker gets there.
// TEST INFRASTRUCTURE ONLY.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <functional>
#include <vector>

#include "../../include/sw_align.h"
#include "../../paper_1805_00106_amd/csrc/sw_api_internal.h"
#include "stub_score.h"

std::atomic<long> g_plain_calls{0}, g_ctx_calls{0};

namespace swapi {
thread_local int g_last_hip = 0;
int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return SW_ERR_HIP;
}
int validate_scoring(const sw_scoring_t *sc, ScoreMode *mode) {
  if (!sc) return SW_ERR_INVALID_ARG;
  mode->max_read_len = sc->max_read_len ? sc->max_read_len : SW_MAX_READ_LEN;
  mode->int16 = sc->precision == SW_PREC_INT16;
  mode->wcap = mode->max_read_len + 2 * sc->band;
  return SW_OK;
}
int validate_refs(const sw_refset_t *refs, int64_t, swk::RefTable *T) {
  if (!refs || refs->n_refs < 1 || refs->n_refs > SW_MAX_REFS) return SW_ERR_INVALID_ARG;
  for (int i = 0; i < refs->n_refs; ++i) {
    T->word_off[i] = refs->word_offset[i];
    T->len[i] = refs->length[i];
  }
  return SW_OK;
}
int device_cus() { return 4; }
}  // namespace swapi

static void reduce_step(const int64_t *cal_ptr, const int16_t *cal_ref, int32_t n_reads, int32_t n_refs,
                        const int32_t *score, int32_t *best_score, int64_t *best_slot, int32_t *n_tied);

static int score_step(const uint32_t *words, const int64_t *word_off, const int32_t *read_len, int32_t n_reads,
                      const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref, const uint8_t *strand,
                      int64_t n_cals, int32_t *score, int64_t *ref_end, int16_t *read_end) {
  if (cal_ptr[0] != 0 || cal_ptr[n_reads] != n_cals) return SW_ERR_INVALID_ARG;
  std::vector<uint8_t> codes;
  for (int32_t r = 0; r < n_reads; ++r) {
    const int L = read_len[r];
    codes.resize((size_t)L);
    for (int i = 0; i < L; ++i) codes[i] = (uint8_t)((words[word_off[r] + i / 16] >> (2 * (i % 16))) & 3u);
    const uint64_t rh = stub_read_hash(codes.data(), L);
    if (cal_ptr[r + 1] < cal_ptr[r]) return SW_ERR_INVALID_ARG;
    for (int64_t c = cal_ptr[r]; c < cal_ptr[r + 1]; ++c)
      for (int h = 0; h < 2; ++h)
        stub_slot(rh, L, cal_pos[c], cal_ref[c], strand[c], h, &score[2 * c + h], &ref_end[2 * c + h],
                  &read_end[2 * c + h]);
  }
  return SW_OK;
}

extern "C" {

// A context keeps its capacity, and a call beyond it fails as the library's does.
struct StubCtx {
  int64_t max_reads, max_cals;
};

int sw_ctx_create(const sw_ctx_opts_t *o, sw_ctx_t **out) {
  *out = reinterpret_cast<sw_ctx_t *>(new StubCtx{o->max_reads, o->max_cals});
  return SW_OK;
}
int sw_ctx_destroy(sw_ctx_t *c) {
  delete reinterpret_cast<StubCtx *>(c);
  return SW_OK;
}
// The plain call's workspace grows with the CAL count, as the library's does; the
// queued stand-in writes all of it, so a short or freed workspace is reported.
size_t sw_workspace_bytes(int32_t, int64_t n_cals, const sw_scoring_t *) {
  return 256 + (size_t)std::max<int64_t>(n_cals, 0) * 4;
}

static void queue_on(sw_stream_t stream, std::function<void()> op) {
  fakehip::as_stream((void *)stream)->push(std::move(op));
}

static int queue_score(const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                       int32_t n_reads, const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref,
                       const uint8_t *strand, int64_t n_cals, int32_t *score, int64_t *ref_end, int16_t *read_end,
                       sw_stream_t stream) {
  if (n_reads < 0 || n_cals < 0 || !cal_ptr) return SW_ERR_INVALID_ARG;
  if (n_cals == 0) return SW_OK;
  queue_on(stream, [=] {
    if (score_step(reads2bit, read_word_off, read_len, n_reads, cal_ptr, cal_pos, cal_ref, strand, n_cals, score,
                   ref_end, read_end) != SW_OK)
      fakehip::die("scoring stand-in: malformed step (CSR row pointer)");
  });
  return SW_OK;
}

int sw_align_batch(const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len, int32_t n_reads,
                   const sw_refset_t *, const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref,
                   const uint8_t *strand, int64_t n_cals, const sw_scoring_t *, int32_t *score, int64_t *ref_end,
                   int16_t *read_end, void *ws, size_t ws_bytes, sw_stream_t stream) {
  g_plain_calls++;
  const size_t need = sw_workspace_bytes(n_reads, n_cals, nullptr);
  if (n_cals > 0 && (!ws || ws_bytes < need)) return SW_ERR_WORKSPACE;
  if (n_cals > 0) queue_on(stream, [=] { memset(ws, 0x5A, need); });
  return queue_score(reads2bit, read_word_off, read_len, n_reads, cal_ptr, cal_pos, cal_ref, strand, n_cals, score,
                     ref_end, read_end, stream);
}

int sw_align_batch_ctx(sw_ctx_t *ctx, const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                       int32_t n_reads, const sw_refset_t *, const int64_t *cal_ptr, const int64_t *cal_pos,
                       const int16_t *cal_ref, const uint8_t *strand, int64_t n_cals, const sw_scoring_t *,
                       int32_t *score, int64_t *ref_end, int16_t *read_end, sw_stream_t stream) {
  g_ctx_calls++;
  const StubCtx *c = reinterpret_cast<const StubCtx *>(ctx);
  if (n_reads > c->max_reads || n_cals > c->max_cals) return SW_ERR_WORKSPACE;
  return queue_score(reads2bit, read_word_off, read_len, n_reads, cal_ptr, cal_pos, cal_ref, strand, n_cals, score,
                     ref_end, read_end, stream);
}

// Score Tracker: per (read, reference) the best score, its lowest slot, and the
// number of slots holding it; -1/-1/0 without a scored slot.
int sw_reduce_best(const int64_t *cal_ptr, const int16_t *cal_ref, int32_t n_reads, int32_t n_refs, int64_t,
                   const int32_t *score, int32_t *best_score, int64_t *best_slot, int32_t *n_tied,
                   sw_stream_t stream) {
  if (n_reads < 0 || n_refs < 1) return SW_ERR_INVALID_ARG;
  queue_on(stream, [=] { reduce_step(cal_ptr, cal_ref, n_reads, n_refs, score, best_score, best_slot, n_tied); });
  return SW_OK;
}

}  // extern "C"

static void reduce_step(const int64_t *cal_ptr, const int16_t *cal_ref, int32_t n_reads, int32_t n_refs,
                        const int32_t *score, int32_t *best_score, int64_t *best_slot, int32_t *n_tied) {
  for (int32_t r = 0; r < n_reads; ++r)
    for (int k = 0; k < n_refs; ++k) {
      int32_t b = -1, nt = 0;
      int64_t sl = -1;
      for (int64_t c = cal_ptr[r]; c < cal_ptr[r + 1]; ++c) {
        if (cal_ref[c] != k) continue;
        for (int h = 0; h < 2; ++h) {
          const int32_t s = score[2 * c + h];
          if (s < 0) continue;
          if (s > b) {
            b = s;
            sl = 2 * c + h;
            nt = 1;
          } else if (s == b) {
            ++nt;
          }
        }
      }
      best_score[(int64_t)r * n_refs + k] = b;
      best_slot[(int64_t)r * n_refs + k] = sl;
      n_tied[(int64_t)r * n_refs + k] = nt;
    }
}
