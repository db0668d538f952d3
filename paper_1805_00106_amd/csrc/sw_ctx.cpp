// Batched execution context (placeholder until the binned persistent path lands).
#include "../../include/sw_align.h"

extern "C" {
int sw_ctx_create(const sw_ctx_opts_t *opts, sw_ctx_t **out) {
  (void)opts;
  if (out) *out = nullptr;
  return SW_ERR_STATE;
}
int sw_ctx_destroy(sw_ctx_t *ctx) { (void)ctx; return SW_OK; }
int sw_align_batch_ctx(sw_ctx_t *, const uint32_t *, const int64_t *, const int32_t *, int32_t,
                       const sw_refset_t *, const int64_t *, const int64_t *, const int16_t *, const uint8_t *,
                       int64_t, const sw_scoring_t *, int32_t *, int64_t *, int16_t *, sw_stream_t) {
  return SW_ERR_STATE;
}
int sw_ctx_error_count(sw_ctx_t *, int64_t *) { return SW_ERR_STATE; }
const char *sw_ctx_last_plan(sw_ctx_t *) { return ""; }
}
