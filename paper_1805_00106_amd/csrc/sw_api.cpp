// C ABI of the library: argument validation, launch planning and the plain
// (one launch per batch) scoring path.  Declarations and contracts are in
// include/sw_align.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "../../include/sw_align.h"
#include "sw_api_internal.h"
#include "sw_filter.h"
#include "sw_launch.h"
#include "sw_trace.h"

namespace swk {
hipError_t measure_alu_peak(int bits, int64_t iters, int blocks, uint32_t *out, hipStream_t st, double *ops_per_s);
hipError_t check_half_max(int64_t *n_bad, hipStream_t st);
}

namespace swapi {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return SW_ERR_HIP;
}

int validate_scoring(const sw_scoring_t *sc, ScoreMode *mode) {
  if (!sc) return SW_ERR_INVALID_ARG;
  if (sc->precision < SW_PREC_AUTO || sc->precision > SW_PREC_INT32) return SW_ERR_INVALID_ARG;
  if (sc->kernel < SW_KERNEL_AUTO || sc->kernel > SW_KERNEL_INTRA) return SW_ERR_INVALID_ARG;
  if (sc->mode != SW_MODE_LOCAL && sc->mode != SW_MODE_FINAL_ROW) return SW_ERR_INVALID_ARG;
  if (sc->match < 1 || sc->mismatch > 0 || sc->gap_open < 0 || sc->gap_extend < 1) return SW_ERR_SCORING;
  if (sc->band < 0 || sc->band > SW_MAX_BAND) return SW_ERR_SCORING;
  int mrl = sc->max_read_len == 0 ? SW_MAX_READ_LEN : sc->max_read_len;
  if (mrl < 1) return SW_ERR_INVALID_ARG;
  if (mrl > SW_MAX_READ_LEN) return SW_ERR_READ_TOO_LONG;
  const int64_t goe2 = (int64_t)sc->gap_open + 2 * (int64_t)sc->gap_extend;
  // int32 path: values are V * 4096 + tag with |V| < 2^19, plus the row offsets
  // of the one-CAL-per-lane sweep (up to 49 * gap_extend)
  const int64_t top = (int64_t)sc->match * mrl;
  if (top + 49 * (int64_t)sc->gap_extend > (1 << 19) - 2 || -(int64_t)sc->mismatch > (1 << 18) ||
      goe2 > (1 << 18))
    return SW_ERR_SCORING;
  // int16 path: biased values with K tag bits and per-row offsets (DpConst) in
  // int16; the bound needs V <= 510 everywhere and a tag width that holds them
  int32_t kb = 0, beta = 0;
  const bool fits16 = top <= 510 && sc->mismatch >= -511 && goe2 <= 511 && int16_layout(sc, &kb, &beta);
  bool int16;
  if (sc->precision == SW_PREC_INT16) {
    if (!fits16) return SW_ERR_BOUND;
    int16 = true;
  } else if (sc->precision == SW_PREC_INT32) {
    int16 = false;
  } else {
    int16 = fits16;
  }
  mode->int16 = int16;
  mode->max_read_len = mrl;
  mode->wcap = mrl + 2 * sc->band;
  return SW_OK;
}

// The int16 layout of the scoring for its read-length bound (see DpConst).
static int int16_layout_for(const sw_scoring_t *sc, swk::DpConst *k) {
  k->match = sc->match;
  k->mismatch = sc->mismatch;
  k->goe = sc->gap_open + sc->gap_extend;
  k->ge = sc->gap_extend;
  const int64_t mrl = sc->max_read_len == 0 ? SW_MAX_READ_LEN : sc->max_read_len;
  return swk::set_int16_layout(*k, (int64_t)sc->match * mrl);
}

int int16_layout(const sw_scoring_t *sc, int32_t *kbits, int32_t *beta) {
  swk::DpConst k{};
  if (!int16_layout_for(sc, &k)) return 0;
  *kbits = k.kbits16;
  *beta = k.beta16;
  return 1;
}

DpConstHost make_consts(const sw_scoring_t *sc) {
  swk::DpConst k{};
  const int32_t goe = sc->gap_open + sc->gap_extend, ge = sc->gap_extend;
  // int16 pairs: the widest tag (K) whose biased values stay below 0x7C00 (the
  // scoring kernels may widen it per tile)
  int16_layout_for(sc, &k);
  k.goe_e32 = goe * 4096 + 1;
  k.ge_e32 = ge * 4096 + 1;
  k.goe_f32 = goe * 4096;
  k.ge_f32 = ge * 4096;
  k.sm32 = sc->match * 4096 - 1;
  k.sx32 = sc->mismatch * 4096 - 1;
  // the one-CAL-per-lane int32 sweep adds the row step gap_extend * 4096 to every
  // diagonal move: its byte tables hold (s + gap_extend) * 4096 - 1
  k.perm32 = sc->match + ge <= 16 && sc->mismatch + ge >= -15 ? 1 : 0;
  if (k.perm32) {
    const uint32_t smr = (uint32_t)(k.sm32 + k.ge_f32), sxr = (uint32_t)(k.sx32 + k.ge_f32);
    const uint32_t m1 = (smr >> 8) & 0xFFu, x1 = (sxr >> 8) & 0xFFu;
    const uint32_t m2 = (smr >> 16) & 0xFFu, x2 = (sxr >> 16) & 0xFFu;
    k.xlo32 = x1 * 0x01010101u;
    k.dlo32 = x1 ^ m1;
    k.xhi32 = x2 * 0x01010101u;
    k.dhi32 = x2 ^ m2;
  }
  k.e0_32 = 0;
  k.final_row = sc->mode == SW_MODE_FINAL_ROW ? 1 : 0;
  return k;
}

static int strip_candidates16[] = {
#define SW_LIST(RR) RR,
    SW_INTER16_STRIPS(SW_LIST)
#undef SW_LIST
};
static int strip_candidates32[] = {
#define SW_LIST(RR) RR,
    SW_INTER32_STRIPS(SW_LIST)
#undef SW_LIST
};

int choose_strip_rows(bool int16, int rows) {
  const int *cand = int16 ? strip_candidates16 : strip_candidates32;
  const int n = int16 ? (int)(sizeof(strip_candidates16) / sizeof(int))
                      : (int)(sizeof(strip_candidates32) / sizeof(int));
  int best = cand[0];
  int64_t best_cost = INT64_MAX;
  for (int i = 0; i < n; ++i) {
    const int R = cand[i];
    const int64_t cost = (int64_t)((rows + R - 1) / R) * R;
    if (cost < best_cost || (cost == best_cost && R > best)) {
      best_cost = cost;
      best = R;
    }
  }
  return best;
}

int strip_rows_supported(bool int16, int R) {
  const int *cand = int16 ? strip_candidates16 : strip_candidates32;
  const int n = int16 ? (int)(sizeof(strip_candidates16) / sizeof(int))
                      : (int)(sizeof(strip_candidates32) / sizeof(int));
  for (int i = 0; i < n; ++i)
    if (cand[i] == R) return 1;
  return 0;
}

static std::mutex g_occ_mu;
static int g_occ[64][2][1100];
static int g_cus[64];

int device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> lk(g_occ_mu);
  if (!g_cus[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    g_cus[dev] = n;
  }
  return g_cus[dev];
}

int blocks_per_cu(bool int16, int R) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || R <= 0 || R >= 1100) return 8;
  std::lock_guard<std::mutex> lk(g_occ_mu);
  int &v = g_occ[dev][int16 ? 1 : 0][R];
  if (!v) {
    int n = swk::inter_blocks_per_cu(int16, R);
    v = n > 0 ? n : 8;
  }
  return v;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int make_plan(int64_t n_cals, const sw_scoring_t *sc, int strip_override, PlainPlan *p) {
  ScoreMode m;
  int rc = validate_scoring(sc, &m);
  if (rc) return rc;
  // Kernel family: the intra-task kernel (one wavefront per task, lanes =
  // window columns) has the lowest latency per task and wins while the batch is
  // too small to give the SIMDs more than one inter-task tile each.  Its
  // wavefronts hold one CAL (both strands) in int16 pairs and one (CAL, strand)
  // in int32.  Measured on 100-bp reads with 7 CALs each (band 32, 256 CUs), one
  // wavefront per task is faster up to about 16 K CALs in int16 (13.9 K: 301 us
  // against 358 us) and about 8 K CALs in int32 (7.0 K: 353 us against 432 us),
  // so AUTO takes it up to 64 wavefronts per CU.
  const int cus = device_cus();
  bool intra = sc->kernel == SW_KERNEL_INTRA;
  const int64_t intra_waves = m.int16 ? n_cals : 2 * n_cals;
  if (sc->kernel == SW_KERNEL_AUTO) intra = intra_waves <= kIntraWavesPerCu * (int64_t)cus;
  p->intra = intra;
  p->mode = m;
  p->wwords = (m.wcap + 15) / 16;
  p->rwords = (m.max_read_len + 15) / 16;
  p->cal_read_off = 0;
  p->scratch_off = align_up((size_t)std::max<int64_t>(n_cals, 1) * sizeof(int32_t), 256);
  if (intra) {
    p->strip_rows = 0;
    p->n_tasks = intra_waves;
    const size_t lds = (size_t)m.max_read_len * 16 + (size_t)p->wwords * 4;
    int occ = swk::intra_blocks_per_cu(m.int16, lds);
    if (occ <= 0) occ = 8;
    p->grid = (int)std::max<int64_t>(1, std::min<int64_t>(p->n_tasks, (int64_t)cus * occ));
    p->bytes = p->scratch_off;
    return SW_OK;
  }
  p->strip_rows = strip_override > 0 ? strip_override
                                     : choose_strip_rows(m.int16, m.max_read_len);
  if (!strip_rows_supported(m.int16, p->strip_rows)) return SW_ERR_INVALID_ARG;
  p->n_tasks = m.int16 ? n_cals : 2 * n_cals;
  const int64_t n_tiles = (p->n_tasks + 63) / 64;
  const int64_t resident = (int64_t)cus * blocks_per_cu(m.int16, p->strip_rows);
  p->grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_tiles, resident));
  p->queue_off = p->scratch_off + (size_t)p->grid * (size_t)m.wcap * 64 * sizeof(uint2);
  p->bytes = p->queue_off + 256;
  return SW_OK;
}

int validate_refs(const sw_refset_t *refs, int64_t n_cals, swk::RefTable *T) {
  if (!refs) return SW_ERR_INVALID_ARG;
  if (refs->n_refs < 1) return SW_ERR_INVALID_ARG;
  if (refs->n_refs > SW_MAX_REFS) return SW_ERR_TOO_MANY_REFS;
  if (!refs->word_offset || !refs->length) return SW_ERR_INVALID_ARG;
  if (n_cals > 0 && !refs->words) return SW_ERR_INVALID_ARG;
  std::memset(T, 0, sizeof(*T));
  for (int i = 0; i < refs->n_refs; ++i) {
    if (refs->length[i] < 1 || refs->word_offset[i] < 0) return SW_ERR_INVALID_ARG;
    T->word_off[i] = refs->word_offset[i];
    T->len[i] = refs->length[i];
  }
  return SW_OK;
}

int validate_batch(const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                   int32_t n_reads, const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref,
                   const uint8_t *strand, int64_t n_cals, int32_t *score, int64_t *ref_end,
                   int16_t *read_end) {
  if (n_reads < 0 || n_cals < 0) return SW_ERR_INVALID_ARG;
  if (!cal_ptr) return SW_ERR_INVALID_ARG;
  if (n_reads > 0 && (!reads2bit || !read_word_off || !read_len)) return SW_ERR_INVALID_ARG;
  if (n_cals > 0 && (!cal_pos || !cal_ref || !strand || !score || !ref_end || !read_end))
    return SW_ERR_INVALID_ARG;
  return SW_OK;
}

int run_plain(const PlainPlan &plan, const swk::RefTable &T, const uint32_t *reads2bit,
              const int64_t *read_word_off, const int32_t *read_len, int32_t n_reads, const sw_refset_t *refs,
              const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref, const uint8_t *strand,
              int64_t n_cals, const sw_scoring_t *sc, int32_t *score, int64_t *ref_end, int16_t *read_end,
              void *workspace, unsigned long long *err, hipStream_t st) {
  char *ws = (char *)workspace;
  int32_t *cal_read = (int32_t *)(ws + plan.cal_read_off);
  hipError_t e = swk::launch_expand(cal_ptr, n_reads, n_cals, cal_read, st);
  if (e != hipSuccess) return hip_fail(e);
  swk::AlignArgs A{};
  A.reads = reads2bit;
  A.read_word_off = read_word_off;
  A.read_len = read_len;
  A.n_reads = n_reads;
  A.n_refs = refs->n_refs;
  A.ref_words = refs->words;
  A.cal_pos = cal_pos;
  A.cal_ref = cal_ref;
  A.strand = strand;
  A.cal_read = cal_read;
  A.order = nullptr;
  A.n_cals = n_cals;
  A.n_tasks = plan.n_tasks;
  A.score = score;
  A.ref_end = ref_end;
  A.read_end = read_end;
  A.scratch = (uint2 *)(ws + plan.scratch_off);
  A.err = err;
  A.wcap = plan.mode.wcap;
  A.wwords = plan.wwords;
  A.rwords = plan.rwords;
  A.max_read_len = plan.mode.max_read_len;
  A.band = sc->band;
  A.strip_rows = plan.strip_rows;
  A.k = make_consts(sc);
  if (!plan.intra) {
    // tiles are popped from a counter rather than dealt by block index, so that a
    // block that finishes early takes the next tile (cleared by a kernel, not a
    // memset, so that a caller may capture the call in a graph)
    A.queue = (int32_t *)(ws + plan.queue_off);
    e = swk::launch_fill_i32(A.queue, 1, 0, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  e = plan.intra ? swk::launch_intra(plan.mode.int16, A, T, plan.grid, st)
                 : swk::launch_inter(plan.mode.int16, A, T, plan.grid, st);
  if (e != hipSuccess) return hip_fail(e);
  return SW_OK;
}

}  // namespace swapi

using namespace swapi;

extern "C" {

const char *sw_strerror(int code) {
  switch (code) {
    case SW_OK: return "ok";
    case SW_ERR_INVALID_ARG: return "invalid argument";
    case SW_ERR_SCORING: return "scoring parameters out of the supported range";
    case SW_ERR_READ_TOO_LONG: return "maximum read length above SW_MAX_READ_LEN";
    case SW_ERR_BOUND: return "int16 precision requested but the score bound does not hold";
    case SW_ERR_WORKSPACE: return "workspace missing or too small";
    case SW_ERR_NOMEM: return "out of memory";
    case SW_ERR_HIP: return "HIP runtime error";
    case SW_ERR_TOO_MANY_REFS: return "more than SW_MAX_REFS references";
    case SW_ERR_REJECTED: return "request larger than the memory budget";
    case SW_ERR_STATE: return "object in the wrong state";
    default: return "unknown error";
  }
}

int sw_last_hip_error(void) { return g_last_hip; }

const char *sw_version(void) { return "swalign-gfx950 0.1"; }

int sw_pack_2bit(const uint8_t *codes, int64_t n, uint32_t *words, sw_stream_t stream) {
  if (n < 0) return SW_ERR_INVALID_ARG;
  if (n == 0) return SW_OK;
  if (!codes || !words) return SW_ERR_INVALID_ARG;
  hipError_t e = swk::launch_pack(codes, n, words, (hipStream_t)stream);
  return e == hipSuccess ? SW_OK : hip_fail(e);
}

size_t sw_workspace_bytes(int32_t n_reads, int64_t n_cals, const sw_scoring_t *sc) {
  (void)n_reads;
  if (n_cals < 0) return 0;
  PlainPlan p;
  if (make_plan(n_cals, sc, 0, &p) != SW_OK) return 0;
  return p.bytes;
}

int sw_align_batch(const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                   int32_t n_reads, const sw_refset_t *refs, const int64_t *cal_ptr, const int64_t *cal_pos,
                   const int16_t *cal_ref, const uint8_t *strand, int64_t n_cals, const sw_scoring_t *sc,
                   int32_t *score, int64_t *ref_end, int16_t *read_end, void *workspace,
                   size_t workspace_bytes, sw_stream_t stream) {
  ScoreMode m;
  int rc = validate_scoring(sc, &m);
  if (rc) return rc;
  rc = validate_batch(reads2bit, read_word_off, read_len, n_reads, cal_ptr, cal_pos, cal_ref, strand, n_cals,
                      score, ref_end, read_end);
  if (rc) return rc;
  swk::RefTable T;
  rc = validate_refs(refs, n_cals, &T);
  if (rc) return rc;
  if (n_cals == 0) return SW_OK;
  if (!workspace) return SW_ERR_WORKSPACE;
  PlainPlan plan;
  rc = make_plan(n_cals, sc, 0, &plan);
  if (rc) return rc;
  if (workspace_bytes < plan.bytes) return SW_ERR_WORKSPACE;
  unsigned long long *err = swk::error_counter();
  if (!err) return hip_fail(hipErrorInvalidDevice);
  return run_plain(plan, T, reads2bit, read_word_off, read_len, n_reads, refs, cal_ptr, cal_pos, cal_ref, strand,
                   n_cals, sc, score, ref_end, read_end, workspace, err, (hipStream_t)stream);
}

// The scratch of sw_align_batch_noalloc: a file-scope device array that the
// code object loads once per device (held until the process ends).  In host
// code its name is only a stand-in for the symbol; the device address comes
// from hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[SW_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[64];

int noalloc_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= 64) return SW_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (!p) return hip_fail(hipErrorInvalidSymbol);
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return SW_OK;
}
}  // namespace

int sw_align_batch_noalloc(const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                           int32_t n_reads, const sw_refset_t *refs, const int64_t *cal_ptr, const int64_t *cal_pos,
                           const int16_t *cal_ref, const uint8_t *strand, int64_t n_cals, const sw_scoring_t *sc,
                           int32_t *score, int64_t *ref_end, int16_t *read_end, sw_stream_t stream) {
  ScoreMode m;
  int rc = validate_scoring(sc, &m);
  if (rc) return rc;
  rc = validate_batch(reads2bit, read_word_off, read_len, n_reads, cal_ptr, cal_pos, cal_ref, strand, n_cals,
                      score, ref_end, read_end);
  if (rc) return rc;
  swk::RefTable T;
  rc = validate_refs(refs, n_cals, &T);
  if (rc) return rc;
  if (n_cals == 0) return SW_OK;
  PlainPlan plan;
  rc = make_plan(n_cals, sc, 0, &plan);
  if (rc) return rc;
  // the plan's owner-read array, strip scratch and tile counter must fit the static array
  if (plan.bytes > (size_t)SW_NOALLOC_SCRATCH_BYTES) return SW_ERR_WORKSPACE;
  void *ws = nullptr;
  rc = noalloc_scratch(&ws);
  if (rc) return rc;
  unsigned long long *err = swk::error_counter();
  if (!err) return hip_fail(hipErrorInvalidDevice);
  // nothing in the scratch has to start at zero: the owner-read array is filled
  // by the expansion kernels and each strip row is written before it is read
  return run_plain(plan, T, reads2bit, read_word_off, read_len, n_reads, refs, cal_ptr, cal_pos, cal_ref, strand,
                   n_cals, sc, score, ref_end, read_end, ws, err, (hipStream_t)stream);
}

int sw_error_count(int64_t *n_invalid, int reset) {
  if (!n_invalid) return SW_ERR_INVALID_ARG;
  unsigned long long *err = swk::error_counter();
  if (!err) return hip_fail(hipErrorInvalidDevice);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e);
  unsigned long long v = 0;
  e = hipMemcpy(&v, err, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e);
  *n_invalid = (int64_t)v;
  if (reset) {
    v = 0;
    e = hipMemcpy(err, &v, sizeof(v), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
  }
  return SW_OK;
}

int sw_reduce_best(const int64_t *cal_ptr, const int16_t *cal_ref, int32_t n_reads, int32_t n_refs, int64_t n_cals,
                   const int32_t *score, int32_t *best_score, int64_t *best_slot, int32_t *n_tied,
                   sw_stream_t stream) {
  if (n_reads < 0 || n_refs < 1 || n_cals < 0) return SW_ERR_INVALID_ARG;
  if (n_refs > SW_MAX_REFS) return SW_ERR_TOO_MANY_REFS;
  if (n_reads == 0) return SW_OK;
  if (!cal_ptr || !best_score || !best_slot || !n_tied) return SW_ERR_INVALID_ARG;
  if (n_cals > 0 && (!cal_ref || !score)) return SW_ERR_INVALID_ARG;
  hipError_t e = swk::launch_reduce(cal_ptr, cal_ref, n_reads, n_refs, n_cals, score, best_score, best_slot, n_tied,
                                    (hipStream_t)stream);
  return e == hipSuccess ? SW_OK : hip_fail(e);
}

namespace {

// Kernel family, grid and workspace of a traceback launch.  One slot per lane
// (64 per wavefront) unless its per-block bit buffer would exceed 4 MiB (very
// long reads or wide bands) or the caller asks for the wavefront-per-slot kernel.
constexpr size_t kTraceInterBlockLimit = 4u << 20;
// Two slots per lane: per-block buffers up to 8 MiB, and the grid trimmed so that
// all blocks' buffers stay within 4 GiB.
constexpr size_t kTracePairBlockLimit = 8u << 20;
constexpr size_t kTracePairWorkspace = (size_t)4 << 30;

struct TraceLaunch {
  bool inter;
  bool pair;         // two slots per lane in int16 halves (else one per lane, int32)
  int32_t beta;      // bias of the two-slots-per-lane kernel's values
  swk::TracePlan P;  // wavefront-per-slot kernel
  int grid;
  size_t block_bytes;     // slot-per-lane kernels: bits + boundary rows per block
  size_t cal_read_bytes;  // slot-per-lane kernels: owner read per CAL
  size_t bytes;           // total workspace
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

int trace_launch(int64_t n_slots, int64_t n_cals, const sw_scoring_t *sc, TraceLaunch *t) {
  ScoreMode m;
  int rc = validate_scoring(sc, &m);
  if (rc) return rc;
  const size_t bb = swk::trace_inter_block_bytes(m.max_read_len, m.wcap);
  const size_t bp = swk::trace_pair_block_bytes(m.max_read_len, m.wcap);
  t->beta = 0;
  const bool pair_fits = swk::trace_pair_fits(sc->match, sc->mismatch, sc->gap_open + sc->gap_extend, sc->gap_extend,
                                              m.max_read_len, m.wcap, &t->beta) != 0;
  t->pair = pair_fits && (sc->kernel == SW_KERNEL_INTER || (sc->kernel == SW_KERNEL_AUTO && bp <= kTracePairBlockLimit));
  t->inter = t->pair || sc->kernel == SW_KERNEL_INTER || (sc->kernel == SW_KERNEL_AUTO && bb <= kTraceInterBlockLimit);
  if (t->pair) {
    const int64_t tiles = (n_slots + 127) / 128;
    const int64_t resident = (int64_t)device_cus() * swk::trace_pair_blocks_per_cu(m.max_read_len);
    const int64_t budget = std::max<int64_t>(device_cus(), (int64_t)(kTracePairWorkspace / align256(bp)));
    t->grid = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(tiles, resident), budget));
    t->block_bytes = align256(bp);
    t->cal_read_bytes = align256(sizeof(int32_t) * (size_t)std::max<int64_t>(n_cals, 1));
    t->bytes = t->cal_read_bytes + (size_t)t->grid * t->block_bytes;
    return SW_OK;
  }
  if (t->inter) {
    const int64_t tiles = (n_slots + 63) / 64;
    const int64_t resident = (int64_t)device_cus() * swk::trace_inter_blocks_per_cu();
    t->grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, resident));
    t->block_bytes = align256(bb);
    t->cal_read_bytes = align256(sizeof(int32_t) * (size_t)std::max<int64_t>(n_cals, 1));
    t->bytes = t->cal_read_bytes + (size_t)t->grid * t->block_bytes;
    return SW_OK;
  }
  t->P = swk::trace_plan(m.max_read_len, m.wcap);
  const int64_t resident = (int64_t)device_cus() * swk::trace_blocks_per_cu(t->P);
  t->grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_slots, resident));
  t->bytes = t->P.lds_planes ? 0 : (size_t)t->grid * t->P.planes_bytes;
  return SW_OK;
}

}  // namespace

size_t sw_traceback_workspace_bytes(int64_t n_slots, int64_t n_cals, const sw_scoring_t *sc) {
  if (n_slots <= 0 || n_cals < 0) return 0;
  TraceLaunch t;
  if (trace_launch(n_slots, n_cals, sc, &t) != SW_OK) return 0;
  return t.bytes;
}

int sw_traceback(const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len, int32_t n_reads,
                 const sw_refset_t *refs, const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref,
                 int64_t n_cals, const sw_scoring_t *sc, const int32_t *score, const int64_t *ref_end,
                 const int16_t *read_end, const int64_t *slots, int64_t n_slots, int32_t cap, int64_t *ref_start,
                 int16_t *read_start, int32_t *n_ops, uint32_t *cigar, void *workspace, size_t workspace_bytes,
                 sw_stream_t stream) {
  ScoreMode m;
  int rc = validate_scoring(sc, &m);
  if (rc) return rc;
  if (n_reads < 0 || n_cals < 0 || n_slots < 0 || cap < 1) return SW_ERR_INVALID_ARG;
  swk::RefTable T;
  rc = validate_refs(refs, n_cals, &T);
  if (rc) return rc;
  if (n_slots == 0) return SW_OK;
  if (!reads2bit || !read_word_off || !read_len || !cal_ptr || !cal_pos || !cal_ref || !score || !ref_end ||
      !read_end || !slots || !ref_start || !read_start || !n_ops || !cigar)
    return SW_ERR_INVALID_ARG;
  TraceLaunch tl;
  rc = trace_launch(n_slots, n_cals, sc, &tl);
  if (rc) return rc;
  if (tl.bytes > 0 && (!workspace || workspace_bytes < tl.bytes)) return SW_ERR_WORKSPACE;
  unsigned long long *err = swk::error_counter();
  if (!err) return hip_fail(hipErrorInvalidDevice);
  swk::TraceArgs A{};
  A.reads = reads2bit;
  A.read_word_off = read_word_off;
  A.read_len = read_len;
  A.n_reads = n_reads;
  A.n_refs = refs->n_refs;
  A.ref_words = refs->words;
  A.cal_ptr = cal_ptr;
  A.cal_pos = cal_pos;
  A.cal_ref = cal_ref;
  A.n_cals = n_cals;
  A.score = score;
  A.ref_end = ref_end;
  A.read_end = read_end;
  A.slots = slots;
  A.n_slots = n_slots;
  A.cap = cap;
  A.ref_start = ref_start;
  A.read_start = read_start;
  A.n_ops = n_ops;
  A.cigar = cigar;
  A.planes_global = tl.P.lds_planes ? nullptr : static_cast<uint64_t *>(workspace);
  A.planes_stride = (int64_t)(tl.P.planes_bytes / 8);
  A.err = err;
  A.max_read_len = m.max_read_len;
  A.band = sc->band;
  A.match = sc->match;
  A.mismatch = sc->mismatch;
  A.goe = sc->gap_open + sc->gap_extend;
  A.ge = sc->gap_extend;
  A.q_bytes = tl.P.q_bytes;
  A.win_words = tl.P.win_words;
  A.run_cap = tl.P.run_cap;
  A.planes_lds_off = (int64_t)tl.P.planes_lds_off;
  hipError_t e;
  if (tl.inter) {
    swk::TraceInterArgs I{};
    I.a = A;
    I.a.planes_global = nullptr;
    int32_t *cal_read = static_cast<int32_t *>(workspace);
    I.cal_read = cal_read;
    I.bits = reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + tl.cal_read_bytes);
    // per block, one block_bytes slice: [bits | boundary rows]
    const size_t bits_bytes = (tl.pair ? swk::trace_pair_block_bytes(m.max_read_len, m.wcap)
                                       : swk::trace_inter_block_bytes(m.max_read_len, m.wcap)) -
                              (size_t)m.wcap * 64 * 8;
    I.bits_stride = (int64_t)(tl.block_bytes / 4);
    I.bscr = reinterpret_cast<uint2 *>(static_cast<char *>(workspace) + tl.cal_read_bytes + bits_bytes);
    I.bscr_stride = (int64_t)(tl.block_bytes / 8);
    I.wcap = m.wcap;
    I.rwords = (m.max_read_len + 15) / 16;
    I.wwords = (m.wcap + 15) / 16;
    I.beta = tl.beta;
    e = swk::launch_expand(cal_ptr, n_reads, n_cals, cal_read, (hipStream_t)stream);
    if (e == hipSuccess)
      e = tl.pair ? swk::launch_trace_pair(I, T, tl.grid, (hipStream_t)stream)
                  : swk::launch_trace_inter(I, T, tl.grid, (hipStream_t)stream);
  } else {
    e = swk::launch_trace(A, T, tl.P, tl.grid, (hipStream_t)stream);
  }
  return e == hipSuccess ? SW_OK : hip_fail(e);
}

size_t sw_cal_filter_workspace_bytes(int32_t n_reads) {
  if (n_reads < 0) return 0;
  return swk::filter_workspace_bytes(n_reads);
}

int sw_cal_filter(const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref, const uint8_t *strand,
                  int32_t n_reads, int64_t n_cals, int32_t bucket_bits, int64_t *out_ptr, int64_t *out_pos,
                  int16_t *out_ref, uint8_t *out_strand, int64_t *cal_map, void *workspace, size_t workspace_bytes,
                  sw_stream_t stream) {
  if (n_reads < 0 || n_cals < 0 || bucket_bits < 0 || bucket_bits > 40) return SW_ERR_INVALID_ARG;
  if (!cal_ptr || !out_ptr) return SW_ERR_INVALID_ARG;
  if (n_cals > 0 && (!cal_pos || !cal_ref || !strand || !out_pos || !out_ref || !out_strand || !cal_map))
    return SW_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < swk::filter_workspace_bytes(n_reads)) return SW_ERR_WORKSPACE;
  swk::FilterArgs A{cal_ptr, cal_pos, cal_ref, strand, n_reads, n_cals, bucket_bits,
                    out_ptr, out_pos, out_ref, out_strand, cal_map};
  hipError_t e = swk::launch_filter(A, workspace, workspace_bytes, (hipStream_t)stream);
  return e == hipSuccess ? SW_OK : hip_fail(e);
}

int sw_alu_peak(int32_t bits, int64_t iters, double *ops_per_s, sw_stream_t stream) {
  if ((bits != 16 && bits != 32) || iters < 16 || !ops_per_s) return SW_ERR_INVALID_ARG;
  const int blocks = 8 * device_cus();  // 8 waves of 64 lanes per SIMD pair: every SIMD kept issuing
  uint32_t *out = nullptr;
  if (hipMalloc(&out, sizeof(uint32_t) * 256 * (size_t)blocks) != hipSuccess) return SW_ERR_NOMEM;
  hipError_t e = swk::measure_alu_peak(bits, iters, blocks, out, (hipStream_t)stream, ops_per_s);
  hipFree(out);
  return e == hipSuccess ? SW_OK : hip_fail(e);
}

int sw_check_half_max(int64_t *n_bad, sw_stream_t stream) {
  if (!n_bad) return SW_ERR_INVALID_ARG;
  *n_bad = -1;
  hipError_t e = swk::check_half_max(n_bad, (hipStream_t)stream);
  return e == hipSuccess ? SW_OK : hip_fail(e);
}

int sw_topk(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, const int32_t *score, int32_t k,
            int32_t *top_score, int64_t *top_slot, sw_stream_t stream) {
  if (n_reads < 0 || n_cals < 0 || k < 1 || k > SW_MAX_TOPK) return SW_ERR_INVALID_ARG;
  if (n_reads == 0) return SW_OK;
  if (!cal_ptr || !top_score || !top_slot || (n_cals > 0 && !score)) return SW_ERR_INVALID_ARG;
  hipError_t e = swk::launch_topk(cal_ptr, n_reads, n_cals, score, k, top_score, top_slot, (hipStream_t)stream);
  return e == hipSuccess ? SW_OK : hip_fail(e);
}

int sw_tied_flags(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, const int32_t *score, uint8_t *flags,
                  sw_stream_t stream) {
  if (n_reads < 0 || n_cals < 0) return SW_ERR_INVALID_ARG;
  if (n_reads == 0) return SW_OK;
  if (!cal_ptr || (n_cals > 0 && (!score || !flags))) return SW_ERR_INVALID_ARG;
  hipError_t e = swk::launch_tied(cal_ptr, n_reads, n_cals, score, flags, (hipStream_t)stream);
  return e == hipSuccess ? SW_OK : hip_fail(e);
}

int sw_classify(const int32_t *best_score, int32_t n_reads, int32_t n_refs, int32_t threshold, int32_t *cls,
                sw_stream_t stream) {
  if (n_reads < 0 || n_refs < 1) return SW_ERR_INVALID_ARG;
  if (n_refs > SW_MAX_REFS) return SW_ERR_TOO_MANY_REFS;
  if (n_reads == 0) return SW_OK;
  if (!best_score || !cls) return SW_ERR_INVALID_ARG;
  hipError_t e = swk::launch_classify(best_score, n_reads, n_refs, threshold, cls, (hipStream_t)stream);
  return e == hipSuccess ? SW_OK : hip_fail(e);
}

}  // extern "C"
