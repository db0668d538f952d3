/*
 * sw_align.h - C ABI of the MI355X (gfx950) affine-gap Smith-Waterman CAL scorer.
 *
 * The library scores short reads against the reference window around each of
 * their candidate alignment locations (CALs), on one or both strands, and
 * reports the best local-alignment score and its end cell per (CAL, strand),
 * then the best per (read, reference).  This is the scoring stage of the
 * aligner described in McVicar et al., "FPGA Acceleration of Short Read
 * Alignment": reads with their CALs go to Smith-Waterman units under the affine
 * gap model (sections 3.5 and 4.2), each CAL carries a strand bit and the
 * reverse strand is aligned as the reverse complement (section 3.1), and a
 * Score Tracker keeps the best CAL per read (sections 3.6 and 4.2).
 *
 * Conventions shared by every entry point
 *   - Array arguments marked "device" are device pointers owned by the caller;
 *     arrays marked "host" are host pointers read before the call returns.  The
 *     library never frees or retains caller memory.
 *   - GPU work is enqueued on `stream` (0 = the null stream) and is
 *     asynchronous; outputs are valid once the stream reaches that point.
 *   - Host-visible arguments are validated before any HIP call; on a
 *     validation error nothing is enqueued.  Functions return SW_OK (0) or a
 *     negative SW_ERR_* code; sw_strerror() names it.  No C++ exception crosses
 *     the ABI.
 *   - Bases are 2-bit codes A=0, C=1, G=2, T=3 (the code of the paper's index
 *     figure, section 3.1, Fig. 3).  Packed sequences store base i of a
 *     sequence at bits [2*(i%16), 2*(i%16)+2) of 32-bit word i/16 (least
 *     significant first); every sequence starts on a word boundary.
 *
 * Scoring (affine gaps, section 3.5): a pair of equal bases scores `match`,
 * a pair of different bases `mismatch`, and a run of k consecutive read-only or
 * window-only columns costs gap_open + k*gap_extend.  The score of a task is
 * the maximum over all local alignments (the empty one scores 0).  Among the
 * cells reaching it the reported end is the smallest reference position, then
 * the smallest read position; a score of 0 reports both ends as -1.
 */
#ifndef SW_ALIGN_H
#define SW_ALIGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *sw_stream_t; /* a hipStream_t */

/* ------------------------------------------------------------------ codes */
#define SW_OK 0
#define SW_ERR_INVALID_ARG (-1)   /* null pointer, negative count, bad enum */
#define SW_ERR_SCORING (-2)       /* scoring parameters outside the supported range: match >= 1,
                                     mismatch <= 0, gap_open >= 0, gap_extend >= 1,
                                     match * max_read_len + 49 * gap_extend <= 2^19 - 2,
                                     -mismatch <= 2^18, gap_open + 2 * gap_extend <= 2^18 */
#define SW_ERR_READ_TOO_LONG (-3) /* max_read_len above SW_MAX_READ_LEN */
#define SW_ERR_BOUND (-4)         /* int16 requested but the score bound does not hold */
#define SW_ERR_WORKSPACE (-5)     /* workspace missing or smaller than sw_workspace_bytes() */
#define SW_ERR_NOMEM (-6)         /* device or host allocation failed */
#define SW_ERR_HIP (-7)           /* a HIP call failed; sw_last_hip_error() has the code */
#define SW_ERR_TOO_MANY_REFS (-8) /* more than SW_MAX_REFS references */
#define SW_ERR_REJECTED (-9)      /* served request larger than the memory budget */
#define SW_ERR_STATE (-10)        /* object used in the wrong state (e.g. no references set) */

#define SW_MAX_READ_LEN 1024 /* longest read accepted */
#define SW_MAX_REFS 64       /* references per reference set */
#define SW_MAX_BAND 1024     /* widest band accepted */

/* precision of the dynamic-programming values inside the kernels.  The int16
 * bound: match * max_read_len <= 510, mismatch >= -511, gap_open + 2 * gap_extend
 * <= 511, and some K in {6, 5, 4} with
 *   (beta + match * max_read_len + 1 + 49 * gap_extend) * 2^K <= 0x7BFF,
 *   beta = max(-mismatch, gap_open + gap_extend + 1, ceil(256 / 2^K) + gap_extend)
 * (the int16 sweep holds biased scores with K position bits, and offsets row r
 * of a strip of at most 50 rows by r * gap_extend).  At K = 4 and gap_extend <= 19
 * the first three conditions imply the fourth. */
#define SW_PREC_AUTO 0  /* int16 pairs when the bound holds, else int32 */
#define SW_PREC_INT16 1 /* error SW_ERR_BOUND if the bound does not hold */
#define SW_PREC_INT32 2

/* kernel family */
#define SW_KERNEL_AUTO 0  /* one wavefront per task for small batches (at most 64 wavefronts
                             per compute unit), one CAL per lane otherwise */
#define SW_KERNEL_INTER 1 /* one CAL per lane (int16: both strands in one lane; int32: one
                             strand per lane) */
#define SW_KERNEL_INTRA 2 /* one wavefront per task, lanes hold window columns (int16: one
                             CAL, both strands in the 16-bit halves; int32: one CAL strand) */

/* which cells may end an alignment */
#define SW_MODE_LOCAL 0     /* any cell: the full local maximum */
#define SW_MODE_FINAL_ROW 1 /* the last read row only: the best cell of the final row
                               of the matrix, so the alignment ends at the read's last
                               base (sections 3.5 and 3.6; read_end is then L-1) */

/* strand mask bits of a CAL (section 3.1: a strand bit is kept with each CAL) */
#define SW_STRAND_FWD 1
#define SW_STRAND_REV 2

typedef struct {
  int32_t match;        /* >= 1 */
  int32_t mismatch;     /* <= 0 */
  int32_t gap_open;     /* >= 0 */
  int32_t gap_extend;   /* >= 1 */
  int32_t band;         /* window = [p - band, p + L + band) clipped to the reference; 0..SW_MAX_BAND */
  int32_t precision;    /* SW_PREC_* */
  int32_t kernel;       /* SW_KERNEL_* */
  int32_t max_read_len; /* upper bound on every read length of the call, 1..SW_MAX_READ_LEN
                           (0 means SW_MAX_READ_LEN); reads above it are flagged as errors */
  int32_t mode;         /* SW_MODE_*; 0 (zero-initialised) is SW_MODE_LOCAL */
} sw_scoring_t;

/* References resident in device memory (the paper keeps the whole 2-bit
 * reference in accelerator memory, sections 4.3 and 5.1). */
typedef struct {
  const uint32_t *words;       /* device: all references packed back to back */
  const int64_t *word_offset;  /* host [n_refs]: first word of each reference */
  const int64_t *length;       /* host [n_refs]: length in bases (>= 1) */
  int32_t n_refs;              /* 1..SW_MAX_REFS */
} sw_refset_t;

/* ------------------------------------------------------------------ packing */
/*
 * Pack `n` base codes (device uint8, values 0..3; only the low 2 bits are
 * used) into ceil(n/16) words (device uint32).  Packing each sequence at a
 * 16-aligned code offset gives word-aligned sequences (section 3.7: 0.25
 * bytes per base).
 */
int sw_pack_2bit(const uint8_t *codes, int64_t n, uint32_t *words, sw_stream_t stream);

/* ------------------------------------------------------------------ scoring */
/*
 * Score every requested (CAL, strand) task.
 *   reads2bit      device: packed reads
 *   read_word_off  device [n_reads]: first word of each read
 *   read_len       device [n_reads]: length in bases, 1..max_read_len
 *   cal_ptr        device [n_reads+1]: CSR row pointer, cal_ptr[0] = 0,
 *                  cal_ptr[n_reads] = n_cals; CALs of read r are
 *                  [cal_ptr[r], cal_ptr[r+1])
 *   cal_pos        device [n_cals]: forward reference position of base 0 of the
 *                  oriented read (the CAL), 0 <= p < reference length
 *   cal_ref        device [n_cals]: reference id
 *   strand         device [n_cals]: mask of SW_STRAND_FWD | SW_STRAND_REV
 * Outputs, device [2*n_cals], slot 2c = forward, 2c+1 = reverse:
 *   score          best score; -1 if the strand was not requested; INT32_MIN if
 *                  the task is invalid (reference id, position or read length
 *                  out of range, or CAL not covered by cal_ptr)
 *   ref_end        absolute forward reference position of the end cell, -1 if
 *                  score <= 0
 *   read_end       position in the oriented read (reverse strand = reverse
 *                  complement of the read), -1 if score <= 0
 * The reverse strand aligns the reverse complement of the read against the same
 * forward window (section 3.1).  `workspace` (device, >= workspace_bytes) must
 * hold sw_workspace_bytes(n_reads, n_cals, sc) bytes and must not be used by
 * another call that overlaps on the device.  The number of invalid tasks is
 * added to the counter read by sw_error_count().
 */
int sw_align_batch(const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                   int32_t n_reads, const sw_refset_t *refs, const int64_t *cal_ptr,
                   const int64_t *cal_pos, const int16_t *cal_ref, const uint8_t *strand,
                   int64_t n_cals, const sw_scoring_t *sc, int32_t *score, int64_t *ref_end,
                   int16_t *read_end, void *workspace, size_t workspace_bytes, sw_stream_t stream);

/*
 * sw_align_batch without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The same kernels and
 * outputs as sw_align_batch; its scratch (the owner-read array, the strip
 * scratch and a tile counter, sw_workspace_bytes(n_reads, n_cals, sc) bytes) lives in one static
 * device array of SW_NOALLOC_SCRATCH_BYTES per device, which the library holds
 * from load until the process ends.  A call whose scratch would exceed it
 * returns SW_ERR_WORKSPACE.  Every call on a device shares that device's array:
 * calls that overlap on one device (other streams, other host threads) race and
 * must be serialised by the caller.  The first call on a device looks up the
 * array's device address (no allocation).  Each call clears the tile counter
 * itself, with a fill kernel on `stream` (not a memset); nothing else in the
 * array needs clearing.
 */
#define SW_NOALLOC_SCRATCH_BYTES (128u << 20)
int sw_align_batch_noalloc(const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                           int32_t n_reads, const sw_refset_t *refs, const int64_t *cal_ptr,
                           const int64_t *cal_pos, const int16_t *cal_ref, const uint8_t *strand,
                           int64_t n_cals, const sw_scoring_t *sc, int32_t *score, int64_t *ref_end,
                           int16_t *read_end, sw_stream_t stream);

/* Workspace size for sw_align_batch (0 is never returned for n_cals > 0). */
size_t sw_workspace_bytes(int32_t n_reads, int64_t n_cals, const sw_scoring_t *sc);

/* Invalid task slots seen by sw_align_batch on this device since load (or the
 * last reset).  Synchronises the device. */
int sw_error_count(int64_t *n_invalid, int reset);

/*
 * Score Tracker (sections 3.6 and 4.2): best slot per (read, reference).
 *   cal_ptr     device [n_reads+1] CSR row pointer as for sw_align_batch; each
 *               row is clamped to [0, n_cals] on the device, so a malformed row
 *               pointer gives fewer slots, never an access outside the arrays
 *   cal_ref     device [n_cals]; score device [2*n_cals] (sw_align_batch output)
 *   best_score  device [n_reads*n_refs] highest score among valid slots (-1 if none)
 *   best_slot   device [n_reads*n_refs] lowest slot index reaching it (-1 if none)
 *   n_tied      device [n_reads*n_refs] number of slots reaching it (0 if none)
 * Slots with negative scores (not requested, invalid) are skipped; CALs whose
 * reference id is outside [0, n_refs) are skipped.
 */
int sw_reduce_best(const int64_t *cal_ptr, const int16_t *cal_ref, int32_t n_reads, int32_t n_refs, int64_t n_cals,
                   const int32_t *score, int32_t *best_score, int64_t *best_slot, int32_t *n_tied,
                   sw_stream_t stream);

/*
 * Score Tracker variants (section 4.2): best CAL, top-k CALs, or all tied CALs.
 *
 * sw_topk: the k best slots of each read over all its CALs and both strands,
 * highest score first and the lower slot index first among equal scores.
 *   k           1..SW_MAX_TOPK
 *   top_score   device [n_reads*k] scores, -1 past the read's valid slots
 *   top_slot    device [n_reads*k] slot indices (2c fwd, 2c+1 rev), -1 likewise
 * Slots with negative scores (not requested, invalid) are skipped.
 *
 * sw_tied_flags: flags[slot] = 1 if the slot's score equals the highest
 * non-negative score of its read over all its slots, else 0.
 *   flags       device [2*n_cals]; slots outside every (clamped) row are not written
 * In both, cal_ptr rows are clamped to [0, n_cals] as for sw_reduce_best.  Both
 * are asynchronous on `stream`; invalid host arguments return
 * SW_ERR_INVALID_ARG before any device work.
 */
#define SW_MAX_TOPK 64
int sw_topk(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, const int32_t *score, int32_t k,
            int32_t *top_score, int64_t *top_slot, sw_stream_t stream);
int sw_tied_flags(const int64_t *cal_ptr, int32_t n_reads, int64_t n_cals, const int32_t *score, uint8_t *flags,
                  sw_stream_t stream);

/* ------------------------------------------------------------------ seeding */
/*
 * Seed index (section 3.1) and CAL finder (section 3.2).
 *
 * The index holds every overlapping seed of seed_len bases of every
 * reference, each reduced to its canonical form (the smaller of the seed and
 * its reverse complement, with a bit saying which one the reference holds)
 * and hashed so that the pointer table's buckets fill evenly; the CAL table
 * lists the seeds' positions sorted by hash, and the pointer table (2^addr_bits
 * entries) points at the first CAL-table entry of each address.  It lives in
 * device memory (16 bytes per reference position, plus 8 per address) and
 * keeps a pointer to the reference set's words only during the build.
 *
 * sw_find_cals cuts each read into seeds starting at offsets 0, stride,
 * 2*stride, ... (stride 1: overlapping seeds; stride = seed_len: non-overlapping)
 * and looks each one up.  A read seed matches reference position x forward
 * when the reference seed there equals it (CAL strand 1 at x - offset), and
 * reverse when the reference holds its reverse complement (strand 2 at
 * x - (L - offset - seed_len), where base 0 of the read's reverse complement
 * falls); a palindromic seed matches both ways.  Positions are clipped to the
 * reference.  A seed with more than max_cals_per_seed matches (0: no limit)
 * contributes nothing.  CALs are listed per read, seed by seed, each seed's
 * matches by (reference, position), forward before reverse.  The output is
 * the CSR input of sw_cal_filter / sw_align_batch (duplicates included).
 *   cal_ptr   device [n_reads+1]    written in every successful or
 *                                   SW_ERR_WORKSPACE return
 *   cal_pos, cal_ref, strand  device [capacity]
 *   n_cals    host: number of CALs found; SW_ERR_WORKSPACE when it exceeds
 *             capacity (nothing else written; call again with room)
 * The call synchronises `stream` once (to read the count).  Reads longer than
 * max_read_len get no CALs and are counted by sw_error_count() when the CALs
 * are written (not on a SW_ERR_WORKSPACE return).  An index is not thread-safe.
 */
typedef struct sw_index sw_index_t;
typedef struct {
  int32_t device;    /* HIP device ordinal */
  int32_t seed_len;  /* 1..32 (the paper's V1 uses 22) */
  int32_t addr_bits; /* pointer-table address bits, 1..min(2*seed_len, 30); 0: about log2 of the
                        number of reference positions (one entry per address on average) */
} sw_index_opts_t;
typedef struct {
  int32_t stride;            /* >= 1 */
  int32_t max_cals_per_seed; /* >= 0; 0: no limit */
  int32_t max_read_len;      /* 1..SW_MAX_READ_LEN; 0 means SW_MAX_READ_LEN */
} sw_find_opts_t;
int sw_index_build(const sw_refset_t *refs, const sw_index_opts_t *opts, sw_index_t **out, sw_stream_t stream);
int sw_index_info(const sw_index_t *ix, int64_t *n_entries, int64_t *device_bytes);
int sw_index_destroy(sw_index_t *ix);
int sw_find_cals(sw_index_t *ix, const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                 int32_t n_reads, const sw_find_opts_t *opts, int64_t *cal_ptr, int64_t *cal_pos,
                 int16_t *cal_ref, uint8_t *strand, int64_t capacity, int64_t *n_cals, sw_stream_t stream);

/* ------------------------------------------------------------------ CAL filter */
/*
 * CAL Filter (section 3.3): the CALs of a read that point at the same part of
 * the reference are combined into one lookup before scoring.  Two CALs of one
 * read are duplicates when they name the same reference and their positions
 * fall in the same bucket of 2^bucket_bits bases (0: identical positions only).
 * Each read keeps the first CAL of every bucket, in input order, carrying the
 * union of the strand masks of its duplicates.
 *   cal_ptr, cal_pos, cal_ref, strand   device: the CSR CAL lists (as for scoring)
 *   bucket_bits  0..40
 * Outputs, device:
 *   out_ptr    [n_reads+1]  CSR row pointer of the kept CALs; out_ptr[n_reads]
 *                           is their number (read it back to size the scoring call)
 *   out_pos, out_ref, out_strand  [n_cals]  kept CALs (first out_ptr[n_reads] used)
 *   cal_map    [n_cals]     kept CAL each input CAL was folded into (-1 for a CAL
 *                           outside every read's range)
 * With bucket_bits = 0, for every strand h that CAL c requests, slot
 * 2*cal_map[c]+h of a scoring call on the kept CALs holds exactly what slot
 * 2c+h of the unfiltered call holds (same read, reference and window).
 * cal_ptr must be non-decreasing with cal_ptr[n_reads] <= n_cals; if it is not,
 * the outputs are unspecified, but nothing outside the arrays is accessed.
 * `workspace` (device) must hold sw_cal_filter_workspace_bytes(n_reads) bytes.
 */
size_t sw_cal_filter_workspace_bytes(int32_t n_reads);
int sw_cal_filter(const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref, const uint8_t *strand,
                  int32_t n_reads, int64_t n_cals, int32_t bucket_bits, int64_t *out_ptr, int64_t *out_pos,
                  int16_t *out_ref, uint8_t *out_strand, int64_t *cal_map, void *workspace,
                  size_t workspace_bytes, sw_stream_t stream);

/* ------------------------------------------------------------------ traceback */
/*
 * Start position and CIGAR of selected slots.  The paper's hardware reports
 * only the score and the end (sections 3.5, 3.6); section 6.4 (Table 5) finds
 * CIGAR string generation the next bottleneck.  For each entry t of `slots` (a slot
 * index 2c+h into the outputs of a scoring call, or -1 to skip) the task's
 * dynamic program is rebuilt up to the reported end cell and walked backwards.
 * Where several alignments reach the score, the walk takes at every cell the
 * first move that explains its value: the diagonal, then a gap consuming a read
 * base, then a gap consuming a window base; inside a gap it returns to H (the
 * gap was opened there) whenever that explains the value; a diagonal step onto
 * a cell with H = 0 ends the alignment.
 *   reads2bit .. n_cals   the arrays of the scoring call (strands come from the slot)
 *   sc                    the scoring of that call (band, max_read_len and the
 *                         penalties must match; precision and mode are not used);
 *                         kernel: SW_KERNEL_INTER traces 64 slots per wavefront,
 *                         one per lane; SW_KERNEL_INTRA one slot per wavefront;
 *                         SW_KERNEL_AUTO the former unless its per-block buffer
 *                         would exceed 4 MiB (very long reads or wide bands)
 *   score, ref_end, read_end   device [2*n_cals]: the scoring call's outputs
 *   slots                 device [n_slots] int64
 *   cap                   CIGAR entries per slot (>= 1)
 * Outputs, device:
 *   ref_start  [n_slots]  absolute forward position of the first aligned window
 *                         base; -1 when n_ops <= 0
 *   read_start [n_slots]  first aligned base of the oriented read; -1 likewise
 *   n_ops      [n_slots]  entries written; 0 for a skipped slot or a score <= 0;
 *                         -1 if more than cap entries are needed (the row is then
 *                         cleared to 0); -2 if the slot,
 *                         its task or its end cell is invalid (the end cell's H
 *                         differs from the reported score), counted by
 *                         sw_error_count()
 *   cigar      [n_slots*cap]  (length << 4) | op in forward reference order, BAM
 *                         op codes: 1 I (read base only), 2 D (window base only),
 *                         4 S (soft clip: unaligned head and tail of the read),
 *                         7 '=' (match), 8 X (mismatch)
 * `workspace` must hold sw_traceback_workspace_bytes(n_slots, n_cals, sc) bytes
 * (the one-slot-per-lane kernel keeps 4 bits per cell of each block's 64 tasks
 * in it: tens of KB per block and read; the wavefront-per-slot kernel needs none
 * when a task's bits fit in LDS) and must not be used by an overlapping call.
 */
int sw_traceback(const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                 int32_t n_reads, const sw_refset_t *refs, const int64_t *cal_ptr, const int64_t *cal_pos,
                 const int16_t *cal_ref, int64_t n_cals, const sw_scoring_t *sc, const int32_t *score,
                 const int64_t *ref_end, const int16_t *read_end, const int64_t *slots, int64_t n_slots,
                 int32_t cap, int64_t *ref_start, int16_t *read_start, int32_t *n_ops, uint32_t *cigar,
                 void *workspace, size_t workspace_bytes, sw_stream_t stream);
size_t sw_traceback_workspace_bytes(int64_t n_slots, int64_t n_cals, const sw_scoring_t *sc);

/*
 * Classification of reads between references by best score (section 6.2,
 * xenograft case study): cls[r] = the reference with the strictly highest best
 * score if it is >= threshold, -2 if two or more references share a top score
 * >= threshold (tie), -1 if no reference reaches the threshold (unaligned).
 */
int sw_classify(const int32_t *best_score, int32_t n_reads, int32_t n_refs, int32_t threshold,
                int32_t *cls, sw_stream_t stream);

/* ------------------------------------------------------------------ batched */
/*
 * A context holds device buffers sized once for a batch capacity, an autotuned
 * launch plan and captured HIP graphs.  sw_align_batch_ctx has the semantics of
 * sw_align_batch (bit-identical outputs).  Its plan either bins the tasks by
 * read length (bin width, longest or shortest first, a strip height per bin)
 * and feeds a persistent kernel from a device work queue of tiles, or keeps
 * the tasks in input order, with one strip height, when that times faster (all
 * reads of one length); the plan is timed on the caller's inputs on first use
 * of a shape class (precision, mode, read-length bound, band, power of two of
 * the task count), and a captured graph is replayed when the shape repeats.
 * A context is not thread-safe: use one per host thread.
 */
typedef struct sw_ctx sw_ctx_t;

typedef struct {
  int32_t device;         /* HIP device ordinal */
  int32_t max_reads;      /* capacity: reads per call */
  int64_t max_cals;       /* capacity: CALs per call, 0..(INT32_MAX / 2): the planner keeps task
                             positions (two per CAL in int32 precision) in int32; larger
                             capacities are rejected with SW_ERR_INVALID_ARG */
  int32_t use_graph;      /* 1: capture and replay HIP graphs per shape */
  int32_t autotune;       /* 1: time candidate plans on first use of a shape class */
  const char *tune_cache; /* optional JSON file for autotune results (may be NULL) */
} sw_ctx_opts_t;

int sw_ctx_create(const sw_ctx_opts_t *opts, sw_ctx_t **out);
int sw_ctx_destroy(sw_ctx_t *ctx);
int sw_align_batch_ctx(sw_ctx_t *ctx, const uint32_t *reads2bit, const int64_t *read_word_off,
                       const int32_t *read_len, int32_t n_reads, const sw_refset_t *refs,
                       const int64_t *cal_ptr, const int64_t *cal_pos, const int16_t *cal_ref,
                       const uint8_t *strand, int64_t n_cals, const sw_scoring_t *sc, int32_t *score,
                       int64_t *ref_end, int16_t *read_end, sw_stream_t stream);
/* Invalid task slots of the last sw_align_batch_ctx call on this context;
 * synchronises the context's device. */
int sw_ctx_error_count(sw_ctx_t *ctx, int64_t *n_invalid);
/* Text description of the last plan used (bins, tiles, kernel variants). */
const char *sw_ctx_last_plan(sw_ctx_t *ctx);

/* ------------------------------------------------------------------ served */
/*
 * A server keeps a reference set resident, admits requests by their footprint
 * in a pinned staging arena that the device maps, and packs chunks of every
 * admitted request into each device step (continuous batching): a request that
 * arrives while a step runs joins the next step as soon as arena memory frees
 * up.  A request is staged with its reads packed to 2 bits in a coherent arena;
 * each step's gather kernels read its chunks from the arena in place and its
 * scatter kernels write the results back there, so device memory holds only the
 * references and the step buffers.  The step's read lengths, word offsets and
 * CAL row pointers come from the server's host copies, so no device address is
 * ever formed from staged bytes.  Each step runs the batched
 * pipeline (sw_align_batch_ctx) and the Score Tracker reduction, and a request's
 * results are bit-identical to sw_align_batch + sw_reduce_best on the request
 * alone.  The paper's V2 streams reads and their CALs from host threads to the
 * accelerator that holds the whole reference (sections 4.2, 4.3).
 * One scheduler thread per server; submit, wait and info may be called from
 * any thread.
 */
typedef struct sw_server sw_server_t;

typedef struct {
  int32_t device;
  sw_scoring_t scoring;     /* scoring of every request (max_read_len bounds the reads) */
  size_t memory_budget;     /* bytes of the pinned, device-mapped staging arena for admitted
                               requests' inputs and outputs (>= 1 MiB) */
  int32_t max_step_reads;   /* reads per device step; also the largest request in reads */
  int64_t max_step_cals;    /* CALs per device step; also the most CALs of one read */
  int32_t max_step_chunks;  /* request chunks per step, 1..4096 */
  int32_t autotune;         /* 1: autotune the binning plan of each step shape class */
  int32_t max_steps_in_flight; /* 1..3: at most that many steps queued on the device.
                                  0 (adaptive): one, and the next is launched early,
                                  once the running step is predicted to end within the
                                  host time of a launch (a fit of step time against DP
                                  cells over recent steps).  Under load a request waits
                                  for every step queued ahead of its own, so one step
                                  in flight gives the lowest latency; launching the next
                                  early keeps the device busy while the host builds it */
} sw_server_opts_t;

typedef struct {
  int64_t steps, step_reads, step_cals; /* device steps run and their totals */
  int64_t pending;                      /* submitted, not yet admitted */
  int64_t in_flight_requests;           /* admitted, not yet done */
  int64_t arena_used, arena_size;       /* bytes */
  int64_t steps_launched_early;         /* adaptive rule: steps queued behind a running one */
} sw_server_stats_t;

int sw_server_create(const sw_server_opts_t *opts, sw_server_t **out);
/* Set the resident references (device words stay owned by the caller and must
 * outlive the server) and start serving.  Once only. */
int sw_server_set_refs(sw_server_t *srv, const sw_refset_t *refs);
/*
 * Submit one request (host arrays, copied before the call returns):
 *   read_codes     host uint8 [n_codes], base codes; read r is
 *                  read_codes[read_code_off[r] .. read_code_off[r] + read_len[r])
 *                  (any layout: the server packs the reads back to back)
 *   read_len       host [n_reads], 0..scoring.max_read_len
 *   cal_ptr        host [n_reads+1] CSR (cal_ptr[0] = 0, cal_ptr[n_reads] = n_cals)
 *   cal_pos, cal_ref, strand: host [n_cals], as for sw_align_batch
 * Outputs (host, written when the request completes; keep them alive until then):
 *   score, ref_end, read_end [2*n_cals] as for sw_align_batch;
 *   best_score, best_slot, n_tied [n_reads*n_refs] as for sw_reduce_best (may be NULL).
 * Returns SW_ERR_REJECTED if the request's footprint exceeds the memory budget,
 * SW_ERR_INVALID_ARG for malformed inputs or a request with more reads than a
 * step.  *req_id identifies the request.
 */
int sw_server_submit(sw_server_t *srv, const uint8_t *read_codes, int64_t n_codes, const int64_t *read_code_off,
                     const int32_t *read_len, int32_t n_reads, const int64_t *cal_ptr, const int64_t *cal_pos,
                     const int16_t *cal_ref, const uint8_t *strand, int64_t n_cals, int32_t *score,
                     int64_t *ref_end, int16_t *read_end, int32_t *best_score, int64_t *best_slot,
                     int32_t *n_tied, int64_t *req_id);
/* Wait up to timeout_ms (-1: forever) for a request; *done = 1 when it has
 * finished.  Returns the error of a failed request (a library call of a step
 * that held some of its reads failed; its output buffers are left untouched),
 * else SW_OK. */
int sw_server_wait(sw_server_t *srv, int64_t req_id, int32_t timeout_ms, int32_t *done);
/* State (0 pending, 1 admitted, 3 done, 4 failed) and steady-clock times in seconds. */
int sw_server_request_info(sw_server_t *srv, int64_t req_id, int32_t *state, double *t_submit, double *t_admit,
                           double *t_done);
/* Forget a finished (done or failed) request. */
int sw_server_release(sw_server_t *srv, int64_t req_id);
int sw_server_stats(sw_server_t *srv, sw_server_stats_t *out);
/* Drain every submitted request, then free the server. */
int sw_server_destroy(sw_server_t *srv);

/* ------------------------------------------------------------------ calibration */
/*
 * Sustained integer VALU rate of the current device: every compute unit runs
 * independent chains of add + max in packed 16-bit (bits = 16; a packed op
 * counts as two lane-ops) or 32-bit (bits = 32) arithmetic for `iters` steps
 * (>= 16).  *ops_per_s receives lane-ops per second.  Synchronises the stream;
 * allocates a small device buffer.
 */
int sw_alu_peak(int32_t bits, int64_t iters, double *ops_per_s, sw_stream_t stream);

/*
 * Check of the one device property the int16 scoring kernels take from the
 * hardware rather than from integer arithmetic: per 16-bit half, the packed
 * half-precision maximum of three operands must return the operand of highest
 * rank when the bit patterns [0, 0x7BFF] rank in integer order and the
 * patterns [0x8000, 0xFBFF] rank below all of them.  Every pair of patterns is
 * tested (6.0e9 halves).  *n_bad receives the number of halves that break the
 * order (0 on a conforming device).  Synchronises the stream; allocates a small
 * device buffer.
 */
int sw_check_half_max(int64_t *n_bad, sw_stream_t stream);

/* ------------------------------------------------------------------ misc */
const char *sw_strerror(int code);
int sw_last_hip_error(void);
const char *sw_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SW_ALIGN_H */
