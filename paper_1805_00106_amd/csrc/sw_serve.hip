// Kernels of the served path: gather the read/CAL chunks of several admitted
// requests into one step batch, and scatter the step's results back into each
// request's output arrays.  Pure data movement; scoring runs in the batched
// pipeline between them.  Each thread moves one element: the chunk holding it
// is found by a binary search over the chunks' step offsets, and the element's
// offset inside the chunk is checked against the chunk's host-computed count.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_serve.h"

namespace swk {

enum ChunkKey { kByRead = 0, kByCal = 1, kByWord = 2 };

__device__ __forceinline__ int64_t chunk_start(const ServeChunk &c, int key) {
  return key == kByRead ? c.step_r0 : (key == kByCal ? c.step_c0 : c.step_w0);
}

// Last chunk whose step start is <= v (chunks are in step order; a chunk with
// no CALs or no words shares its start with the next one, which then wins).
__device__ __forceinline__ int find_chunk(const ServeChunk *ch, int n, int64_t v, int key) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (chunk_start(ch[mid], key) <= v) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One thread per step word.
__global__ void k_serve_gather_words(const ServeChunk *__restrict__ ch, int n_chunks, int64_t n_words,
                                     uint32_t *__restrict__ words) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n_words) return;
  const ServeChunk &c = ch[find_chunk(ch, n_chunks, w, kByWord)];
  const int64_t o = w - c.step_w0;
  words[w] = (o >= 0 && o < c.n_words) ? c.words[o] : 0u;
}

// One thread per step CAL: position, reference id, strand mask.  A CAL outside
// every chunk (only possible if the host counts disagree) becomes an invalid
// task rather than an access.
__global__ void k_serve_gather_cals(const ServeChunk *__restrict__ ch, int n_chunks, int64_t n_cals,
                                    int64_t *__restrict__ cal_pos, int16_t *__restrict__ cal_ref,
                                    uint8_t *__restrict__ strand) {
  const int64_t cs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cs >= n_cals) return;
  const ServeChunk &c = ch[find_chunk(ch, n_chunks, cs, kByCal)];
  const int64_t o = cs - c.step_c0;
  if (o >= 0 && o < c.n_cals) {
    cal_pos[cs] = c.cal_pos[o];
    cal_ref[cs] = c.cal_ref[o];
    strand[cs] = c.strand[o];
  } else {
    cal_pos[cs] = -1;
    cal_ref[cs] = -1;
    strand[cs] = 0;
  }
}

// One thread per step CAL: both slots back into the request.
__global__ void k_serve_scatter_cals(const ServeChunk *__restrict__ ch, int n_chunks, int64_t n_cals,
                                     const int32_t *__restrict__ score, const int64_t *__restrict__ ref_end,
                                     const int16_t *__restrict__ read_end) {
  const int64_t cs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cs >= n_cals) return;
  const ServeChunk &c = ch[find_chunk(ch, n_chunks, cs, kByCal)];
  const int64_t o = cs - c.step_c0;
  if (o < 0 || o >= c.n_cals) return;
  for (int h = 0; h < 2; ++h) {
    c.score[2 * o + h] = score[2 * cs + h];
    c.ref_end[2 * o + h] = ref_end[2 * cs + h];
    c.read_end[2 * o + h] = read_end[2 * cs + h];
  }
}

// One thread per step read: the per-reference best of the read, with the best
// slot renumbered to the request's CAL indices.
__global__ void k_serve_scatter_reads(const ServeChunk *__restrict__ ch, int n_chunks, int64_t n_reads,
                                      int32_t n_refs, const int32_t *__restrict__ best_score,
                                      const int64_t *__restrict__ best_slot, const int32_t *__restrict__ n_tied) {
  const int64_t rs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rs >= n_reads) return;
  const ServeChunk &c = ch[find_chunk(ch, n_chunks, rs, kByRead)];
  const int64_t o = rs - c.step_r0;
  if (o < 0 || o >= c.n_reads) return;
  for (int k = 0; k < n_refs; ++k) {
    const int64_t so = rs * n_refs + k, ro = o * n_refs + k;
    c.best_score[ro] = best_score[so];
    const int64_t sl = best_slot[so];
    c.best_slot[ro] = sl >= 0 ? sl + c.slot_shift : sl;
    c.n_tied[ro] = n_tied[so];
  }
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_serve_gather(const ServeChunk *ch, int n_chunks, int64_t n_words, int64_t n_cals, uint32_t *words,
                               int64_t *cal_pos, int16_t *cal_ref, uint8_t *strand, hipStream_t st) {
  if (n_chunks < 1) return hipSuccess;
  if (n_words > 0)
    hipLaunchKernelGGL(k_serve_gather_words, dim3(nblk(n_words)), dim3(256), 0, st, ch, n_chunks, n_words, words);
  if (n_cals > 0)
    hipLaunchKernelGGL(k_serve_gather_cals, dim3(nblk(n_cals)), dim3(256), 0, st, ch, n_chunks, n_cals, cal_pos,
                       cal_ref, strand);
  return hipGetLastError();
}

hipError_t launch_serve_scatter(const ServeChunk *ch, int n_chunks, int64_t n_reads, int64_t n_cals, int32_t n_refs,
                                const int32_t *score, const int64_t *ref_end, const int16_t *read_end,
                                const int32_t *best_score, const int64_t *best_slot, const int32_t *n_tied,
                                hipStream_t st) {
  if (n_chunks < 1) return hipSuccess;
  if (n_cals > 0)
    hipLaunchKernelGGL(k_serve_scatter_cals, dim3(nblk(n_cals)), dim3(256), 0, st, ch, n_chunks, n_cals, score,
                       ref_end, read_end);
  if (n_reads > 0)
    hipLaunchKernelGGL(k_serve_scatter_reads, dim3(nblk(n_reads)), dim3(256), 0, st, ch, n_chunks, n_reads, n_refs,
                       best_score, best_slot, n_tied);
  return hipGetLastError();
}

}  // namespace swk
