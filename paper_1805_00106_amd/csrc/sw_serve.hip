// Kernels of the served path: gather the read/CAL chunks of several admitted
// requests into one step batch, and scatter the step's results back into each
// request's output arrays.  Pure data movement; scoring runs in the batched
// pipeline between them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_serve.h"

namespace swk {

__device__ __forceinline__ int find_chunk(const ServeChunk *ch, int n, int64_t v, bool by_read) {
  int lo = 0, hi = n - 1;  // last chunk whose step start is <= v
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t s = by_read ? ch[mid].step_r0 : ch[mid].step_c0;
    if (s <= v) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One thread per step read: read length, packed words, word offset and CAL row pointer.
__global__ void k_serve_gather_reads(const ServeChunk *__restrict__ ch, int n_chunks, int64_t n_reads,
                                     int64_t n_cals, uint32_t *__restrict__ words, int64_t *__restrict__ word_off,
                                     int32_t *__restrict__ read_len, int64_t *__restrict__ cal_ptr) {
  const int64_t rs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rs == 0) cal_ptr[n_reads] = n_cals;
  if (rs >= n_reads) return;
  const ServeChunk &c = ch[find_chunk(ch, n_chunks, rs, true)];
  const int64_t r = c.r0 + (rs - c.step_r0);
  const int32_t L = c.len[r];
  read_len[rs] = L;
  const int64_t src = c.word_off[r];
  const int64_t dst = c.step_w0 + (src - c.word_off[c.r0]);
  word_off[rs] = dst;
  const int nw = (L + 15) >> 4;
  for (int k = 0; k < nw; ++k) words[dst + k] = c.words[src + k];
  cal_ptr[rs] = c.step_c0 + (c.cal_ptr[r] - c.cal_ptr[c.r0]);
}

// One thread per step CAL: position, reference id, strand mask.
__global__ void k_serve_gather_cals(const ServeChunk *__restrict__ ch, int n_chunks, int64_t n_cals,
                                    int64_t *__restrict__ cal_pos, int16_t *__restrict__ cal_ref,
                                    uint8_t *__restrict__ strand) {
  const int64_t cs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cs >= n_cals) return;
  const ServeChunk &c = ch[find_chunk(ch, n_chunks, cs, false)];
  const int64_t cr = c.cal_ptr[c.r0] + (cs - c.step_c0);
  cal_pos[cs] = c.cal_pos[cr];
  cal_ref[cs] = c.cal_ref[cr];
  strand[cs] = c.strand[cr];
}

// One thread per step CAL: both slots back into the request (slots renumbered
// to the request's own CAL indices).
__global__ void k_serve_scatter_cals(const ServeChunk *__restrict__ ch, int n_chunks, int64_t n_cals,
                                     const int32_t *__restrict__ score, const int64_t *__restrict__ ref_end,
                                     const int16_t *__restrict__ read_end) {
  const int64_t cs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cs >= n_cals) return;
  const ServeChunk &c = ch[find_chunk(ch, n_chunks, cs, false)];
  const int64_t cr = c.cal_ptr[c.r0] + (cs - c.step_c0);
  for (int h = 0; h < 2; ++h) {
    c.score[2 * cr + h] = score[2 * cs + h];
    c.ref_end[2 * cr + h] = ref_end[2 * cs + h];
    c.read_end[2 * cr + h] = read_end[2 * cs + h];
  }
}

// One thread per step read: the per-reference best of the read, with the best
// slot renumbered to the request's CAL indices.
__global__ void k_serve_scatter_reads(const ServeChunk *__restrict__ ch, int n_chunks, int64_t n_reads,
                                      int32_t n_refs, const int32_t *__restrict__ best_score,
                                      const int64_t *__restrict__ best_slot, const int32_t *__restrict__ n_tied) {
  const int64_t rs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rs >= n_reads) return;
  const ServeChunk &c = ch[find_chunk(ch, n_chunks, rs, true)];
  const int64_t r = c.r0 + (rs - c.step_r0);
  const int64_t shift = 2 * (c.cal_ptr[c.r0] - c.step_c0);
  for (int k = 0; k < n_refs; ++k) {
    const int64_t so = rs * n_refs + k, ro = r * n_refs + k;
    c.best_score[ro] = best_score[so];
    const int64_t sl = best_slot[so];
    c.best_slot[ro] = sl >= 0 ? sl + shift : sl;
    c.n_tied[ro] = n_tied[so];
  }
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_serve_gather(const ServeChunk *ch, int n_chunks, int64_t n_reads, int64_t n_cals, uint32_t *words,
                               int64_t *word_off, int32_t *read_len, int64_t *cal_ptr, int64_t *cal_pos,
                               int16_t *cal_ref, uint8_t *strand, hipStream_t st) {
  hipLaunchKernelGGL(k_serve_gather_reads, dim3(nblk(std::max<int64_t>(n_reads, 1))), dim3(256), 0, st, ch, n_chunks,
                     n_reads, n_cals, words, word_off, read_len, cal_ptr);
  if (n_cals > 0)
    hipLaunchKernelGGL(k_serve_gather_cals, dim3(nblk(n_cals)), dim3(256), 0, st, ch, n_chunks, n_cals, cal_pos,
                       cal_ref, strand);
  return hipGetLastError();
}

hipError_t launch_serve_scatter(const ServeChunk *ch, int n_chunks, int64_t n_reads, int64_t n_cals, int32_t n_refs,
                                const int32_t *score, const int64_t *ref_end, const int16_t *read_end,
                                const int32_t *best_score, const int64_t *best_slot, const int32_t *n_tied,
                                hipStream_t st) {
  if (n_cals > 0)
    hipLaunchKernelGGL(k_serve_scatter_cals, dim3(nblk(n_cals)), dim3(256), 0, st, ch, n_chunks, n_cals, score,
                       ref_end, read_end);
  if (n_reads > 0)
    hipLaunchKernelGGL(k_serve_scatter_reads, dim3(nblk(n_reads)), dim3(256), 0, st, ch, n_chunks, n_reads, n_refs,
                       best_score, best_slot, n_tied);
  return hipGetLastError();
}

}  // namespace swk
