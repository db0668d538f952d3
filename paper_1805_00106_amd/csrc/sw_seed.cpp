// C ABI of the seed index and the CAL finder (sections 3.1 and 3.2 of the
// paper).  Declarations and contracts are in include/sw_align.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>

#include "../../include/sw_align.h"
#include "sw_api_internal.h"
#include "sw_index.h"
#include "sw_launch.h"

struct sw_index {
  int device = 0;
  swk::SeedParams p{};
  int32_t n_refs = 0;
  int64_t n = 0;
  uint64_t *key = nullptr, *val = nullptr;
  int64_t *ptr = nullptr;
  int64_t *ref_len = nullptr;  // device [n_refs]
  size_t bytes = 0;
  // CAL finder scratch, grown on demand
  int64_t *cnt = nullptr, *offs = nullptr, *run_lo = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0;
  int64_t slots_cap = -1;
};

namespace {

void free_index(sw_index *ix) {
  if (!ix) return;
  hipSetDevice(ix->device);
  hipFree(ix->key);
  hipFree(ix->val);
  hipFree(ix->ptr);
  hipFree(ix->ref_len);
  hipFree(ix->cnt);
  hipFree(ix->offs);
  hipFree(ix->run_lo);
  hipFree(ix->temp);
  delete ix;
}

template <typename T>
int dev_alloc(T **p, size_t bytes) {
  *p = nullptr;
  return hipMalloc(reinterpret_cast<void **>(p), bytes ? bytes : 1) == hipSuccess ? SW_OK : SW_ERR_NOMEM;
}

}  // namespace

extern "C" {

int sw_index_build(const sw_refset_t *refs, const sw_index_opts_t *opts, sw_index_t **out, sw_stream_t stream) {
  if (!out) return SW_ERR_INVALID_ARG;
  *out = nullptr;
  if (!opts || opts->device < 0) return SW_ERR_INVALID_ARG;
  const int S = opts->seed_len;
  if (S < 1 || S > 32) return SW_ERR_INVALID_ARG;
  if (opts->addr_bits != 0 && (opts->addr_bits < 1 || opts->addr_bits > std::min(2 * S, 30)))
    return SW_ERR_INVALID_ARG;
  swk::RefTable T;
  int rc = swapi::validate_refs(refs, 1, &T);
  if (rc) return rc;
  swk::SeedRefs R{};
  R.words = refs->words;
  R.n_refs = refs->n_refs;
  int64_t n = 0;
  for (int k = 0; k < refs->n_refs; ++k) {
    R.word_off[k] = refs->word_offset[k];
    R.len[k] = refs->length[k];
    R.occ_off[k] = n;
    if (refs->length[k] >= S) n += refs->length[k] - S + 1;
  }
  R.occ_off[refs->n_refs] = n;
  if (n > (int64_t)INT32_MAX) return SW_ERR_INVALID_ARG;  // radix sort item count
  // default: about one CAL-table entry per pointer-table address
  int A = opts->addr_bits;
  if (A == 0) {
    A = 1;
    while (A < std::min(2 * S, 30) && (1ll << A) < n) ++A;
  }
  hipError_t e = hipSetDevice(opts->device);
  if (e != hipSuccess) return swapi::hip_fail(e);
  sw_index *ix = new (std::nothrow) sw_index();
  if (!ix) return SW_ERR_NOMEM;
  ix->device = opts->device;
  ix->p.seed_len = S;
  ix->p.addr_bits = A;
  ix->n_refs = refs->n_refs;
  ix->n = n;
  const int64_t n_addr = 1ll << A;
  uint64_t *key_alt = nullptr, *val_alt = nullptr;
  void *temp = nullptr;
  const size_t temp_bytes = swk::index_sort_temp_bytes(std::max<int64_t>(n, 1), S);
  if (dev_alloc(&ix->key, 8 * (size_t)n) || dev_alloc(&ix->val, 8 * (size_t)n) ||
      dev_alloc(&ix->ptr, 8 * (size_t)(n_addr + 1)) || dev_alloc(&ix->ref_len, 8 * (size_t)refs->n_refs) ||
      dev_alloc(&key_alt, 8 * (size_t)n) || dev_alloc(&val_alt, 8 * (size_t)n) || dev_alloc(&temp, temp_bytes)) {
    hipFree(key_alt);
    hipFree(val_alt);
    hipFree(temp);
    free_index(ix);
    return SW_ERR_NOMEM;
  }
  ix->bytes = 16 * (size_t)n + 8 * (size_t)(n_addr + 1) + 8 * (size_t)refs->n_refs;
  hipStream_t st = (hipStream_t)stream;
  e = hipMemcpyAsync(ix->ref_len, refs->length, 8 * (size_t)refs->n_refs, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = swk::launch_index_build(R, ix->p, n, ix->key, ix->val, key_alt, val_alt, temp, temp_bytes, ix->ptr, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the build buffers are released below
  hipFree(key_alt);
  hipFree(val_alt);
  hipFree(temp);
  if (e != hipSuccess) {
    free_index(ix);
    return swapi::hip_fail(e);
  }
  *out = ix;
  return SW_OK;
}

int sw_index_info(const sw_index_t *ix, int64_t *n_entries, int64_t *device_bytes) {
  if (!ix) return SW_ERR_INVALID_ARG;
  if (n_entries) *n_entries = ix->n;
  if (device_bytes) *device_bytes = (int64_t)ix->bytes;
  return SW_OK;
}

int sw_index_destroy(sw_index_t *ix) {
  if (!ix) return SW_ERR_INVALID_ARG;
  hipSetDevice(ix->device);
  hipDeviceSynchronize();
  free_index(ix);
  return SW_OK;
}

int sw_find_cals(sw_index_t *ix, const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                 int32_t n_reads, const sw_find_opts_t *o, int64_t *cal_ptr, int64_t *cal_pos, int16_t *cal_ref,
                 uint8_t *strand, int64_t capacity, int64_t *n_cals, sw_stream_t stream) {
  if (!ix || !o || !n_cals || n_reads < 0 || capacity < 0) return SW_ERR_INVALID_ARG;
  *n_cals = 0;
  if (o->stride < 1 || o->max_cals_per_seed < 0) return SW_ERR_INVALID_ARG;
  const int mrl = o->max_read_len == 0 ? SW_MAX_READ_LEN : o->max_read_len;
  if (mrl < 1) return SW_ERR_INVALID_ARG;
  if (mrl > SW_MAX_READ_LEN) return SW_ERR_READ_TOO_LONG;
  if (!cal_ptr) return SW_ERR_INVALID_ARG;
  if (n_reads > 0 && (!reads2bit || !read_word_off || !read_len)) return SW_ERR_INVALID_ARG;
  if (capacity > 0 && (!cal_pos || !cal_ref || !strand)) return SW_ERR_INVALID_ARG;
  const int S = ix->p.seed_len;
  const int max_seeds = mrl >= S ? (mrl - S) / o->stride + 1 : 1;
  const int64_t n_slots = (int64_t)n_reads * max_seeds;
  if (n_slots + 1 > (int64_t)INT32_MAX) return SW_ERR_INVALID_ARG;  // scan item count
  hipError_t e = hipSetDevice(ix->device);
  if (e != hipSuccess) return swapi::hip_fail(e);
  hipStream_t st = (hipStream_t)stream;
  if (n_slots > ix->slots_cap) {
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return swapi::hip_fail(e);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return swapi::hip_fail(e);
    hipFree(ix->cnt);
    hipFree(ix->offs);
    hipFree(ix->run_lo);
    hipFree(ix->temp);
    ix->cnt = nullptr;
    ix->offs = nullptr;
    ix->run_lo = nullptr;
    ix->temp = nullptr;
    ix->slots_cap = -1;
    const int64_t cap = std::max<int64_t>(n_slots, 1 << 16);
    ix->temp_bytes = swk::find_temp_bytes(cap);
    if (dev_alloc(&ix->cnt, 8 * (size_t)(cap + 1)) || dev_alloc(&ix->offs, 8 * (size_t)(cap + 1)) ||
        dev_alloc(&ix->run_lo, 8 * (size_t)(cap + 1)) || dev_alloc(&ix->temp, ix->temp_bytes))
      return SW_ERR_NOMEM;
    ix->slots_cap = cap;
  }
  unsigned long long *err = swk::error_counter();
  if (!err) return swapi::hip_fail(hipErrorInvalidDevice);
  swk::FindArgs A{};
  A.ix = swk::IndexView{ix->key, ix->val, ix->ptr, ix->n, ix->p};
  A.reads = reads2bit;
  A.read_word_off = read_word_off;
  A.read_len = read_len;
  A.n_reads = n_reads;
  A.stride = o->stride;
  A.max_cals_per_seed = o->max_cals_per_seed;
  A.max_read_len = mrl;
  A.max_seeds = max_seeds;
  A.ref_len = ix->ref_len;
  A.cal_ptr = cal_ptr;
  A.cal_pos = cal_pos;
  A.cal_ref = cal_ref;
  A.strand = strand;
  A.err = err;
  e = swk::launch_find_count(A, ix->cnt, ix->offs, ix->run_lo, ix->temp, ix->temp_bytes, st);
  if (e != hipSuccess) return swapi::hip_fail(e);
  int64_t total = 0;
  if ((e = hipMemcpyAsync(&total, ix->offs + n_slots, 8, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return swapi::hip_fail(e);
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return swapi::hip_fail(e);
  *n_cals = total;
  if (total > capacity) return SW_ERR_WORKSPACE;
  e = swk::launch_find_write(A, ix->offs, ix->run_lo, st);
  return e == hipSuccess ? SW_OK : swapi::hip_fail(e);
}

}  // extern "C"
