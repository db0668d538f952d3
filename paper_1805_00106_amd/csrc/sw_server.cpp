// Served execution: resident references, admission by staging-memory footprint,
// continuous batching of admitted requests into device steps, and per-request
// timestamps for latency.  Contracts are in include/sw_align.h.
//
// The paper's V2 host keeps the reference resident on the accelerator and
// streams each read followed by its CALs to it, with separate threads feeding
// and draining the device (sections 4.2 and 4.3).  Here a request is staged
// (reads packed to 2 bits, back to back) in a pinned, coherent arena that the
// device maps; one scheduler thread packs chunks of every admitted request
// into each device step, whose gather kernels read the chunks straight from
// the mapped arena and whose scatter kernels write the results straight back,
// so a request costs no device copy or kernel of its own and requests that
// arrive while a step runs join the next one.  The step's per-read arrays
// (lengths, word offsets, CAL row pointers) are built by the scheduler from its
// host copies and sent with the chunk descriptors in one transfer: no device
// address is formed from bytes read out of the arena.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/sw_align.h"
#include "sw_api_internal.h"
#include "sw_launch.h"
#include "sw_serve.h"

// Test builds of the host logic define SW_SERVE_MARK_BLOCK(host_ptr, bytes, live)
// to poison the host bytes of arena blocks while they are free, so that the
// address sanitizer reports any access outside a reservation; in the library it
// does nothing.
#ifndef SW_SERVE_MARK_BLOCK
#define SW_SERVE_MARK_BLOCK(ptr, bytes, live) ((void)0)
#endif

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// First-fit allocator over [0, size) with coalescing of freed blocks.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t *off) {
    bytes = up256(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = up256(std::max<size_t>(bytes, 1));
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_, used_ = 0;
  std::map<size_t, size_t> free_;
};

enum ReqState { RS_PENDING = 0, RS_ADMITTED = 1, RS_DONE = 3, RS_FAILED = 4 };

struct Layout {  // byte offsets of one request's arrays inside its arena block
  size_t words, cal_pos, cal_ref, strand;
  size_t score, ref_end, read_end, best_score, best_slot, n_tied;
  size_t in_end, total;
};

struct Request {
  int64_t id = 0;
  int32_t n_reads = 0;
  int64_t n_cals = 0, n_codes = 0;
  // host copies of the inputs (the caller may reuse its buffers after submit);
  // codes, code_off and the CAL arrays are dropped once staged
  std::vector<uint8_t> codes;
  std::vector<int64_t> code_off, cal_ptr, cal_pos;
  std::vector<int64_t> wptr;  // [n_reads + 1] first packed word of each read in the staged words
  std::vector<int32_t> len;
  std::vector<int16_t> cal_ref;
  std::vector<uint8_t> strand;
  // caller's output buffers (host), filled at completion
  int32_t *o_score;
  int64_t *o_ref_end;
  int16_t *o_read_end;
  int32_t *o_best_score;
  int64_t *o_best_slot;
  int32_t *o_n_tied;
  Layout lay{};
  size_t off = 0;
  int64_t next_read = 0;  // first read not yet placed in a step
  int64_t reads_done = 0;
  int state = RS_PENDING;
  int error = 0;        // first error of a step holding some of its reads
  bool staged = false;  // inputs already staged in the pinned arena at `off`
  double t_submit = 0, t_admit = 0, t_done = 0;
};

struct StepSlot {  // device buffers of one step (the slots are used in turn)
  uint32_t *words = nullptr;
  int64_t *cal_pos = nullptr;
  int16_t *cal_ref = nullptr;
  uint8_t *strand = nullptr;
  int32_t *score = nullptr;
  int64_t *ref_end = nullptr;
  int16_t *read_end = nullptr;
  int32_t *best_score = nullptr;
  int64_t *best_slot = nullptr;
  int32_t *n_tied = nullptr;
  // per-step header (read lengths, word offsets, CAL row pointers, chunk
  // descriptors), built on the host in pinned memory and copied in one transfer
  char *hdr_host = nullptr;
  char *hdr_dev = nullptr;
  void *base = nullptr;
  hipEvent_t done = nullptr;
  // All slots share one stream: steps run back to back, and the scheduler can
  // queue the next steps while one runs.  (On separate streams the small kernels
  // of one step waited behind the persistent scoring kernel of the next.)
  hipStream_t stream = nullptr;
  sw_ctx_t *ctx = nullptr;  // one batched context per slot
  void *small_ws = nullptr;  // workspace of the plain call that small steps use
  size_t small_ws_bytes = 0;
  bool busy = false;
  bool small = false;     // took the plain call
  double t_launch = 0;    // host time its launch began
  double cells = 0;       // DP cells of its tasks (both strands), for the step-time model
  int error = 0;  // error of the step's library calls, passed to its requests
  std::vector<std::pair<std::shared_ptr<Request>, int64_t>> parts;  // request and reads placed
  std::vector<int64_t> part_r0;                                      // first read of each part
};

// Byte offsets of one step's header: read lengths, word offsets and CAL row
// pointers of the step's reads, then the chunk descriptors.
struct StepHeader {
  size_t len, word_off, cal_ptr, chunks, bytes;
};

StepHeader header_layout(int64_t n_reads, int64_t n_chunks) {
  StepHeader h{};
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t r = o;
    o = up256(o + bytes);
    return r;
  };
  h.len = put(sizeof(int32_t) * n_reads);
  h.word_off = put(sizeof(int64_t) * n_reads);
  h.cal_ptr = put(sizeof(int64_t) * (n_reads + 1));
  h.chunks = put(sizeof(swk::ServeChunk) * n_chunks);
  h.bytes = o;
  return h;
}

constexpr int kSlots = 3;

// Device time of a step against its DP cells, t = a + b * cells, fitted by least
// squares over the steps seen so far with older steps weighted down by 0.9 per
// step (the request mix drifts).  When the cells hardly vary (every step full)
// the fit falls back to t = b * cells.
class StepModel {
 public:
  void add(double x, double y) {
    const double f = 0.9;
    s0_ = f * s0_ + 1;
    sx_ = f * sx_ + x;
    sy_ = f * sy_ + y;
    sxx_ = f * sxx_ + x * x;
    sxy_ = f * sxy_ + x * y;
    ++n_;
  }
  bool predict(double x, double *y) const {
    if (n_ < 4 || sx_ <= 0) return false;
    const double d = s0_ * sxx_ - sx_ * sx_;
    double b = sy_ / sx_, a = 0;
    if (d > 1e-6 * s0_ * sxx_) {
      const double bl = (s0_ * sxy_ - sx_ * sy_) / d;
      const double al = (sy_ - bl * sx_) / s0_;
      if (bl > 0 && al >= 0) {
        b = bl;
        a = al;
      }
    }
    *y = a + b * x;
    return true;
  }

 private:
  double s0_ = 0, sx_ = 0, sy_ = 0, sxx_ = 0, sxy_ = 0;
  int64_t n_ = 0;
};

}  // namespace

struct sw_server {
  sw_server_opts_t opts{};
  sw_scoring_t sc{};
  sw_scoring_t sc_small{};       // the scoring of small steps (kernel choice left to AUTO)
  int64_t small_step_cals = 0;   // steps up to this many CALs take the plain call
  swapi::ScoreMode mode{};
  int32_t n_refs = 0;
  sw_refset_t refs{};
  std::vector<int64_t> ref_off, ref_len;
  bool refs_set = false;
  uint8_t *arena_host = nullptr;  // pinned staging arena (requests' inputs and outputs)
  uint8_t *arena_map = nullptr;   // the same memory as the device addresses it
  std::unique_ptr<Arena> arena;
  StepSlot slots[kSlots];
  int next_slot = 0;
  std::deque<std::shared_ptr<Request>> pending;
  std::deque<std::shared_ptr<Request>> admitted;  // admitted, not fully placed in steps
  std::deque<StepSlot *> in_flight;
  std::map<int64_t, std::shared_ptr<Request>> all;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_fin;
  std::thread worker;
  std::thread finisher;                            // copies results out, frees blocks
  std::deque<std::shared_ptr<Request>> to_finish;  // all reads done, results in the arena
  int64_t finishing = 0;                           // handed to the finisher, not yet done
  bool worker_running = false;
  std::atomic<bool> stop{false};
  int64_t next_id = 1;
  int last_error = 0;
  int64_t steps = 0, step_reads = 0, step_cals = 0, steps_early = 0;
  // adaptive launch (max_steps_in_flight 0): one step runs, and the next is
  // launched once the running one is predicted to end within a launch's host time
  StepModel model[2];     // batched and small (plain-call) steps
  double t_gpu_free = 0;  // host time the last retired step was seen done
  double lead_s = 3e-4;   // host time of a step launch (running mean) plus a margin
};

namespace {

Layout make_layout(int32_t n_reads, int64_t n_cals, int64_t n_words, int32_t n_refs) {
  Layout L{};
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t r = o;
    o = up256(o + bytes);
    return r;
  };
  L.words = put(sizeof(uint32_t) * n_words);
  L.cal_pos = put(sizeof(int64_t) * n_cals);
  L.cal_ref = put(sizeof(int16_t) * n_cals);
  L.strand = put(n_cals);
  L.in_end = o;
  L.score = put(sizeof(int32_t) * 2 * n_cals);
  L.ref_end = put(sizeof(int64_t) * 2 * n_cals);
  L.read_end = put(sizeof(int16_t) * 2 * n_cals);
  L.best_score = put(sizeof(int32_t) * n_reads * n_refs);
  L.best_slot = put(sizeof(int64_t) * n_reads * n_refs);
  L.n_tied = put(sizeof(int32_t) * n_reads * n_refs);
  L.total = o;
  return L;
}

template <class T>
T *dptr(sw_server *s, const Request &r, size_t field) {  // device address of an arena field
  return reinterpret_cast<T *>(s->arena_map + r.off + field);
}
template <class T>
T *hptr(sw_server *s, const Request &r, size_t field) {
  return reinterpret_cast<T *>(s->arena_host + r.off + field);
}

// Stage a request's inputs in its block of the pinned arena, packing the reads
// to 2 bits per base (16 bases per word, first base least significant), each
// read from its own code offset into the words from r.wptr[i] on: back to back,
// whatever the caller's layout.
// Eight base codes (one byte each, low 2 bits used) to 16 bits, base k at bits
// 2k: adjacent fields are merged pairwise in three shift-or steps.
inline uint32_t pack8(const uint8_t *q) {
  uint64_t x;
  std::memcpy(&x, q, 8);
  x &= 0x0303030303030303ull;
  x = (x | (x >> 6)) & 0x000F000F000F000Full;
  x = (x | (x >> 12)) & 0x000000FF000000FFull;
  return (uint32_t)((x | (x >> 24)) & 0xFFFFu);
}

void stage_inputs(sw_server *s, Request &r, const uint8_t *codes, const int64_t *code_off, const int64_t *cal_pos,
                  const int16_t *cal_ref, const uint8_t *strand) {
  uint32_t *words = hptr<uint32_t>(s, r, r.lay.words);
  for (int32_t i = 0; i < r.n_reads; ++i) {
    const uint8_t *q = codes + code_off[i];
    const int32_t L = r.len[i];
    uint32_t *out = words + r.wptr[i];
    int32_t b = 0;
    for (; b + 16 <= L; b += 16) *out++ = pack8(q + b) | pack8(q + b + 8) << 16;
    if (b < L) {  // the last, partial word
      uint32_t v = 0;
      for (int k = 0; b + k < L; ++k) v |= (uint32_t)(q[b + k] & 3u) << (2 * k);
      *out = v;
    }
  }
  if (r.n_cals > 0) {
    std::memcpy(hptr<int64_t>(s, r, r.lay.cal_pos), cal_pos, sizeof(int64_t) * r.n_cals);
    std::memcpy(hptr<int16_t>(s, r, r.lay.cal_ref), cal_ref, sizeof(int16_t) * r.n_cals);
    std::memcpy(hptr<uint8_t>(s, r, r.lay.strand), strand, r.n_cals);
  }
  r.staged = true;
}

// Admission (scheduler thread, lock held): reserve the footprint and stage the
// inputs if the request did not get its block at submit.  The device reads the
// staged inputs in place, so admission needs no device work.
bool admit(sw_server *s, std::shared_ptr<Request> &rq) {
  Request &r = *rq;
  if (!r.staged) {
    size_t off = 0;
    if (!s->arena->alloc(r.lay.total, &off)) return false;
    r.off = off;
    SW_SERVE_MARK_BLOCK(s->arena_host + off, up256(r.lay.total), 1);
    stage_inputs(s, r, r.codes.data(), r.code_off.data(), r.cal_pos.data(), r.cal_ref.data(), r.strand.data());
  }
  r.t_admit = now_s();
  r.state = RS_ADMITTED;
  std::vector<uint8_t>().swap(r.codes);
  std::vector<int64_t>().swap(r.code_off);
  std::vector<int64_t>().swap(r.cal_pos);
  std::vector<int16_t>().swap(r.cal_ref);
  std::vector<uint8_t>().swap(r.strand);
  return true;
}

// Whether another step may be launched now.  A fixed depth allows that many
// steps queued on the device.  The adaptive rule keeps one: a request that
// arrives while a step runs joins the step launched next, so a queued step would
// add its whole run to that request's wait.  But the next step's host work
// (building its header, a dozen launches) would then leave the device idle
// between steps, so it is launched early, once the running step's predicted end
// is within that host time.
bool may_launch(const sw_server *s, double now) {
  const int n = (int)s->in_flight.size();
  if (s->opts.max_steps_in_flight > 0) return n < s->opts.max_steps_in_flight;
  if (n == 0) return true;
  if (n > 1) return false;
  const StepSlot &run = *s->in_flight.front();
  double dur = 0;
  if (!s->model[run.small].predict(run.cells, &dur)) return false;
  return now >= std::max(run.t_launch, s->t_gpu_free) + dur - s->lead_s;
}

// Build and launch one step from the admitted requests (scheduler thread, lock held).
bool launch_step(sw_server *s) {
  StepSlot &st = s->slots[s->next_slot];
  const double t_begin = now_s();
  if (st.busy || s->admitted.empty() || !may_launch(s, t_begin)) return false;
  const int64_t max_reads = s->opts.max_step_reads, max_cals = s->opts.max_step_cals;
  const int64_t max_words = max_reads * ((s->mode.max_read_len + 15) / 16);
  // pass 1: which reads of which requests go into the step
  int64_t nr = 0, nc = 0, nw = 0;
  st.parts.clear();
  st.part_r0.clear();
  for (auto &rq : s->admitted) {
    if ((int64_t)st.parts.size() >= s->opts.max_step_chunks) break;
    Request &r = *rq;
    const int64_t r0 = r.next_read;
    int64_t r1 = r0;
    // take whole reads while the step has room (a single read always fits an
    // empty step: submit bounds the CALs of one read by the step capacity)
    while (r1 < r.n_reads && nr + (r1 - r0) < max_reads) {
      if (nc + (r.cal_ptr[r1 + 1] - r.cal_ptr[r0]) > max_cals) break;
      if (nw + (r.wptr[r1 + 1] - r.wptr[r0]) > max_words) break;
      ++r1;
    }
    if (r1 == r0) break;
    nr += r1 - r0;
    nc += r.cal_ptr[r1] - r.cal_ptr[r0];
    nw += r.wptr[r1] - r.wptr[r0];
    r.next_read = r1;
    st.parts.emplace_back(rq, r1 - r0);
    st.part_r0.push_back(r0);
  }
  while (!s->admitted.empty() && s->admitted.front()->next_read >= s->admitted.front()->n_reads)
    s->admitted.pop_front();
  const int nch = (int)st.parts.size();
  if (nch == 0) return false;
  // pass 2: the step header, from the host copies of the requests' read lengths
  // and CAL rows; every chunk address is offset on the host
  const StepHeader H = header_layout(nr, nch);
  int32_t *h_len = reinterpret_cast<int32_t *>(st.hdr_host + H.len);
  int64_t *h_wo = reinterpret_cast<int64_t *>(st.hdr_host + H.word_off);
  int64_t *h_cp = reinterpret_cast<int64_t *>(st.hdr_host + H.cal_ptr);
  swk::ServeChunk *h_ch = reinterpret_cast<swk::ServeChunk *>(st.hdr_host + H.chunks);
  int64_t sr = 0, sc = 0, sw = 0;
  double cells = 0;
  const double band2 = 2.0 * s->sc.band;
  for (int k = 0; k < nch; ++k) {
    Request &r = *st.parts[k].first;
    const int64_t r0 = st.part_r0[k], r1 = r0 + st.parts[k].second;
    const int64_t c0 = r.cal_ptr[r0], w0 = r.wptr[r0];
    for (int64_t i = r0; i < r1; ++i) {
      h_len[sr + (i - r0)] = r.len[i];
      h_wo[sr + (i - r0)] = sw + (r.wptr[i] - w0);
      h_cp[sr + (i - r0)] = sc + (r.cal_ptr[i] - c0);
      cells += 2.0 * (double)(r.cal_ptr[i + 1] - r.cal_ptr[i]) * r.len[i] * (r.len[i] + band2);
    }
    swk::ServeChunk &c = h_ch[k];
    c.words = dptr<uint32_t>(s, r, r.lay.words) + w0;
    c.cal_pos = dptr<int64_t>(s, r, r.lay.cal_pos) + c0;
    c.cal_ref = dptr<int16_t>(s, r, r.lay.cal_ref) + c0;
    c.strand = dptr<uint8_t>(s, r, r.lay.strand) + c0;
    c.score = dptr<int32_t>(s, r, r.lay.score) + 2 * c0;
    c.ref_end = dptr<int64_t>(s, r, r.lay.ref_end) + 2 * c0;
    c.read_end = dptr<int16_t>(s, r, r.lay.read_end) + 2 * c0;
    c.best_score = dptr<int32_t>(s, r, r.lay.best_score) + r0 * s->n_refs;
    c.best_slot = dptr<int64_t>(s, r, r.lay.best_slot) + r0 * s->n_refs;
    c.n_tied = dptr<int32_t>(s, r, r.lay.n_tied) + r0 * s->n_refs;
    c.n_reads = r1 - r0;
    c.n_cals = r.cal_ptr[r1] - c0;
    c.n_words = r.wptr[r1] - w0;
    c.step_r0 = sr;
    c.step_c0 = sc;
    c.step_w0 = sw;
    c.slot_shift = 2 * (c0 - sc);
    sr += c.n_reads;
    sc += c.n_cals;
    sw += c.n_words;
  }
  h_cp[nr] = nc;
  hipStream_t cs = st.stream;
  const int32_t *d_len = reinterpret_cast<const int32_t *>(st.hdr_dev + H.len);
  const int64_t *d_wo = reinterpret_cast<const int64_t *>(st.hdr_dev + H.word_off);
  const int64_t *d_cp = reinterpret_cast<const int64_t *>(st.hdr_dev + H.cal_ptr);
  const swk::ServeChunk *d_ch = reinterpret_cast<const swk::ServeChunk *>(st.hdr_dev + H.chunks);
  hipError_t he = hipMemcpyAsync(st.hdr_dev, st.hdr_host, H.bytes, hipMemcpyHostToDevice, cs);
  if (he == hipSuccess) he = swk::launch_serve_gather(d_ch, nch, nw, nc, st.words, st.cal_pos, st.cal_ref, st.strand, cs);
  int rc = he == hipSuccess ? SW_OK : swapi::hip_fail(he);
  st.small = nc > 0 && nc <= s->small_step_cals;
  st.cells = cells;
  st.t_launch = t_begin;
  if (rc == SW_OK && st.small) {
    // a small step: the plain call, whose AUTO kernel choice runs one wavefront
    // per task (a lane working through a whole long read alone would set the
    // latency); the outputs are the same
    rc = sw_align_batch(st.words, d_wo, d_len, (int32_t)nr, &s->refs, d_cp, st.cal_pos,
                        st.cal_ref, st.strand, nc, &s->sc_small, st.score, st.ref_end, st.read_end, st.small_ws,
                        st.small_ws_bytes, (sw_stream_t)cs);
  } else if (rc == SW_OK && nc > 0) {
    rc = sw_align_batch_ctx(st.ctx, st.words, d_wo, d_len, (int32_t)nr, &s->refs, d_cp,
                            st.cal_pos, st.cal_ref, st.strand, nc, &s->sc, st.score, st.ref_end, st.read_end,
                            (sw_stream_t)cs);
  }
  if (rc == SW_OK)
    rc = sw_reduce_best(d_cp, st.cal_ref, (int32_t)nr, s->n_refs, nc, st.score, st.best_score, st.best_slot,
                        st.n_tied, (sw_stream_t)cs);
  st.error = rc;
  if (rc != SW_OK) s->last_error = rc;
  // no scatter without this step's descriptors on the device
  if (he == hipSuccess)
    swk::launch_serve_scatter(d_ch, nch, nr, nc, s->n_refs, st.score, st.ref_end, st.read_end, st.best_score,
                              st.best_slot, st.n_tied, cs);
  hipEventRecord(st.done, cs);
  if (!s->in_flight.empty()) s->steps_early++;
  st.busy = true;
  s->in_flight.push_back(&st);
  s->next_slot = (s->next_slot + 1) % kSlots;
  s->steps++;
  s->step_reads += nr;
  s->step_cals += nc;
  s->lead_s = 0.8 * s->lead_s + 0.2 * (now_s() - t_begin + 1e-4);  // 0.1 ms margin (polling, jitter)
  return true;
}

// Retire finished steps (lock held).  A request whose reads are all done has
// its results in the arena already (written there by the scatter kernels); it
// goes to the finisher thread, so the scheduler keeps launching steps.
void retire_steps(sw_server *s) {
  // steps retire in launch order (a request's chunks complete in order)
  int n_retired = 0;
  while (!s->in_flight.empty() && hipEventQuery(s->in_flight.front()->done) == hipSuccess) {
    StepSlot &st = *s->in_flight.front();
    s->in_flight.pop_front();
    // device time as seen from here: from its launch, or from the end of the step
    // ahead of it, to now (a second step found done in the same pass has no
    // separate end, and gives no sample)
    const double t = now_s();
    if (n_retired++ == 0 && st.cells > 0) s->model[st.small].add(st.cells, t - std::max(st.t_launch, s->t_gpu_free));
    s->t_gpu_free = t;
    for (auto &p : st.parts) {
      Request &r = *p.first;
      r.reads_done += p.second;
      if (st.error && !r.error) r.error = st.error;
      if (r.reads_done == r.n_reads) {
        s->to_finish.push_back(p.first);
        s->finishing++;
        s->cv_fin.notify_one();
      }
    }
    st.parts.clear();
    st.busy = false;
  }
}

// Finisher thread: copy the results of finished requests to the callers'
// buffers (lock not held: the blocks stay reserved until the copies end), then
// free the blocks and mark the requests done.  Ends once the scheduler has
// ended and nothing is left to finish.
void finish_loop(sw_server *s) {
  std::unique_lock<std::mutex> lk(s->mu);
  std::vector<std::shared_ptr<Request>> done;
  while (true) {
    s->cv_fin.wait(lk, [&] { return !s->to_finish.empty() || !s->worker_running; });
    if (s->to_finish.empty()) break;
    done.assign(s->to_finish.begin(), s->to_finish.end());
    s->to_finish.clear();
    lk.unlock();
    for (auto &rq : done) {
      Request &r = *rq;
      if (r.error) continue;  // failed: the caller's buffers are left as they were
      if (r.n_cals > 0) {
        std::memcpy(r.o_score, hptr<int32_t>(s, r, r.lay.score), sizeof(int32_t) * 2 * r.n_cals);
        std::memcpy(r.o_ref_end, hptr<int64_t>(s, r, r.lay.ref_end), sizeof(int64_t) * 2 * r.n_cals);
        std::memcpy(r.o_read_end, hptr<int16_t>(s, r, r.lay.read_end), sizeof(int16_t) * 2 * r.n_cals);
      }
      if (r.o_best_score)
        std::memcpy(r.o_best_score, hptr<int32_t>(s, r, r.lay.best_score), sizeof(int32_t) * r.n_reads * s->n_refs);
      if (r.o_best_slot)
        std::memcpy(r.o_best_slot, hptr<int64_t>(s, r, r.lay.best_slot), sizeof(int64_t) * r.n_reads * s->n_refs);
      if (r.o_n_tied)
        std::memcpy(r.o_n_tied, hptr<int32_t>(s, r, r.lay.n_tied), sizeof(int32_t) * r.n_reads * s->n_refs);
    }
    const double t = now_s();
    lk.lock();
    for (auto &rq : done) {
      SW_SERVE_MARK_BLOCK(s->arena_host + rq->off, up256(rq->lay.total), 0);
      s->arena->release(rq->off, rq->lay.total);
      rq->t_done = t;
      rq->state = rq->error ? RS_FAILED : RS_DONE;
      s->finishing--;
    }
    done.clear();
    s->cv_done.notify_all();
    s->cv_work.notify_one();  // freed blocks may admit waiting requests
  }
}

void serve_loop(sw_server *s) {
  hipSetDevice(s->opts.device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    while (!s->pending.empty()) {  // admission, in arrival order
      if (!admit(s, s->pending.front())) break;
      s->admitted.push_back(s->pending.front());
      s->pending.pop_front();
    }
    while (launch_step(s)) {
    }
    retire_steps(s);
    const bool idle = s->pending.empty() && s->admitted.empty() && s->in_flight.empty() && s->finishing == 0;
    if (s->stop && idle) break;
    if (idle)
      s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    else
      s->cv_work.wait_for(lk, std::chrono::microseconds(50));
  }
  s->worker_running = false;  // every request is done: the finisher may end
  s->cv_fin.notify_all();
}

}  // namespace

extern "C" {

int sw_server_create(const sw_server_opts_t *opts, sw_server_t **out) {
  if (!opts || !out) return SW_ERR_INVALID_ARG;
  *out = nullptr;
  swapi::ScoreMode m;
  int rc = swapi::validate_scoring(&opts->scoring, &m);
  if (rc) return rc;
  if (opts->memory_budget < (1 << 20) || opts->max_step_reads < 1 || opts->max_step_cals < 1 ||
      opts->max_step_chunks < 1 || opts->max_step_chunks > 4096 || opts->max_steps_in_flight < 0 ||
      opts->max_steps_in_flight > kSlots)
    return SW_ERR_INVALID_ARG;
  hipError_t e = hipSetDevice(opts->device);
  if (e != hipSuccess) return swapi::hip_fail(e);
  auto *s = new (std::nothrow) sw_server();
  if (!s) return SW_ERR_NOMEM;
  s->opts = *opts;
  s->sc = opts->scoring;
  s->mode = m;
  s->sc_small = opts->scoring;
  s->sc_small.kernel = SW_KERNEL_AUTO;
  // steps small enough for the AUTO rule's one-wavefront-per-task kernel (one
  // wavefront per CAL in int16 pairs, two in int32) take the plain call; with a
  // fixed kernel family every step stays on the batched path
  s->small_step_cals = opts->scoring.kernel != SW_KERNEL_AUTO
                           ? 0
                           : (int64_t)swapi::kIntraWavesPerCu * swapi::device_cus() / (m.int16 ? 1 : 2);
  s->arena.reset(new Arena(opts->memory_budget));
  // coherent: blocks are rewritten by the host for each new request, and the
  // device must never see a previous request's bytes through its caches
  if (hipHostMalloc((void **)&s->arena_host, opts->memory_budget, hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess) {
    sw_server_destroy(s);
    return SW_ERR_NOMEM;
  }
  if ((e = hipHostGetDevicePointer((void **)&s->arena_map, s->arena_host, 0)) != hipSuccess) {
    sw_server_destroy(s);
    return swapi::hip_fail(e);
  }
  SW_SERVE_MARK_BLOCK(s->arena_host, opts->memory_budget, 0);
  const int64_t R = opts->max_step_reads, C = opts->max_step_cals;
  const int64_t W = R * ((m.max_read_len + 15) / 16);
  for (auto &st : s->slots) {
    size_t o = 0;
    auto take = [&](size_t b) {
      size_t r = o;
      o = up256(o + b);
      return r;
    };
    const size_t o_words = take(4 * W), o_pos = take(8 * C), o_ref = take(2 * C), o_str = take(C),
                 o_sc = take(4 * 2 * C), o_re = take(8 * 2 * C), o_qe = take(2 * 2 * C),
                 o_bs = take(4 * R * SW_MAX_REFS), o_bl = take(8 * R * SW_MAX_REFS), o_nt = take(4 * R * SW_MAX_REFS);
    const size_t hdr = header_layout(R, opts->max_step_chunks).bytes;
    if (hipMalloc(&st.base, o) != hipSuccess || hipMalloc((void **)&st.hdr_dev, hdr) != hipSuccess ||
        hipHostMalloc((void **)&st.hdr_host, hdr, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess ||
        (&st == &s->slots[0] ? hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking)
                             : (st.stream = s->slots[0].stream, hipSuccess)) != hipSuccess) {  // shared
      sw_server_destroy(s);
      return SW_ERR_NOMEM;
    }
    char *b = (char *)st.base;
    st.words = (uint32_t *)(b + o_words);
    st.cal_pos = (int64_t *)(b + o_pos);
    st.cal_ref = (int16_t *)(b + o_ref);
    st.strand = (uint8_t *)(b + o_str);
    st.score = (int32_t *)(b + o_sc);
    st.ref_end = (int64_t *)(b + o_re);
    st.read_end = (int16_t *)(b + o_qe);
    st.best_score = (int32_t *)(b + o_bs);
    st.best_slot = (int64_t *)(b + o_bl);
    st.n_tied = (int32_t *)(b + o_nt);
  }
  sw_ctx_opts_t co{};
  co.device = opts->device;
  co.max_reads = (int32_t)R;
  co.max_cals = C;
  co.use_graph = 0;  // step shapes change every step
  co.autotune = opts->autotune;
  co.tune_cache = nullptr;
  for (auto &st : s->slots) {
    rc = sw_ctx_create(&co, &st.ctx);
    if (rc) {
      sw_server_destroy(s);
      return rc;
    }
    if (s->small_step_cals > 0) {
      st.small_ws_bytes = sw_workspace_bytes((int32_t)R, s->small_step_cals, &s->sc_small);
      if (hipMalloc(&st.small_ws, std::max<size_t>(st.small_ws_bytes, 256)) != hipSuccess) {
        sw_server_destroy(s);
        return SW_ERR_NOMEM;
      }
    }
  }
  *out = s;
  return SW_OK;
}

int sw_server_set_refs(sw_server_t *s, const sw_refset_t *refs) {
  if (!s) return SW_ERR_INVALID_ARG;
  swk::RefTable T;
  int rc = swapi::validate_refs(refs, 1, &T);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->worker.joinable()) return SW_ERR_STATE;  // references are fixed once serving starts
  s->ref_off.assign(refs->word_offset, refs->word_offset + refs->n_refs);
  s->ref_len.assign(refs->length, refs->length + refs->n_refs);
  s->refs.words = refs->words;
  s->refs.word_offset = s->ref_off.data();
  s->refs.length = s->ref_len.data();
  s->refs.n_refs = refs->n_refs;
  s->n_refs = refs->n_refs;
  s->refs_set = true;
  s->worker_running = true;
  s->worker = std::thread(serve_loop, s);
  s->finisher = std::thread(finish_loop, s);
  return SW_OK;
}

int sw_server_submit(sw_server_t *s, const uint8_t *read_codes, int64_t n_codes, const int64_t *read_code_off,
                     const int32_t *read_len, int32_t n_reads, const int64_t *cal_ptr, const int64_t *cal_pos,
                     const int16_t *cal_ref, const uint8_t *strand, int64_t n_cals, int32_t *score, int64_t *ref_end,
                     int16_t *read_end, int32_t *best_score, int64_t *best_slot, int32_t *n_tied, int64_t *req_id) {
  const double t = now_s();
  if (!s || !req_id) return SW_ERR_INVALID_ARG;
  if (!s->refs_set) return SW_ERR_STATE;
  if (n_reads < 1 || n_cals < 0 || n_codes < 0) return SW_ERR_INVALID_ARG;
  if (!read_codes || !read_code_off || !read_len || !cal_ptr) return SW_ERR_INVALID_ARG;
  if (n_cals > 0 && (!cal_pos || !cal_ref || !strand || !score || !ref_end || !read_end)) return SW_ERR_INVALID_ARG;
  if (n_reads > s->opts.max_step_reads) return SW_ERR_INVALID_ARG;
  if (cal_ptr[0] != 0 || cal_ptr[n_reads] != n_cals) return SW_ERR_INVALID_ARG;
  for (int32_t i = 0; i < n_reads; ++i) {
    if (cal_ptr[i + 1] < cal_ptr[i]) return SW_ERR_INVALID_ARG;
    if (cal_ptr[i + 1] - cal_ptr[i] > s->opts.max_step_cals) return SW_ERR_INVALID_ARG;
    if (read_code_off[i] < 0 || read_len[i] < 0 || read_len[i] > s->mode.max_read_len ||
        read_code_off[i] + read_len[i] > n_codes)
      return SW_ERR_INVALID_ARG;
  }
  auto rq = std::make_shared<Request>();
  Request &r = *rq;
  r.n_reads = n_reads;
  r.n_cals = n_cals;
  r.n_codes = n_codes;
  // the step builder works from host copies of the read lengths, the packed
  // word offsets (reads back to back in the arena) and the CAL rows
  r.len.assign(read_len, read_len + n_reads);
  r.cal_ptr.assign(cal_ptr, cal_ptr + n_reads + 1);
  r.wptr.resize((size_t)n_reads + 1);
  r.wptr[0] = 0;
  for (int32_t i = 0; i < n_reads; ++i) r.wptr[i + 1] = r.wptr[i] + (read_len[i] + 15) / 16;
  r.lay = make_layout(n_reads, n_cals, r.wptr[n_reads], s->n_refs);
  if (r.lay.total > s->arena->size()) return SW_ERR_REJECTED;
  bool reserved = false;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    // reserve now if nobody waits ahead (arrival order) and memory is free
    if (s->pending.empty()) reserved = s->arena->alloc(r.lay.total, &r.off);
    if (reserved) SW_SERVE_MARK_BLOCK(s->arena_host + r.off, up256(r.lay.total), 1);
  }
  if (reserved) {
    // the caller's thread stages its own inputs (reads packed) into the pinned arena
    stage_inputs(s, r, read_codes, read_code_off, cal_pos, cal_ref, strand);
  } else {
    r.codes.assign(read_codes, read_codes + n_codes);
    r.code_off.assign(read_code_off, read_code_off + n_reads);
    if (n_cals) {
      r.cal_pos.assign(cal_pos, cal_pos + n_cals);
      r.cal_ref.assign(cal_ref, cal_ref + n_cals);
      r.strand.assign(strand, strand + n_cals);
    }
  }
  r.o_score = score;
  r.o_ref_end = ref_end;
  r.o_read_end = read_end;
  r.o_best_score = best_score;
  r.o_best_slot = best_slot;
  r.o_n_tied = n_tied;
  r.t_submit = t;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      if (reserved) {
        SW_SERVE_MARK_BLOCK(s->arena_host + r.off, up256(r.lay.total), 0);
        s->arena->release(r.off, r.lay.total);
      }
      return SW_ERR_STATE;
    }
    r.id = s->next_id++;
    s->pending.push_back(rq);
    s->all[r.id] = rq;
  }
  s->cv_work.notify_one();
  *req_id = r.id;
  return SW_OK;
}

int sw_server_wait(sw_server_t *s, int64_t req_id, int32_t timeout_ms, int32_t *done) {
  if (!s || !done) return SW_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(req_id);
  if (it == s->all.end()) return SW_ERR_INVALID_ARG;
  auto rq = it->second;
  auto pred = [&] { return rq->state == RS_DONE || rq->state == RS_FAILED; };
  if (timeout_ms < 0)
    s->cv_done.wait(lk, pred);
  else
    s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
  *done = pred() ? 1 : 0;
  return rq->state == RS_FAILED ? rq->error : SW_OK;
}

int sw_server_request_info(sw_server_t *s, int64_t req_id, int32_t *state, double *t_submit, double *t_admit,
                           double *t_done) {
  if (!s) return SW_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(req_id);
  if (it == s->all.end()) return SW_ERR_INVALID_ARG;
  const Request &r = *it->second;
  if (state) *state = r.state;
  if (t_submit) *t_submit = r.t_submit;
  if (t_admit) *t_admit = r.t_admit;
  if (t_done) *t_done = r.t_done;
  return SW_OK;
}

int sw_server_release(sw_server_t *s, int64_t req_id) {
  if (!s) return SW_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(req_id);
  if (it == s->all.end()) return SW_ERR_INVALID_ARG;
  if (it->second->state != RS_DONE && it->second->state != RS_FAILED) return SW_ERR_STATE;
  s->all.erase(it);
  return SW_OK;
}

int sw_server_stats(sw_server_t *s, sw_server_stats_t *out) {
  if (!s || !out) return SW_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  out->steps = s->steps;
  out->step_reads = s->step_reads;
  out->step_cals = s->step_cals;
  out->pending = (int64_t)s->pending.size();
  out->in_flight_requests = (int64_t)s->admitted.size();
  out->arena_used = (int64_t)s->arena->used();
  out->arena_size = (int64_t)s->arena->size();
  out->steps_launched_early = s->steps_early;
  return s->last_error ? s->last_error : SW_OK;
}

int sw_server_destroy(sw_server_t *s) {
  if (!s) return SW_OK;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->worker.join();  // drains every submitted request first
    if (s->finisher.joinable()) s->finisher.join();
  }
  hipSetDevice(s->opts.device);
  for (auto &st : s->slots)
    if (st.stream) hipStreamSynchronize(st.stream);
  for (auto &st : s->slots) {
    if (st.ctx) sw_ctx_destroy(st.ctx);
    if (st.small_ws) hipFree(st.small_ws);
    if (st.stream && &st == &s->slots[0]) hipStreamDestroy(st.stream);
    if (st.base) hipFree(st.base);
    if (st.hdr_dev) hipFree(st.hdr_dev);
    if (st.hdr_host) hipHostFree(st.hdr_host);
    if (st.done) hipEventDestroy(st.done);
  }
  if (s->arena_host) {
    SW_SERVE_MARK_BLOCK(s->arena_host, s->opts.memory_budget, 1);
    hipHostFree(s->arena_host);
  }
  delete s;
  return SW_OK;
}

}  // extern "C"
