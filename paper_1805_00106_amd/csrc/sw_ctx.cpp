// Batched execution context: length-binned persistent work queue, captured
// HIP graphs per call shape, and a small autotuner over the binning plan.
// Contracts are in include/sw_align.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/sw_align.h"
#include "sw_api_internal.h"
#include "sw_launch.h"

namespace {

// One batched plan: how tasks are binned and ordered, which strip height each
// bin takes, and how many persistent blocks pop the queue.
struct TunedPlan {
  int unbinned = 0;       // 1: no bins, tasks in input order, one strip height (the plain kernel)
  int bin_width = 4;
  int descending = 1;
  int strip_cap = 0;      // tallest strip height a bin may take (0: any)
  int strip_slack = 0;    // padding rows accepted to save one strip hand-over
  int grid_quarters = 4;  // persistent blocks, in quarters of the resident capacity
  float ms = 0.f;
};

struct GraphEntry {
  std::string key;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

const int kQueueStrips16[] = {
#define SW_LIST(RR) RR,
    SW_QUEUE16_STRIPS(SW_LIST)
#undef SW_LIST
};
const int kQueueStrips32[] = {
#define SW_LIST(RR) RR,
    SW_QUEUE32_STRIPS(SW_LIST)
#undef SW_LIST
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct sw_ctx {
  int device = 0;
  int32_t max_reads = 0;
  int64_t max_cals = 0;
  bool use_graph = true;
  bool autotune = true;
  std::string tune_cache;
  hipStream_t stream = nullptr;  // graphs are captured and replayed here
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  void *buf = nullptr;  // planning and order buffers, sized for the capacity
  swk::BatchBufs B{};
  unsigned long long *err = nullptr;
  uint2 *scratch = nullptr;
  size_t scratch_bytes = 0;
  std::map<std::string, TunedPlan> tuned;
  std::vector<GraphEntry> graphs;
  uint64_t clock = 0;
  std::string last_plan;
};

namespace {

int hip_rc(hipError_t e) { return e == hipSuccess ? SW_OK : swapi::hip_fail(e); }

void load_tune_cache(sw_ctx *c) {
  if (c->tune_cache.empty()) return;
  FILE *f = std::fopen(c->tune_cache.c_str(), "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    // one entry per line: "key": {"unbinned": N, "bin_width": N, "descending": N,
    // "strip_cap": N, "strip_slack": N, "grid_quarters": N, "ms": X}
    char key[256];
    TunedPlan p;
    if (std::sscanf(line,
                    " \"%255[^\"]\": {\"unbinned\": %d, \"bin_width\": %d, \"descending\": %d, "
                    "\"strip_cap\": %d, \"strip_slack\": %d, \"grid_quarters\": %d, \"ms\": %f",
                    key, &p.unbinned, &p.bin_width, &p.descending, &p.strip_cap, &p.strip_slack, &p.grid_quarters,
                    &p.ms) == 8 &&
        (p.unbinned == 0 || p.unbinned == 1) && p.bin_width >= 1 && p.bin_width <= SW_MAX_READ_LEN &&
        p.grid_quarters >= 1 && p.grid_quarters <= 4 && p.strip_cap >= 0 && p.strip_slack >= 0)
      c->tuned[key] = p;
  }
  std::fclose(f);
}

void save_tune_cache(const sw_ctx *c) {
  if (c->tune_cache.empty()) return;
  FILE *f = std::fopen(c->tune_cache.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (const auto &kv : c->tuned) {
    const TunedPlan &t = kv.second;
    std::fprintf(f,
                 "  \"%s\": {\"unbinned\": %d, \"bin_width\": %d, \"descending\": %d, \"strip_cap\": %d, "
                 "\"strip_slack\": %d, \"grid_quarters\": %d, \"ms\": %.4f}%s\n",
                 kv.first.c_str(), t.unbinned, t.bin_width, t.descending, t.strip_cap, t.strip_slack,
                 t.grid_quarters, t.ms,
                 ++i < c->tuned.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  std::fclose(f);
}

struct CallArgs {
  const uint32_t *reads2bit;
  const int64_t *read_word_off;
  const int32_t *read_len;
  int32_t n_reads;
  const sw_refset_t *refs;
  const int64_t *cal_ptr, *cal_pos;
  const int16_t *cal_ref;
  const uint8_t *strand;
  int64_t n_cals;
  const sw_scoring_t *sc;
  int32_t *score;
  int64_t *ref_end;
  int16_t *read_end;
};

swk::BinParams bin_params(const swapi::ScoreMode &m, const TunedPlan &t) {
  swk::BinParams P{};
  P.bin_width = t.bin_width;
  P.max_read_len = m.max_read_len;
  P.nb = (m.max_read_len + t.bin_width - 1) / t.bin_width;
  P.per_cal = m.int16 ? 1 : 2;
  P.descending = t.descending;
  const int *s = m.int16 ? kQueueStrips16 : kQueueStrips32;
  const int n = m.int16 ? (int)(sizeof(kQueueStrips16) / sizeof(int)) : (int)(sizeof(kQueueStrips32) / sizeof(int));
  P.n_strips = 0;
  for (int i = 0; i < n; ++i) P.strips[P.n_strips++] = s[i];
  P.strip_cap = t.strip_cap;
  P.strip_slack = t.strip_slack;
  return P;
}

// The strip height of every length bin under plan t, as "lo-hi:R" runs.
std::string plan_heights(const swk::BinParams &P) {
  std::string out;
  int run_lo = 1, run_r = -1;
  for (int b = 0; b < P.nb; ++b) {
    const int lo = b * P.bin_width + 1, hi = std::min((b + 1) * P.bin_width, P.max_read_len);
    const int R = swk::bin_strip_height(P, hi);
    if (R != run_r) {
      if (run_r > 0) out += std::to_string(run_lo) + "-" + std::to_string(lo - 1) + ":" + std::to_string(run_r) + " ";
      run_lo = lo;
      run_r = R;
    }
  }
  if (run_r > 0) out += std::to_string(run_lo) + "-" + std::to_string(P.max_read_len) + ":" + std::to_string(run_r);
  return out;
}

int queue_grid(bool int16, int64_t n_tasks) {
  static int occ[2] = {0, 0};
  int &o = occ[int16 ? 1 : 0];
  if (!o) {
    o = swk::queue_blocks_per_cu(int16);
    if (o <= 0) o = 2;
  }
  const int64_t resident = (int64_t)swapi::device_cus() * o;
  const int64_t tiles = (n_tasks + 63) / 64 + 1;
  return (int)std::max<int64_t>(1, std::min<int64_t>(resident, tiles));
}

// Enqueue the whole batched pipeline on `st` (capturable: kernels only).
int enqueue(sw_ctx *c, const CallArgs &a, const swapi::ScoreMode &m, const swk::RefTable &T, const TunedPlan &t,
            int grid, hipStream_t st) {
  const int64_t n_tasks = m.int16 ? a.n_cals : 2 * a.n_cals;
  // the invalid-task counter reports the last call (a fill kernel, so the reset is capturable)
  hipError_t e = swk::launch_fill_i32(reinterpret_cast<int32_t *>(c->err), 2, 0, st);
  if (e != hipSuccess) return swapi::hip_fail(e);
  e = swk::launch_expand(a.cal_ptr, a.n_reads, a.n_cals, c->B.cal_read, st);
  if (e != hipSuccess) return swapi::hip_fail(e);
  if (!t.unbinned) {
    const swk::BinParams P = bin_params(m, t);
    e = swk::launch_batch_plan(c->B, a.read_len, a.n_reads, n_tasks, P, st);
  } else {
    e = swk::launch_fill_i32(c->B.queue, 1, 0, st);  // the tile counter, in input order
  }
  if (e != hipSuccess) return swapi::hip_fail(e);
  swk::AlignArgs A{};
  A.reads = a.reads2bit;
  A.read_word_off = a.read_word_off;
  A.read_len = a.read_len;
  A.n_reads = a.n_reads;
  A.n_refs = a.refs->n_refs;
  A.ref_words = a.refs->words;
  A.cal_pos = a.cal_pos;
  A.cal_ref = a.cal_ref;
  A.strand = a.strand;
  A.cal_read = c->B.cal_read;
  A.order = c->B.order;
  A.n_cals = a.n_cals;
  A.n_tasks = n_tasks;
  A.score = a.score;
  A.ref_end = a.ref_end;
  A.read_end = a.read_end;
  A.scratch = c->scratch;
  A.err = c->err;
  A.tiles = c->B.tiles;
  A.tile_len = c->B.tile_len;
  A.tile_strips = c->B.tile_strips;
  A.queue = c->B.queue;
  A.n_tiles_dev = c->B.n_tiles;
  A.wcap = m.wcap;
  A.wwords = (m.wcap + 15) / 16;
  A.rwords = (m.max_read_len + 15) / 16;
  A.max_read_len = m.max_read_len;
  A.band = a.sc->band;
  A.strip_rows = 0;
  A.k = swapi::make_consts(a.sc);
  if (t.unbinned) {
    // the plain kernel, its tiles 64 consecutive tasks popped from the counter
    A.order = nullptr;
    A.tiles = nullptr;
    A.tile_len = nullptr;
    A.tile_strips = nullptr;
    A.n_tiles_dev = nullptr;
    A.strip_rows = swapi::choose_strip_rows(m.int16, m.max_read_len);
    e = swk::launch_inter(m.int16, A, T, grid, st);
  } else {
    e = swk::launch_inter_queue(m.int16, A, T, grid, st);
  }
  if (e != hipSuccess) return swapi::hip_fail(e);
  return SW_OK;
}

std::string graph_key(const CallArgs &a, const swapi::ScoreMode &m, const TunedPlan &t, int grid) {
  char k[1024];
  std::snprintf(k, sizeof k, "%p %p %p %d %p %d %p %p %p %p %p %lld %d %d %d %d %d %d %p %p %p %d %d %d %d %d %d %d %d",
                (const void *)a.reads2bit, (const void *)a.read_word_off, (const void *)a.read_len, a.n_reads,
                (const void *)a.refs->words, a.refs->n_refs, (const void *)a.cal_ptr, (const void *)a.cal_pos,
                (const void *)a.cal_ref, (const void *)a.strand, (const void *)a.score, (long long)a.n_cals,
                a.sc->match, a.sc->mismatch, a.sc->gap_open, a.sc->gap_extend, a.sc->band, m.max_read_len,
                (const void *)a.ref_end, (const void *)a.read_end, (const void *)nullptr, (int)m.int16, t.bin_width,
                t.descending, grid, a.sc->mode, t.strip_cap, t.strip_slack, t.unbinned);
  std::string s(k);
  for (int i = 0; i < a.refs->n_refs; ++i) {
    char r[64];
    std::snprintf(r, sizeof r, " %lld:%lld", (long long)a.refs->word_offset[i], (long long)a.refs->length[i]);
    s += r;
  }
  return s;
}

std::string tune_key(const swapi::ScoreMode &m, const sw_scoring_t *sc, int64_t n_tasks) {
  char k[128];
  std::snprintf(k, sizeof k, "gfx950/%s%s/L%d/b%d/t%d", m.int16 ? "int16" : "int32",
                sc->mode == SW_MODE_FINAL_ROW ? "-final-row" : "", m.max_read_len, sc->band,
                (int)std::floor(std::log2((double)std::max<int64_t>(n_tasks, 1))));
  return k;
}

}  // namespace

extern "C" {

int sw_ctx_create(const sw_ctx_opts_t *opts, sw_ctx_t **out) {
  if (!opts || !out) return SW_ERR_INVALID_ARG;
  *out = nullptr;
  if (opts->max_reads < 0 || opts->max_cals < 0 || opts->device < 0) return SW_ERR_INVALID_ARG;
  // the planner keeps task positions (up to two per CAL) in int32
  if (opts->max_cals > (int64_t)INT32_MAX / 2) return SW_ERR_INVALID_ARG;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return swapi::hip_fail(e);
  if (opts->device >= ndev) return SW_ERR_INVALID_ARG;
  e = hipSetDevice(opts->device);
  if (e != hipSuccess) return swapi::hip_fail(e);
  sw_ctx *c = new (std::nothrow) sw_ctx();
  if (!c) return SW_ERR_NOMEM;
  c->device = opts->device;
  c->max_reads = opts->max_reads;
  c->max_cals = std::max<int64_t>(opts->max_cals, 1);
  c->use_graph = opts->use_graph != 0;
  c->autotune = opts->autotune != 0;
  if (opts->tune_cache) c->tune_cache = opts->tune_cache;
  // capacity buffers: per-task arrays for the int32 task count (2 per CAL)
  const int64_t max_tasks = 2 * c->max_cals;
  const int64_t max_tiles = (max_tasks + 63) / 64 + SW_MAX_READ_LEN + 2;
  const int64_t nbins = SW_MAX_READ_LEN + 2;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_cal_read = take(sizeof(int32_t) * c->max_cals);
  const size_t o_order = take(sizeof(int32_t) * max_tasks);
  const size_t o_bins = take(sizeof(int32_t) * nbins * 6);
  const size_t o_tiles = take(sizeof(int32_t) * max_tiles * 3);
  const size_t o_misc = take(256);
  const size_t o_err = take(sizeof(unsigned long long));
  e = hipMalloc(&c->buf, off);
  if (e != hipSuccess) {
    delete c;
    return SW_ERR_NOMEM;
  }
  char *b = (char *)c->buf;
  c->B.cal_read = (int32_t *)(b + o_cal_read);
  c->B.order = (int32_t *)(b + o_order);
  int32_t *bins = (int32_t *)(b + o_bins);
  c->B.bin_count = bins;
  c->B.bin_off = bins + nbins;
  c->B.bin_cursor = bins + 2 * nbins;
  c->B.tile_off = bins + 3 * nbins;
  c->B.tile_bin = bins + 4 * nbins;
  c->B.strip_of_bin = bins + 5 * nbins;
  int32_t *tl = (int32_t *)(b + o_tiles);
  c->B.tiles = tl;
  c->B.tile_len = tl + max_tiles;
  c->B.tile_strips = tl + 2 * max_tiles;
  c->B.n_tiles = (int32_t *)(b + o_misc);
  c->B.queue = (int32_t *)(b + o_misc) + 1;
  c->err = (unsigned long long *)(b + o_err);
  if ((e = hipMemset(c->err, 0, sizeof(unsigned long long))) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreate(&c->ev_t0)) != hipSuccess || (e = hipEventCreate(&c->ev_t1)) != hipSuccess) {
    sw_ctx_destroy(c);
    return swapi::hip_fail(e);
  }
  load_tune_cache(c);
  *out = c;
  return SW_OK;
}

int sw_ctx_destroy(sw_ctx_t *c) {
  if (!c) return SW_OK;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  for (auto &g : c->graphs)
    if (g.exec) hipGraphExecDestroy(g.exec);
  if (c->scratch) hipFree(c->scratch);
  if (c->buf) hipFree(c->buf);
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  if (c->ev_t0) hipEventDestroy(c->ev_t0);
  if (c->ev_t1) hipEventDestroy(c->ev_t1);
  if (c->stream) hipStreamDestroy(c->stream);
  delete c;
  return SW_OK;
}

int sw_align_batch_ctx(sw_ctx_t *c, const uint32_t *reads2bit, const int64_t *read_word_off, const int32_t *read_len,
                       int32_t n_reads, const sw_refset_t *refs, const int64_t *cal_ptr, const int64_t *cal_pos,
                       const int16_t *cal_ref, const uint8_t *strand, int64_t n_cals, const sw_scoring_t *sc,
                       int32_t *score, int64_t *ref_end, int16_t *read_end, sw_stream_t stream) {
  if (!c) return SW_ERR_INVALID_ARG;
  swapi::ScoreMode m;
  int rc = swapi::validate_scoring(sc, &m);
  if (rc) return rc;
  rc = swapi::validate_batch(reads2bit, read_word_off, read_len, n_reads, cal_ptr, cal_pos, cal_ref, strand, n_cals,
                             score, ref_end, read_end);
  if (rc) return rc;
  swk::RefTable T;
  rc = swapi::validate_refs(refs, n_cals, &T);
  if (rc) return rc;
  // within the capacity, which also keeps every task position inside int32
  if (n_reads > c->max_reads || n_cals > c->max_cals) return SW_ERR_WORKSPACE;
  if (n_cals == 0) return SW_OK;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return swapi::hip_fail(e);
  const int64_t n_tasks = m.int16 ? n_cals : 2 * n_cals;
  const int full_grid = queue_grid(m.int16, n_tasks);
  auto grid_of = [&](const TunedPlan &t) { return std::max(1, full_grid * t.grid_quarters / 4); };
  // scratch for the full resident grid, so that shapes with fewer tiles reuse it
  // (and the graphs captured with it) instead of reallocating
  const size_t need = (size_t)queue_grid(m.int16, INT64_MAX / 4) * (size_t)m.wcap * 64 * sizeof(uint2);
  if (need > c->scratch_bytes) {
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return swapi::hip_fail(e);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return swapi::hip_fail(e);
    if (c->scratch) hipFree(c->scratch);
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    if (hipMalloc(&c->scratch, need) != hipSuccess) return SW_ERR_NOMEM;
    c->scratch_bytes = need;
    // graphs captured with the old scratch pointer are stale
    for (auto &g : c->graphs)
      if (g.exec) hipGraphExecDestroy(g.exec);
    c->graphs.clear();
  }
  CallArgs a{reads2bit, read_word_off, read_len, n_reads, refs, cal_ptr, cal_pos, cal_ref, strand,
             n_cals, sc, score, ref_end, read_end};
  hipStream_t user = (hipStream_t)stream;

  // plan: tuned on first use of this shape class, by coordinate search over the
  // bin width and order, then the strip-height policy, then the grid; each
  // candidate runs the whole pipeline once on the caller's inputs (every plan
  // gives the same outputs)
  const std::string tk = tune_key(m, sc, n_tasks);
  auto it = c->tuned.find(tk);
  bool tuned_now = false;
  int n_tried = 0;
  if (it == c->tuned.end()) {
    TunedPlan best;
    if (c->autotune) {
      float best_ms = 1e30f;
      auto time_plan = [&](const TunedPlan &cand) -> int {
        hipError_t he;
        if ((he = hipEventRecord(c->ev_t0, user)) != hipSuccess) return swapi::hip_fail(he);
        int r = enqueue(c, a, m, T, cand, grid_of(cand), user);
        if (r) return r;
        if ((he = hipEventRecord(c->ev_t1, user)) != hipSuccess) return swapi::hip_fail(he);
        if ((he = hipEventSynchronize(c->ev_t1)) != hipSuccess) return swapi::hip_fail(he);
        float ms = 0.f;
        hipEventElapsedTime(&ms, c->ev_t0, c->ev_t1);
        ++n_tried;
        if (ms < best_ms) {
          best_ms = ms;
          best = cand;
          best.ms = ms;
        }
        return SW_OK;
      };
      for (int w : {1, 2, 4, 8, 16})
        for (int d = 1; d >= 0; --d) {
          TunedPlan cand;
          cand.bin_width = w;
          cand.descending = d;
          if ((rc = time_plan(cand))) return rc;
        }
      {
        // no bins: where the reads have one length, binning only reorders
        TunedPlan cand;
        cand.unbinned = 1;
        if ((rc = time_plan(cand))) return rc;
      }
      const TunedPlan base = best;
      const int strip_policies[][2] = {{0, 8}, {0, 16}, {0, 32}, {40, 0}, {44, 0}};
      for (const auto &sp : strip_policies) {
        if (base.unbinned) break;  // the strip policies shape the bins
        TunedPlan cand = base;
        cand.strip_cap = sp[0];
        cand.strip_slack = sp[1];
        if ((rc = time_plan(cand))) return rc;
      }
      const TunedPlan base2 = best;
      for (int q : {3, 2}) {
        TunedPlan cand = base2;
        cand.grid_quarters = q;
        if ((rc = time_plan(cand))) return rc;
      }
      tuned_now = true;
    }
    it = c->tuned.emplace(tk, best).first;
    if (tuned_now) save_tune_cache(c);
  }
  const TunedPlan plan = it->second;
  const int grid = grid_of(plan);

  bool graph_hit = false;
  if (c->use_graph) {
    const std::string gk = graph_key(a, m, plan, grid);
    GraphEntry *g = nullptr;
    for (auto &x : c->graphs)
      if (x.key == gk) g = &x;
    if (!g) {
      if (c->graphs.size() >= 8) {
        auto lru = std::min_element(c->graphs.begin(), c->graphs.end(),
                                    [](const GraphEntry &p, const GraphEntry &q) { return p.last_use < q.last_use; });
        // a launch of the evicted graph may still be queued on the context stream
        if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return swapi::hip_fail(e);
        hipGraphExecDestroy(lru->exec);
        c->graphs.erase(lru);
      }
      hipGraph_t graph = nullptr;
      if ((e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return swapi::hip_fail(e);
      rc = enqueue(c, a, m, T, plan, grid, c->stream);
      hipError_t ec = hipStreamEndCapture(c->stream, &graph);
      if (rc) {
        if (graph) hipGraphDestroy(graph);
        return rc;
      }
      if (ec != hipSuccess) return swapi::hip_fail(ec);
      GraphEntry ne;
      ne.key = gk;
      e = hipGraphInstantiate(&ne.exec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (e != hipSuccess) return swapi::hip_fail(e);
      c->graphs.push_back(ne);
      g = &c->graphs.back();
    } else {
      graph_hit = true;
    }
    g->last_use = ++c->clock;
    // fork onto the context stream, replay, join back (works for the null stream too)
    if ((e = hipEventRecord(c->ev_fork, user)) != hipSuccess) return swapi::hip_fail(e);
    if ((e = hipStreamWaitEvent(c->stream, c->ev_fork, 0)) != hipSuccess) return swapi::hip_fail(e);
    if ((e = hipGraphLaunch(g->exec, c->stream)) != hipSuccess) return swapi::hip_fail(e);
    if ((e = hipEventRecord(c->ev_join, c->stream)) != hipSuccess) return swapi::hip_fail(e);
    if ((e = hipStreamWaitEvent(user, c->ev_join, 0)) != hipSuccess) return swapi::hip_fail(e);
  } else {
    rc = enqueue(c, a, m, T, plan, grid, user);
    if (rc) return rc;
  }
  char desc[320];
  const int unbinned_rows = swapi::choose_strip_rows(m.int16, m.max_read_len);
  if (plan.unbinned)
    std::snprintf(desc, sizeof desc, "%s tasks=%lld unbinned(input order) grid=%d(%d/4) graph=%s tuned=%s(%.3f ms",
                  m.int16 ? "int16-pairs" : "int32", (long long)n_tasks, grid, plan.grid_quarters,
                  c->use_graph ? (graph_hit ? "replay" : "captured") : "off", tuned_now ? "now" : "cached", plan.ms);
  else
    std::snprintf(desc, sizeof desc,
                  "%s tasks=%lld bins=%d(width %d, %s) strips(cap %d, slack %d) grid=%d(%d/4) graph=%s tuned=%s(%.3f ms",
                  m.int16 ? "int16-pairs" : "int32", (long long)n_tasks,
                  (m.max_read_len + plan.bin_width - 1) / plan.bin_width, plan.bin_width,
                  plan.descending ? "longest first" : "shortest first", plan.strip_cap, plan.strip_slack, grid,
                  plan.grid_quarters, c->use_graph ? (graph_hit ? "replay" : "captured") : "off",
                  tuned_now ? "now" : "cached", plan.ms);
  c->last_plan = desc;
  if (tuned_now) c->last_plan += ", " + std::to_string(n_tried) + " plans";
  c->last_plan += ") heights " + (plan.unbinned ? "1-" + std::to_string(m.max_read_len) + ":" + std::to_string(unbinned_rows)
                                                : plan_heights(bin_params(m, plan)));
  return SW_OK;
}

int sw_ctx_error_count(sw_ctx_t *c, int64_t *n) {
  if (!c || !n) return SW_ERR_INVALID_ARG;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return swapi::hip_fail(e);
  if ((e = hipDeviceSynchronize()) != hipSuccess) return swapi::hip_fail(e);
  unsigned long long v = 0;
  if ((e = hipMemcpy(&v, c->err, sizeof v, hipMemcpyDeviceToHost)) != hipSuccess) return swapi::hip_fail(e);
  *n = (int64_t)v;
  return SW_OK;
}

const char *sw_ctx_last_plan(sw_ctx_t *c) { return c ? c->last_plan.c_str() : ""; }

}  // extern "C"
