// Host test of the served path on the CPU stand-in runtime: several client
// threads submit random requests (reads laid out with gaps and out of order,
// reads of length 0, reads without CALs, requests split over several steps),
// under a staging budget small enough that admission waits and arena blocks are
// reused; every output must be the stub scoring of the request's own inputs.
// Run under the host address and undefined-behaviour sanitizers, it also shows
// that no gather or scatter access leaves its buffers.  TEST INFRASTRUCTURE ONLY.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <sys/resource.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <string>
#include <numeric>
#include <random>
#include <thread>
#include <vector>

#include "../../include/sw_align.h"
#include "stub_score.h"

extern std::atomic<long> g_plain_calls, g_ctx_calls;

namespace {

constexpr int kRefs = 2;
int kMaxLen = 60;

struct Req {
  int n_reads = 0;
  std::vector<uint8_t> codes;
  std::vector<int64_t> code_off, cal_ptr, cal_pos;
  std::vector<int32_t> len;
  std::vector<int16_t> cal_ref;
  std::vector<uint8_t> strand;
  std::vector<int32_t> score, best_score, n_tied;
  std::vector<int64_t> ref_end, best_slot;
  std::vector<int16_t> read_end;
  int64_t id = 0;
};

// layout 0: reads back to back at 16-aligned offsets, in order; 1: 16-aligned
// offsets with gaps, in a shuffled order; 2: any offsets, gaps, shuffled.
Req make_request(std::mt19937_64 &g, int max_reads, int max_cals_per_read, int layout) {
  Req q;
  q.n_reads = 1 + (int)(g() % (uint64_t)max_reads);
  q.len.resize(q.n_reads);
  for (auto &L : q.len) L = (g() % 8 == 0) ? 0 : 1 + (int)(g() % kMaxLen);
  // reads placed in a shuffled order with random gaps between them
  std::vector<int> order(q.n_reads);
  std::iota(order.begin(), order.end(), 0);
  if (layout > 0) std::shuffle(order.begin(), order.end(), g);
  q.code_off.resize(q.n_reads);
  int64_t at = layout == 2 ? (int64_t)(g() % 7) : 0;
  for (int i : order) {
    q.code_off[i] = at;
    at += q.len[i] + (layout > 0 ? (int64_t)(g() % 40) : 0);
    if (layout < 2) at = (at + 15) / 16 * 16;
  }
  q.codes.resize((size_t)at + 1);
  for (auto &c : q.codes) c = (uint8_t)(g() % 4);
  q.cal_ptr.assign(q.n_reads + 1, 0);
  for (int i = 0; i < q.n_reads; ++i) {
    const int n = (g() % 6 == 0) ? 0 : (int)(g() % (uint64_t)(max_cals_per_read + 1));
    q.cal_ptr[i + 1] = q.cal_ptr[i] + n;
  }
  const int64_t nc = q.cal_ptr[q.n_reads];
  q.cal_pos.resize(nc);
  q.cal_ref.resize(nc);
  q.strand.resize(nc);
  for (int64_t c = 0; c < nc; ++c) {
    q.cal_pos[c] = (int64_t)(g() % 100000);
    q.cal_ref[c] = (int16_t)(g() % kRefs);
    q.strand[c] = (uint8_t)(1 + g() % 3);
  }
  q.score.assign(2 * nc, -7);
  q.ref_end.assign(2 * nc, -7);
  q.read_end.assign(2 * nc, -7);
  q.best_score.assign(q.n_reads * kRefs, -7);
  q.best_slot.assign(q.n_reads * kRefs, -7);
  q.n_tied.assign(q.n_reads * kRefs, -7);
  return q;
}

// Expected outputs from the request's own inputs; returns the number of mismatches.
long check(const Req &q) {
  long bad = 0;
  for (int r = 0; r < q.n_reads; ++r) {
    const uint64_t rh = stub_read_hash(q.codes.data() + q.code_off[r], q.len[r]);
    for (int k = 0; k < kRefs; ++k) {
      int32_t b = -1, nt = 0;
      int64_t sl = -1;
      for (int64_t c = q.cal_ptr[r]; c < q.cal_ptr[r + 1]; ++c)
        for (int h = 0; h < 2; ++h) {
          int32_t s;
          int64_t re;
          int16_t qe;
          stub_slot(rh, q.len[r], q.cal_pos[c], q.cal_ref[c], q.strand[c], h, &s, &re, &qe);
          if (k == 0)
            bad += s != q.score[2 * c + h] || re != q.ref_end[2 * c + h] || qe != q.read_end[2 * c + h];
          if (q.cal_ref[c] != k || s < 0) continue;
          if (s > b) {
            b = s;
            sl = 2 * c + h;
            nt = 1;
          } else if (s == b) {
            ++nt;
          }
        }
      const int64_t o = (int64_t)r * kRefs + k;
      bad += b != q.best_score[o] || sl != q.best_slot[o] || nt != q.n_tied[o];
    }
  }
  return bad;
}


// ---------------------------------------------------------------------------
// The served benchmark's configuration, replayed on the CPU: a 4 GiB staging
// budget, steps of up to 1024 chunks, 65536 reads and 1 M CALs, references of
// 3.2 and 2.7 Gbp, a pool of requests of log-uniform 1..10000 reads (lengths
// 75..250, 1..32 CALs per read, both strands), each reads' codes at a 16-aligned
// offset back to back; a warm-up, then the pool submitted `rounds` times from
// four client threads at once, then three Poisson load phases whose feeder
// thread submits at scheduled times while the main thread waits, reads the
// timestamps and releases each request in turn.  Every submission has its own
// output buffers and shares its inputs with the other submissions of the same
// pool request, as the benchmark's prepared submissions do.

struct Sub {  // one submission of a pool request
  const Req *in = nullptr;
  Req out;  // only the output vectors and the id are used
};

Req make_bench_request(std::mt19937_64 &g, int n_reads, const int64_t *ref_len) {
  Req q;
  q.n_reads = n_reads;
  q.len.resize(n_reads);
  q.code_off.resize(n_reads);
  int64_t at = 0;
  for (int i = 0; i < n_reads; ++i) {
    q.len[i] = 75 + (int)(g() % 176);
    q.code_off[i] = at;
    at += (q.len[i] + 15) / 16 * 16;
  }
  q.codes.resize((size_t)at);
  for (auto &c : q.codes) c = (uint8_t)(g() % 4);
  q.cal_ptr.assign(n_reads + 1, 0);
  for (int i = 0; i < n_reads; ++i) q.cal_ptr[i + 1] = q.cal_ptr[i] + 1 + (int64_t)(g() % 32);
  const int64_t nc = q.cal_ptr[n_reads];
  q.cal_pos.resize(nc);
  q.cal_ref.resize(nc);
  q.strand.assign(nc, 3);
  for (int64_t c = 0; c < nc; ++c) {
    q.cal_ref[c] = (int16_t)(g() % kRefs);
    q.cal_pos[c] = (int64_t)(g() % (uint64_t)ref_len[q.cal_ref[c]]);
  }
  return q;
}

void fresh_outputs(Sub &s) {
  const Req &q = *s.in;
  const int64_t nc = q.cal_ptr[q.n_reads];
  s.out = Req();
  s.out.n_reads = q.n_reads;
  s.out.score.assign(2 * nc, -7);
  s.out.ref_end.assign(2 * nc, -7);
  s.out.read_end.assign(2 * nc, -7);
  s.out.best_score.assign(q.n_reads * kRefs, -7);
  s.out.best_slot.assign(q.n_reads * kRefs, -7);
  s.out.n_tied.assign(q.n_reads * kRefs, -7);
}

int submit_sub(sw_server_t *srv, Sub &s) {
  const Req &q = *s.in;
  return sw_server_submit(srv, q.codes.data(), (int64_t)q.codes.size(), q.code_off.data(), q.len.data(), q.n_reads,
                          q.cal_ptr.data(), q.cal_pos.data(), q.cal_ref.data(), q.strand.data(),
                          q.cal_ptr[q.n_reads], s.out.score.data(), s.out.ref_end.data(), s.out.read_end.data(),
                          s.out.best_score.data(), s.out.best_slot.data(), s.out.n_tied.data(), &s.out.id);
}

long check_sub(const Sub &s) {
  Req view = *s.in;  // inputs of the pool request, outputs of this submission
  view.score = s.out.score;
  view.ref_end = s.out.ref_end;
  view.read_end = s.out.read_end;
  view.best_score = s.out.best_score;
  view.best_slot = s.out.best_slot;
  view.n_tied = s.out.n_tied;
  return check(view);
}

double mono_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int run_bench(uint64_t seed, int pool_size, int rounds, int per_load) {
  kMaxLen = 250;
  sw_scoring_t sc{};
  sc.match = 2;
  sc.mismatch = -3;
  sc.gap_open = 5;
  sc.gap_extend = 2;
  sc.band = 32;
  sc.precision = SW_PREC_AUTO;
  sc.kernel = SW_KERNEL_AUTO;
  sc.max_read_len = 250;
  sw_server_opts_t o{};
  o.device = 0;
  o.scoring = sc;
  o.memory_budget = (size_t)4 << 30;
  o.max_step_reads = 65536;
  o.max_step_cals = 1 << 20;
  o.max_step_chunks = 1024;
  o.autotune = 0;
  sw_server_t *srv = nullptr;
  if (sw_server_create(&o, &srv) != SW_OK) {
    fprintf(stderr, "create failed\n");
    return 2;
  }
  static const int64_t rlen[kRefs] = {3200000000ll, 2700000000ll};
  const int64_t woff[kRefs] = {0, (rlen[0] + 15) / 16};
  std::vector<uint32_t> ref_words(64, 0);  // the scoring stand-in reads no reference words
  sw_refset_t refs{ref_words.data(), woff, rlen, kRefs};
  if (sw_server_set_refs(srv, &refs) != SW_OK) {
    fprintf(stderr, "set_refs failed\n");
    return 2;
  }
  std::mt19937_64 g(seed);
  std::vector<Req> pool;
  pool.reserve(pool_size);
  double mean_reads = 0;
  for (int k = 0; k < pool_size; ++k) {
    const double u = (double)(g() >> 11) * (1.0 / 9007199254740992.0);
    const int n = std::min(10000, std::max(1, (int)std::floor(std::exp(u * std::log(10001.0)))));
    pool.push_back(make_bench_request(g, n, rlen));
    mean_reads += n;
  }
  mean_reads /= pool_size;
  long bad = 0, failed = 0, n_done = 0;
  std::atomic<long> submit_errors{0};
  auto finish = [&](Sub &s) {
    int32_t done = 0;
    if (sw_server_wait(srv, s.out.id, -1, &done) != SW_OK || !done) ++failed;
    int32_t state = 0;
    double t_sub = 0, t_adm = 0, t_done = 0;
    if (sw_server_request_info(srv, s.out.id, &state, &t_sub, &t_adm, &t_done) != SW_OK || state != 3 ||
        !(t_sub <= t_adm && t_adm <= t_done))
      ++failed;
    bad += check_sub(s);
    if (sw_server_release(srv, s.out.id) != SW_OK) ++failed;
    ++n_done;
  };
  // warm-up: the first requests one at a time
  for (int k = 0; k < std::min(8, pool_size); ++k) {
    Sub s;
    s.in = &pool[k];
    fresh_outputs(s);
    if (submit_sub(srv, s) != SW_OK) submit_errors++;
    finish(s);
  }
  // saturation: the pool `rounds` times over from four client threads
  std::vector<Sub> subs((size_t)rounds * pool_size);
  for (size_t i = 0; i < subs.size(); ++i) {
    subs[i].in = &pool[i % pool_size];
    fresh_outputs(subs[i]);
  }
  const int n_clients = 4;
  double t0 = mono_s();
  {
    std::vector<std::thread> th;
    for (int k = 0; k < n_clients; ++k)
      th.emplace_back([&, k] {
        for (size_t i = k; i < subs.size(); i += n_clients)
          if (submit_sub(srv, subs[i]) != SW_OK) submit_errors++;
      });
    for (auto &x : th) x.join();
  }
  for (auto &s : subs) finish(s);
  const double dt = mono_s() - t0;
  double sat_reads = 0;
  for (auto &s : subs) sat_reads += s.in->n_reads;
  sat_reads /= dt;
  subs.clear();
  subs.shrink_to_fit();
  // three Poisson load phases
  for (double load : {0.3, 0.6, 0.9}) {
    const double rate = load * sat_reads / mean_reads;
    std::mt19937_64 gl(seed * 7919 + (uint64_t)(load * 1000));
    std::exponential_distribution<double> gap(rate);
    std::vector<double> arrive(per_load);
    double t = 0;
    std::vector<Sub> ls(per_load);
    for (int i = 0; i < per_load; ++i) {
      t += gap(gl);
      arrive[i] = t;
      ls[i].in = &pool[gl() % (uint64_t)pool_size];
      fresh_outputs(ls[i]);
    }
    const double start = mono_s() + 0.05;
    std::thread feeder([&] {
      for (int i = 0; i < per_load; ++i) {
        const double d = start + arrive[i] - mono_s();
        if (d > 0) std::this_thread::sleep_for(std::chrono::duration<double>(d));
        if (submit_sub(srv, ls[i]) != SW_OK) submit_errors++;
      }
    });
    feeder.join();
    for (auto &s : ls) finish(s);
  }
  sw_server_stats_t st{};
  sw_server_stats(srv, &st);
  sw_server_destroy(srv);
  struct rusage ru {};
  getrusage(RUSAGE_SELF, &ru);
  printf("bench config: pool %d (mean %.1f reads), saturated %.0f reads/s on the stand-in\n", pool_size, mean_reads,
         sat_reads);
  printf("requests %ld, steps %lld (plain %ld, batched %ld, launched early %lld), submit errors %ld, failed %ld, "
         "mismatches %ld, peak rss %ld MiB\n",
         n_done, (long long)st.steps, g_plain_calls.load(), g_ctx_calls.load(), (long long)st.steps_launched_early,
         submit_errors.load(), failed, bad, (long)(ru.ru_maxrss / 1024));
  return (bad || failed || submit_errors || g_ctx_calls == 0) ? 1 : 0;
}

}  // namespace

int main(int argc, char **argv) {
  if (argc > 1 && std::string(argv[1]) == "bench") {
    const uint64_t seed = argc > 2 ? strtoull(argv[2], nullptr, 10) : 1;
    const int pool_size = argc > 3 ? atoi(argv[3]) : 300;
    const int rounds = argc > 4 ? atoi(argv[4]) : 8;
    const int per_load = argc > 5 ? atoi(argv[5]) : 2000;
    return run_bench(seed, pool_size, rounds, per_load);
  }

  const uint64_t seed = argc > 1 ? strtoull(argv[1], nullptr, 10) : 1;
  const int n_clients = argc > 2 ? atoi(argv[2]) : 4;
  const int per_client = argc > 3 ? atoi(argv[3]) : 60;
  const int layout = argc > 4 ? atoi(argv[4]) : 2;
  // scale 1: step and request sizes of the served benchmark (1024 chunks, 65536
  // reads and 1 M CALs per step, requests of up to 10000 reads of up to 250
  // bases with up to 32 CALs each); scale 0: small steps that split requests
  const int scale = argc > 5 ? atoi(argv[5]) : 0;
  const int depth = argc > 6 ? atoi(argv[6]) : 0;  // steps in flight (0: the server's default)
  if (scale) kMaxLen = 250;
  sw_scoring_t sc{};
  sc.match = 2;
  sc.mismatch = -3;
  sc.gap_open = 5;
  sc.gap_extend = 2;
  sc.band = 8;
  sc.precision = SW_PREC_AUTO;
  sc.kernel = SW_KERNEL_AUTO;
  sc.max_read_len = kMaxLen;
  sw_server_opts_t o{};
  o.device = 0;
  o.scoring = sc;
  o.memory_budget = scale ? (size_t)256 << 20 : (size_t)1 << 20;
  o.max_step_reads = scale ? 65536 : 48;
  o.max_step_cals = scale ? 1 << 20 : 200;
  o.max_step_chunks = scale ? 1024 : 6;
  o.max_steps_in_flight = depth;
  sw_server_t *srv = nullptr;
  if (sw_server_create(&o, &srv) != SW_OK) {
    fprintf(stderr, "create failed\n");
    return 2;
  }
  std::vector<uint32_t> ref_words(64, 0);
  const int64_t woff[kRefs] = {0, 32}, rlen[kRefs] = {500, 500};
  sw_refset_t refs{ref_words.data(), woff, rlen, kRefs};
  if (sw_server_set_refs(srv, &refs) != SW_OK) {
    fprintf(stderr, "set_refs failed\n");
    return 2;
  }
  std::vector<std::vector<Req>> reqs(n_clients);
  std::atomic<long> submit_errors{0};
  std::vector<std::thread> th;
  for (int t = 0; t < n_clients; ++t)
    th.emplace_back([&, t] {
      std::mt19937_64 g(seed * 1000003ull + (uint64_t)t);
      auto &mine = reqs[t];
      mine.reserve(per_client);
      for (int i = 0; i < per_client; ++i) {
        // mostly small requests, some as large as a whole step (at scale: log-uniform
        // 1..10000 reads with up to 32 CALs each)
        if (scale) {
          const int n = (int)std::exp(std::log(10000.0) * (double)(g() % 1000000) / 1e6);
          mine.push_back(make_request(g, std::max(1, n), 32, layout));
        } else {
          const bool big = g() % 5 == 0;
          mine.push_back(make_request(g, big ? o.max_step_reads : 12, big ? 40 : 12, layout));
        }
        Req &q = mine.back();
        const int rc = sw_server_submit(srv, q.codes.data(), (int64_t)q.codes.size(), q.code_off.data(),
                                        q.len.data(), q.n_reads, q.cal_ptr.data(), q.cal_pos.data(),
                                        q.cal_ref.data(), q.strand.data(), q.cal_ptr[q.n_reads], q.score.data(),
                                        q.ref_end.data(), q.read_end.data(), q.best_score.data(),
                                        q.best_slot.data(), q.n_tied.data(), &q.id);
        if (rc != SW_OK) {
          submit_errors++;
          fprintf(stderr, "submit rc %d: %d reads, %lld CALs\n", rc, q.n_reads, (long long)q.cal_ptr[q.n_reads]);
        }
      }
    });
  for (auto &x : th) x.join();
  long bad = 0, n = 0, failed = 0;
  for (auto &mine : reqs)
    for (auto &q : mine) {
      int32_t done = 0;
      if (sw_server_wait(srv, q.id, -1, &done) != SW_OK || !done) ++failed;
      bad += check(q);
      if (sw_server_release(srv, q.id) != SW_OK) ++failed;
      ++n;
    }
  sw_server_stats_t st{};
  sw_server_stats(srv, &st);
  sw_server_destroy(srv);
  printf("requests %ld, steps %lld (plain %ld, batched %ld, launched early %lld), submit errors %ld, failed %ld, "
         "mismatches %ld\n",
         n, (long long)st.steps, g_plain_calls.load(), g_ctx_calls.load(), (long long)st.steps_launched_early,
         submit_errors.load(), failed, bad);
  // small steps split requests, so both step paths always run; at the benchmark's
  // sizes a step is small only when few reads happen to be waiting, which depends
  // on thread timing
  const bool both_paths = g_plain_calls > 0 && g_ctx_calls > 0;
  return (bad || failed || submit_errors || (!scale && !both_paths)) ? 1 : 0;
}
