// Host test of the request server's scheduler (paper_1801_02417_amd/csrc/server_core.cpp) with a
// stub device on a simulated clock, built with the host sanitizers (AddressSanitizer +
// UndefinedBehaviorSanitizer, or ThreadSanitizer) by tests/test_server_host.py.  No GPU.
//
// The stub models the device as the scheduler sees it: a request's solve holds its footprint
// of simulated device memory; a lane's round takes a time proportional to its members' sizes on
// the simulated clock; adaptive members halt at a point derived from their ticket.  It checks the
// scheduler's invariants as it goes (admission within the budget, one request at a time under
// FIFO, batches built only from live solves of one group, no work for a halted or finished
// request) and aborts on a violation.  Scenarios (argv[1]): trace, fifo, cancel, oversize,
// zero_stage, destroy_busy, graph_key.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "graph_key.hpp"
#include "server_core.hpp"

#define CHECK(c)                                                                  \
  do {                                                                            \
    if (!(c)) {                                                                   \
      std::fprintf(stderr, "CHECK failed at %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::abort();                                                               \
    }                                                                             \
  } while (0)

namespace psara {
namespace serve {
namespace {

constexpr uint64_t kAlive = 0x5eedf00dcafe1234ull;

// Simulated device shared by every server of the process (one at a time).
struct Sim {
  std::mutex mu;
  double clock = 0.0;
  size_t capacity = 64ull << 30;
  size_t budget = 0;          // the server's budget, for the admission check
  int max_live = 1 << 30;     // the server's slot count
  size_t live_bytes = 0;
  int live = 0;
  int peak_live = 0;
  std::set<uint64_t> live_tickets;
  int alone_oversize = 0;     // solves opened above the budget (each must have been alone)
  void advance_to(double t) {
    std::lock_guard<std::mutex> lk(mu);
    clock = std::max(clock, t);
  }
  double now() {
    std::lock_guard<std::mutex> lk(mu);
    return clock;
  }
};
Sim g_sim;

size_t stub_footprint(const psara_request& r) {
  return (size_t)r.n * r.n * 640 + (size_t)r.M * 72;
}

// per iteration of one member on the simulated device: the footprint streamed at 0.5 TB/s plus
// launch latency (about what the library's iteration takes at 256^2 with 2e5 rows)
double iter_seconds(const Job& j) { return 20e-6 + (double)stub_footprint(j.req) / 5e11; }

struct StubHost : HostPrep {
  std::vector<int> perm;   // stands in for the sorted geometry
};

struct StubSolve : Solve {
  uint64_t magic = kAlive;
  uint64_t ticket = 0;
  size_t foot = 0;
  int64_t iters = 0;        // iterations the device ran for it
  int stage_it = 0;         // iterations of the current adaptive stage
  int bound = 0;            // adaptive stage bound (0: not adaptive / stage ended)
  int stop_at = 0;          // the iteration at which its stopping test holds
  bool halted = false;
  bool in_stage = false;
  double crit[3] = {0, 0, 0};
  ~StubSolve() override {
    CHECK(magic == kAlive);
    magic = 0;
    std::lock_guard<std::mutex> lk(g_sim.mu);
    g_sim.live_bytes -= foot;
    g_sim.live -= 1;
    g_sim.live_tickets.erase(ticket);
  }
};

StubSolve* solve_of(Job& j) {
  auto* s = static_cast<StubSolve*>(j.solve.get());
  CHECK(s != nullptr);
  CHECK(s->magic == kAlive);
  return s;
}

struct StubLane : Lane {
  std::vector<Job*> mem;
  std::vector<uint64_t> tickets;
  bool built = false;
  double dur = 0.0, start = 0.0;
  bool queued = false;
  void prepare(const std::vector<Job*>& members, bool rebuild, int kind, int check_every) override {
    CHECK(!members.empty());
    CHECK(!queued);
    if (rebuild || !built) {
      mem = members;
      tickets.clear();
      for (Job* j : mem) tickets.push_back(j->ticket);
      built = true;
    }
    CHECK(mem.size() == members.size());
    for (size_t i = 0; i < mem.size(); ++i) {
      CHECK(mem[i] == members[i] && tickets[i] == members[i]->ticket);
      StubSolve* s = solve_of(*members[i]);
      CHECK(s->ticket == members[i]->ticket);
      CHECK(members[i]->kind() == kind && members[i]->req.check_every == check_every);
      CHECK(members[i]->req.n == members[0]->req.n && members[i]->req.taps == members[0]->req.taps &&
            members[i]->req.precision == members[0]->req.precision);
    }
  }
  void launch(int kind, int iters, int check_every) override {
    CHECK(built && !queued && iters >= 1);
    double per = 0.0;
    for (Job* j : mem) {
      StubSolve* s = solve_of(*j);
      CHECK(j->kind() == kind);
      per += iter_seconds(*j);
      if (check_every > 0) {
        CHECK(iters % check_every == 0);
        CHECK(s->in_stage);
        for (int c = 0; c < iters / check_every; ++c) {
          if (s->halted) break;
          s->stage_it += check_every;
          s->iters += check_every;
          if (s->stage_it >= s->stop_at || s->stage_it >= s->bound) s->halted = true;
        }
      } else {
        CHECK(j->left >= iters);       // never beyond the stage
        s->iters += iters;
      }
    }
    start = g_sim.now();
    dur = 20e-6 + per * iters;
    queued = true;
  }
  double wait() override {
    CHECK(queued);
    queued = false;
    g_sim.advance_to(start + dur);
    return dur;
  }
  void drop() override {
    CHECK(!queued);
    mem.clear();
    tickets.clear();
    built = false;
  }
};

class StubDevice : public Device {
 public:
  double now() override { return g_sim.now(); }
  size_t capacity() override { return g_sim.capacity; }
  size_t footprint(const psara_request& r) override { return stub_footprint(r); }
  void prepare_host(Job& j) override {
    if (j.req.taps != 4 && j.req.taps != 6 && j.req.taps != 8) throw Error(PSARA_EINVAL, "taps must be 4, 6 or 8");
    std::unique_ptr<StubHost> h(new StubHost());
    h->perm.resize((size_t)j.req.M);
    for (int64_t i = 0; i < j.req.M; ++i) h->perm[(size_t)i] = (int)(j.req.M - 1 - i);
    std::this_thread::sleep_for(std::chrono::microseconds(50 + j.req.n / 4));
    j.host = std::move(h);
  }
  std::unique_ptr<Solve> open(Job& j) override {
    CHECK(j.host != nullptr);
    CHECK(static_cast<StubHost*>(j.host.get())->perm.size() == (size_t)j.req.M);
    if (j.req.epsilon == 777.0) throw Error(PSARA_EDEVICE, "injected device failure at set-up");
    std::unique_ptr<StubSolve> s(new StubSolve());
    s->ticket = j.ticket;
    s->foot = stub_footprint(j.req);
    s->stop_at = 20 * (1 + (int)(j.ticket % 4));
    {
      std::lock_guard<std::mutex> lk(g_sim.mu);
      // admission: within the budget, or alone
      if (g_sim.live_bytes + s->foot > g_sim.budget) {
        CHECK(g_sim.live == 0);
        g_sim.alone_oversize += 1;
      }
      CHECK(g_sim.live + 1 <= g_sim.max_live);
      g_sim.live_bytes += s->foot;
      g_sim.live += 1;
      g_sim.peak_live = std::max(g_sim.peak_live, g_sim.live);
      g_sim.live_tickets.insert(j.ticket);
      g_sim.clock += 1e-3 + 2e-9 * (double)j.req.M;        // set-up: power iteration, uploads
    }
    return s;
  }
  void stop_begin(Job& j, const double crit[3], int bound) override {
    StubSolve* s = solve_of(j);
    CHECK(!s->in_stage && bound > 0);
    s->in_stage = true;
    s->halted = false;
    s->stage_it = 0;
    s->bound = bound;
    std::memcpy(s->crit, crit, sizeof(s->crit));
  }
  void stop_poll(Job& j, bool* halted, int* iters) override {
    StubSolve* s = solve_of(j);
    CHECK(s->in_stage);
    *halted = s->halted;
    *iters = s->stage_it;
  }
  void stop_end(Job& j) override {
    StubSolve* s = solve_of(j);
    CHECK(s->in_stage && s->halted);
    s->in_stage = false;
  }
  double coef_std(Job& j) override {
    StubSolve* s = solve_of(j);
    CHECK(j.stage == 0 && !s->in_stage);
    return j.req.epsilon == 779.0 ? 0.0 : 0.25;
  }
  void reweight(Job& j, double delta) override {
    StubSolve* s = solve_of(j);
    CHECK(!s->in_stage && delta > 0.0);
  }
  void finish(Job& j, psara_report* rep, std::vector<double>* image) override {
    StubSolve* s = solve_of(j);
    CHECK(!s->in_stage);
    CHECK(s->iters == j.iterations);
    if (j.req.epsilon == 778.0) throw Error(PSARA_EDEVICE, "injected failure at the result read-back");
    rep->residual = (double)s->iters;
    image->assign((size_t)j.req.n * j.req.n * 4, (double)j.ticket + 0.5);
  }
  std::unique_ptr<Lane> lane() override { return std::unique_ptr<Lane>(new StubLane()); }
};

}  // namespace

std::unique_ptr<Device> make_device(int device) {
  if (device != 0) throw Error(PSARA_EINVAL, "bad device ordinal");
  return std::unique_ptr<Device>(new StubDevice());
}

}  // namespace serve
}  // namespace psara

// ------------------------------------------------------------------------------------------------
// driver

namespace {

using psara::serve::g_sim;

struct Req {
  int n;
  int64_t M;
  std::vector<double> uv, Y;
  std::vector<int> stages;
  int check_every = 0;
  double epsilon = 1.0;
  int taps = 8;
};

Req make_req(std::mt19937_64& rng, int n, int64_t M, int check_every) {
  Req r;
  r.n = n;
  r.M = M;
  r.uv.resize(2 * M);
  r.Y.resize(8 * M);
  std::uniform_real_distribution<double> u(-3.0, 3.0);
  for (auto& v : r.uv) v = u(rng);
  for (auto& v : r.Y) v = u(rng);
  r.check_every = check_every;
  r.stages = check_every > 0 ? std::vector<int>{100, 100, 100} : std::vector<int>{100, 100, 100};
  return r;
}

psara_request to_c(const Req& r) {
  psara_request q;
  std::memset(&q, 0, sizeof(q));
  q.n = r.n;
  q.M = r.M;
  q.uv = r.uv.data();
  q.Y = r.Y.data();
  q.epsilon = r.epsilon;
  q.taps = r.taps;
  q.levels = 4;
  q.basis_mask = 0x1FF;
  q.precision = PSARA_FP32_MIXED;
  q.mode = PSARA_CONSTRAINED;
  q.cycles = (int)r.stages.size() - 1;
  q.iters_per_stage = r.stages.data();
  q.delta_decay = 10.0;
  q.gamma_factor = 1e-3;
  q.opnorm_iters = 100;
  q.opnorm_rtol = 1e-4;
  q.check_every = r.check_every;
  q.stop.theta = 5e-3;
  q.stop.rel_var = 1e-3;
  q.stop.np_max = 0.5;
  return q;
}

double pct(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const size_t i = std::min(v.size() - 1, (size_t)std::floor(p / 100.0 * (double)(v.size() - 1) + 0.5));
  return v[i];
}

// A seeded Poisson stream of `count` requests at `rate`/s (sides {64, 128, 256, 512}, 512 with
// 1e6 rows, the others log-uniform in [1e3, 1e5]; every 4th adaptive; a few with injected
// failures), submitted on the simulated clock while a second thread polls and cancels.
int run_trace(psara_serve_policy policy, int count, double rate, size_t budget, int max_slots, uint64_t seed,
              double cancel_share) {
  std::mt19937_64 rng(seed);
  std::exponential_distribution<double> gap(rate);
  std::uniform_int_distribution<int> side(0, 3);
  std::uniform_real_distribution<double> lm(3.0, 5.0), u01(0.0, 1.0);
  std::vector<Req> reqs;
  std::vector<double> arrive;
  double t = 0.0;
  for (int i = 0; i < count; ++i) {
    t += gap(rng);
    arrive.push_back(t);
    const int n = 64 << side(rng);
    const int64_t M = n == 512 ? 200000 : (int64_t)std::llround(std::pow(10.0, lm(rng)));
    Req r = make_req(rng, n, M, (i % 4 == 3) ? 20 : 0);
    if (i % 37 == 5) r.epsilon = 777.0;     // fails at device set-up
    if (i % 41 == 7) r.epsilon = 778.0;     // fails at the result read-back
    if (i % 43 == 9) r.taps = 5;            // fails at host set-up
    reqs.push_back(std::move(r));
  }
  g_sim.budget = budget;
  g_sim.max_live = policy == PSARA_SERVE_FIFO ? 1 : max_slots;
  psara_server* S = nullptr;
  CHECK(psara_server_create(&S, 0, budget, max_slots, 300, policy) == PSARA_OK);
  std::vector<uint64_t> tickets(count, 0);
  std::atomic<int> submitted{0}, ended{0};
  std::vector<int> final_state(count, -1);
  std::vector<double> lat(count, 0.0);
  std::mutex mu;
  std::atomic<bool> done_submitting{false};
  // a share of the requests is cancelled, each after a seeded number of polls that find it
  // outstanding (so some while queued, some while running)
  std::vector<bool> cancel_sent(count, false);
  std::vector<int> cancel_after(count, -1);
  {
    std::mt19937_64 prng(seed ^ 0x9e3779b97f4a7c15ull);
    for (int i = 0; i < count; ++i)
      if (std::uniform_real_distribution<double>(0.0, 1.0)(prng) < cancel_share) cancel_after[i] = (int)(prng() % 30);
  }
  std::thread poller([&] {
    for (;;) {
      const int sub = submitted.load();
      for (int i = 0; i < sub; ++i) {
        if (final_state[i] >= 0) continue;
        const int n = reqs[i].n;
        psara_result res;
        CHECK(psara_server_poll(S, tickets[i], &res, nullptr) == PSARA_OK);
        if (res.state == PSARA_REQ_QUEUED || res.state == PSARA_REQ_RUNNING) {
          if (!cancel_sent[i] && cancel_after[i] >= 0 && cancel_after[i]-- == 0) {
            const psara_status st = psara_server_cancel(S, tickets[i]);
            CHECK(st == PSARA_OK || st == PSARA_ESTATE);
            cancel_sent[i] = true;
          }
          continue;
        }
        std::vector<double> img;
        if (res.state == PSARA_REQ_DONE) {
          img.resize((size_t)n * n * 4);
          CHECK(psara_server_poll(S, tickets[i], &res, img.data()) == PSARA_OK);
        }
        CHECK(res.t_submit <= res.t_done + 1e-12);
        if (res.state == PSARA_REQ_DONE) {
          CHECK(res.status == PSARA_OK);
          CHECK(res.t_start >= res.t_submit);
          for (double v : img) CHECK(v == (double)tickets[i] + 0.5);
          if (reqs[i].check_every == 0) CHECK(res.report.iterations == 300);
          else CHECK(res.report.iterations >= 60 && res.report.iterations <= 300);
          CHECK(res.report.residual == (double)res.report.iterations);
          lat[i] = res.t_done - res.t_submit;
        } else if (res.state == PSARA_REQ_FAILED) {
          CHECK(res.status != PSARA_OK);
          CHECK(reqs[i].epsilon == 777.0 || reqs[i].epsilon == 778.0 || reqs[i].taps == 5);
        } else {
          CHECK(res.state == PSARA_REQ_CANCELLED && cancel_sent[i]);
        }
        // a finished request is forgotten once collected
        CHECK(psara_server_poll(S, tickets[i], &res, nullptr) == PSARA_EINVAL);
        final_state[i] = res.state;
        ended.fetch_add(1);
      }
      if (done_submitting.load() && ended.load() == count) return;
      std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
  });
  for (int i = 0; i < count; ++i) {
    // wait on the simulated clock for the arrival; when nothing is outstanding, jump to it
    while (psara_server_clock(S) < arrive[i]) {
      if (submitted.load() == ended.load()) g_sim.advance_to(arrive[i]);
      else std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    psara_request q = to_c(reqs[i]);
    uint64_t tk = 0;
    CHECK(psara_server_submit(S, &q, &tk) == PSARA_OK);
    tickets[i] = tk;
    submitted.fetch_add(1);
  }
  done_submitting = true;
  CHECK(psara_server_drain(S) == PSARA_OK);
  poller.join();
  const double t_end = psara_server_clock(S);
  psara_server_destroy(S);
  int n_done = 0, n_failed = 0, n_cancelled = 0;
  std::vector<double> l;
  for (int i = 0; i < count; ++i) {
    if (final_state[i] == PSARA_REQ_DONE) { ++n_done; l.push_back(lat[i]); }
    else if (final_state[i] == PSARA_REQ_FAILED) ++n_failed;
    else if (final_state[i] == PSARA_REQ_CANCELLED) ++n_cancelled;
  }
  CHECK(g_sim.live == 0 && g_sim.live_bytes == 0);
  std::printf("{\"scenario\": \"trace\", \"policy\": %d, \"requests\": %d, \"done\": %d, \"failed\": %d, "
              "\"cancelled\": %d, \"solves_per_s\": %.3f, \"p50_s\": %.4f, \"p99_s\": %.4f, \"peak_live\": %d, "
              "\"alone_over_budget\": %d}\n",
              (int)policy, count, n_done, n_failed, n_cancelled, n_done / std::max(1e-9, t_end - arrive[0]), pct(l, 50),
              pct(l, 99), g_sim.peak_live, g_sim.alone_oversize);
  CHECK(n_done + n_failed + n_cancelled == count);
  CHECK(n_failed >= 1 && n_done >= count / 2);
  if (policy == PSARA_SERVE_FIFO) CHECK(g_sim.peak_live == 1);
  else CHECK(g_sim.peak_live > 1);
  return 0;
}

void wait_state(psara_server* S, uint64_t t, int want) {
  for (int k = 0; k < 200000; ++k) {
    psara_result r;
    CHECK(psara_server_poll(S, t, &r, nullptr) == PSARA_OK);
    if (r.state == want) return;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  CHECK(!"state not reached");
}

int run_cancel() {
  std::mt19937_64 rng(5);
  g_sim.budget = 8ull << 30;
  g_sim.max_live = 1;
  psara_server* S = nullptr;
  // one slot, one-iteration rounds: a long request holds the slot round after round
  CHECK(psara_server_create(&S, 0, 8ull << 30, 1, 1, PSARA_SERVE_BATCHED) == PSARA_OK);
  Req a = make_req(rng, 256, 50000, 0), b = make_req(rng, 64, 2000, 0), c = make_req(rng, 64, 1000, 0);
  a.stages = {100000, 100, 100};
  psara_request qa = to_c(a), qb = to_c(b), qc = to_c(c);
  uint64_t ta = 0, tb = 0, tc = 0;
  CHECK(psara_server_submit(S, &qa, &ta) == PSARA_OK);
  wait_state(S, ta, PSARA_REQ_RUNNING);
  CHECK(psara_server_submit(S, &qb, &tb) == PSARA_OK);
  CHECK(psara_server_submit(S, &qc, &tc) == PSARA_OK);
  // c is queued behind b: cancelled at once, without ever holding the device
  CHECK(psara_server_cancel(S, tc) == PSARA_OK);
  psara_result r;
  CHECK(psara_server_poll(S, tc, &r, nullptr) == PSARA_OK && r.state == PSARA_REQ_CANCELLED);
  CHECK(psara_server_poll(S, tc, &r, nullptr) == PSARA_EINVAL);     // forgotten once reported
  CHECK(psara_server_cancel(S, tc) == PSARA_EINVAL);
  // b waits for the slot a holds; cancelling a (running) frees it and b completes
  CHECK(psara_server_poll(S, tb, &r, nullptr) == PSARA_OK && r.state == PSARA_REQ_QUEUED);
  CHECK(psara_server_cancel(S, ta) == PSARA_OK);
  wait_state(S, ta, PSARA_REQ_CANCELLED);
  std::vector<double> img(64 * 64 * 4);
  wait_state(S, tb, PSARA_REQ_DONE);
  CHECK(psara_server_poll(S, tb, &r, img.data()) == PSARA_OK && r.report.iterations == 300);
  CHECK(img[0] == (double)tb + 0.5);
  CHECK(psara_server_cancel(S, tb) == PSARA_EINVAL);       // collected
  CHECK(psara_server_drain(S) == PSARA_OK);
  psara_server_destroy(S);
  CHECK(g_sim.live == 0);
  std::printf("{\"scenario\": \"cancel\", \"ok\": true}\n");
  return 0;
}

int run_oversize() {
  std::mt19937_64 rng(6);
  g_sim.capacity = 512ull << 20;
  g_sim.budget = 128ull << 20;
  g_sim.max_live = 8;
  psara_server* S = nullptr;
  CHECK(psara_server_create(&S, 0, 128ull << 20, 8, 50, PSARA_SERVE_BATCHED) == PSARA_OK);
  // above the device's whole memory: refused at submission, before its arrays are read (they
  // hold 1000 rows of the 1e9 the request declares; reading them would be caught here)
  Req huge = make_req(rng, 1024, 1000, 0);
  psara_request qh = to_c(huge);
  qh.M = 1000000000;
  uint64_t th = 0;
  CHECK(psara_server_submit(S, &qh, &th) == PSARA_ENOMEM);
  CHECK(std::strstr(psara_server_last_error(S), "device memory") != nullptr);
  // above the budget but within the device: runs alone, others queue behind it
  Req big = make_req(rng, 512, 200000, 0), s1 = make_req(rng, 64, 3000, 0), s2 = make_req(rng, 128, 3000, 0);
  psara_request qb = to_c(big), q1 = to_c(s1), q2 = to_c(s2);
  uint64_t tb = 0, t1 = 0, t2 = 0;
  CHECK(psara_server_submit(S, &q1, &t1) == PSARA_OK);
  CHECK(psara_server_submit(S, &qb, &tb) == PSARA_OK);
  CHECK(psara_server_submit(S, &q2, &t2) == PSARA_OK);
  CHECK(psara_server_drain(S) == PSARA_OK);
  for (uint64_t t : {t1, tb, t2}) {
    psara_result r;
    CHECK(psara_server_poll(S, t, &r, nullptr) == PSARA_OK && r.state == PSARA_REQ_DONE);
  }
  CHECK(g_sim.alone_oversize == 1);
  // malformed requests
  Req bad = make_req(rng, 64, 100, 0);
  bad.epsilon = -1.0;
  psara_request qbad = to_c(bad);
  uint64_t tbad = 0;
  CHECK(psara_server_submit(S, &qbad, &tbad) == PSARA_EINVAL);
  bad.epsilon = 1.0;
  bad.stages = {15, 20, 20};
  bad.check_every = 10;
  qbad = to_c(bad);
  CHECK(psara_server_submit(S, &qbad, &tbad) == PSARA_EINVAL);
  psara_server_destroy(S);
  g_sim.capacity = 64ull << 30;
  std::printf("{\"scenario\": \"oversize\", \"ok\": true}\n");
  return 0;
}

int run_zero_stage() {
  std::mt19937_64 rng(7);
  g_sim.budget = 8ull << 30;
  g_sim.max_live = 4;
  psara_server* S = nullptr;
  CHECK(psara_server_create(&S, 0, 8ull << 30, 4, 16, PSARA_SERVE_BATCHED) == PSARA_OK);
  std::vector<std::vector<int>> stage_sets = {{5, 0, 7}, {3, 0, 0}, {4, 9}, {6}};
  std::vector<uint64_t> t;
  std::vector<Req> keep;
  for (auto& st : stage_sets) {
    Req r = make_req(rng, 64, 500, 0);
    r.stages = st;
    keep.push_back(r);
  }
  Req a = make_req(rng, 64, 500, 10);
  a.stages = {20, 0, 30};
  keep.push_back(a);
  Req z = make_req(rng, 64, 500, 0);
  z.stages = {0, 5};
  z.epsilon = 779.0;           // zero initialisation stage: no reweighting scale, fails cleanly
  keep.push_back(z);
  for (auto& r : keep) {
    psara_request q = to_c(r);
    uint64_t tk = 0;
    CHECK(psara_server_submit(S, &q, &tk) == PSARA_OK);
    t.push_back(tk);
  }
  CHECK(psara_server_drain(S) == PSARA_OK);
  for (size_t i = 0; i < keep.size(); ++i) {
    psara_result r;
    CHECK(psara_server_poll(S, t[i], &r, nullptr) == PSARA_OK);
    if (i + 1 == keep.size()) {
      CHECK(r.state == PSARA_REQ_FAILED && r.status == PSARA_EINVAL);
      continue;
    }
    CHECK(r.state == PSARA_REQ_DONE);
    int total = 0;
    for (int v : keep[i].stages) total += v;
    if (keep[i].check_every == 0) CHECK(r.report.iterations == total);
    else CHECK(r.report.iterations <= total);
  }
  psara_server_destroy(S);
  CHECK(g_sim.live == 0);
  std::printf("{\"scenario\": \"zero_stage\", \"ok\": true}\n");
  return 0;
}

int run_destroy_busy() {
  std::mt19937_64 rng(8);
  g_sim.budget = 8ull << 30;
  g_sim.max_live = 8;
  psara_server* S = nullptr;
  CHECK(psara_server_create(&S, 0, 8ull << 30, 8, 4, PSARA_SERVE_BATCHED) == PSARA_OK);
  std::vector<Req> keep;
  for (int i = 0; i < 24; ++i) keep.push_back(make_req(rng, 64 << (i % 3), 2000 + 100 * i, (i % 3 == 2) ? 20 : 0));
  for (auto& r : keep) {
    psara_request q = to_c(r);
    uint64_t tk = 0;
    CHECK(psara_server_submit(S, &q, &tk) == PSARA_OK);
  }
  std::this_thread::sleep_for(std::chrono::milliseconds(20));
  psara_server_destroy(S);      // requests still queued and running
  CHECK(g_sim.live == 0 && g_sim.live_bytes == 0);
  std::printf("{\"scenario\": \"destroy_busy\", \"ok\": true}\n");
  return 0;
}

int run_graph_key() {
  // distinct (adaptive, mode, count) triples never share a key, including counts above 1000
  std::set<uint64_t> seen;
  int total = 0;
  for (int a = 0; a < 2; ++a)
    for (int m = 0; m < 5; ++m)
      for (int c : {0, 1, 7, 8, 31, 32, 999, 1000, 1001, 4096, 123456, 2147483647}) {
        seen.insert(psara::graph_key(a != 0, m, c));
        ++total;
      }
  CHECK((int)seen.size() == total);
  CHECK(psara::graph_key(true, 1, 1001) != psara::graph_key(true, 2, 1));
  std::printf("{\"scenario\": \"graph_key\", \"ok\": true}\n");
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  const std::string sc = argc > 1 ? argv[1] : "trace";
  const int count = argc > 2 ? std::atoi(argv[2]) : 120;
  const uint64_t seed = argc > 3 ? (uint64_t)std::strtoull(argv[3], nullptr, 10) : 2417;
  // a 1 GiB budget: the 512^2 requests (about 0.2 GB each) fill it, so admission queues
  if (sc == "trace") return run_trace(PSARA_SERVE_BATCHED, count, 20.0, 1ull << 30, 64, seed, 0.1);
  if (sc == "fifo") return run_trace(PSARA_SERVE_FIFO, count, 20.0, 1ull << 30, 64, seed, 0.1);
  if (sc == "cancel") return run_cancel();
  if (sc == "oversize") return run_oversize();
  if (sc == "zero_stage") return run_zero_stage();
  if (sc == "destroy_busy") return run_destroy_busy();
  if (sc == "graph_key") return run_graph_key();
  std::fprintf(stderr, "unknown scenario %s\n", sc.c_str());
  return 2;
}
