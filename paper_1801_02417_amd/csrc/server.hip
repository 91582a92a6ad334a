// Request server of the C ABI (declared in include/psara.h): admission by device-memory
// footprint, host-side set-up (the visibility sort and tile binning) on helper threads, and
// continuous batching of the admitted solves on one GPU.  Only the worker thread makes HIP
// calls: a call from another thread while the worker captures a graph could disturb the
// capture.  A request is Algorithm 2 on its own problem; while it runs it is a member
// of the batch of its stage's mode (the initialisation stage and the reweighted stages use
// different primal steps), which advances in rounds of at most `quantum` iterations; after a
// round the members that reached the end of a stage are reweighted (or finished) on their own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "ctx.hpp"
#include "engine.hpp"
#include "psara.h"

namespace {

struct Job {
  uint64_t ticket = 0;
  psara_request req{};             // array pointers are not used after the copy
  std::vector<double> uv, Y;
  std::vector<int> stages;
  size_t foot = 0;
  psara::Geometry geo;             // built by a set-up thread
  // progress, owned by the thread that holds the job
  psara_ctx* ctx = nullptr;
  int stage = 0, left = 0;
  int it_seen = 0;                 // adaptive stages: iterations of the stage already booked
  double delta = 0.0;
  // result, guarded by the server mutex
  int state = PSARA_REQ_QUEUED;
  psara_status status = PSARA_OK;
  double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
  psara_report report{};
  std::vector<double> image;
};
using JobP = std::shared_ptr<Job>;

int stage_mode(const Job& j) {
  if (j.stage == 0) return psara::PM_INIT;
  return j.req.mode == PSARA_UNCONSTRAINED ? psara::PM_UNCONSTRAINED : psara::PM_CONSTRAINED;
}

bool adaptive(const Job& j) { return j.req.check_every > 0; }

// Sets the device-side stopping state of an adaptive job's current stage: its criteria (the
// initialisation stage leaves N_p out, as psara_reweighted_solve_adaptive does) and its
// iteration bound, at which the device halts it as well.
void begin_stage(Job& j) {
  j.it_seen = 0;
  if (!adaptive(j)) return;
  const double v[3] = {j.req.stop.theta, j.req.stop.rel_var, j.stage == 0 ? -1.0 : j.req.stop.np_max};
  if (j.req.precision == PSARA_FP64) j.ctx->f64->stop_begin(v, j.stages[j.stage]);
  else j.ctx->f32->stop_begin(v, j.stages[j.stage]);
}

void stop_poll(Job& j, bool* halted, int* iters) {
  if (j.req.precision == PSARA_FP64) j.ctx->f64->stop_poll(halted, iters);
  else j.ctx->f32->stop_poll(halted, iters);
}

void stop_end(Job& j) {
  if (j.req.precision == PSARA_FP64) (void)j.ctx->f64->stop_end();
  else (void)j.ctx->f32->stop_end();
}

}  // namespace

struct psara_server {
  int device = 0;
  size_t budget = 0;
  int max_slots = 1, quantum = 1;
  psara_serve_policy policy = PSARA_SERVE_BATCHED;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  size_t used = 0;            // footprint of the admitted, unfinished requests
  int in_flight = 0;          // admitted, unfinished
  std::deque<JobP> queue;     // submitted, not yet admitted
  std::deque<JobP> ready;     // set up, waiting to join the batch
  std::map<uint64_t, JobP> jobs;
  std::string err;
  std::vector<std::thread> setup_threads;
  std::thread worker;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  bool can_admit() const {
    if (queue.empty() || in_flight >= max_slots) return false;
    return used + queue.front()->foot <= budget || in_flight == 0;
  }
};

namespace {

// Releases a finished or failed job's context and books the result (mutex held by the caller).
void retire(psara_server* S, Job& j, int state, psara_status st, const std::string& msg) {
  j.state = state;
  j.status = st;
  j.t_done = S->now();
  if (st != PSARA_OK) {
    S->err = "request " + std::to_string(j.ticket) + ": " + msg;
    std::fprintf(stderr, "psara server: %s\n", S->err.c_str());
  }
  S->used -= j.foot;
  S->in_flight -= 1;
}

// Host half of a request's set-up (set-up threads): argument checks and the geometry.
psara_status prepare_host(Job& j, std::string& msg) {
  const psara_request& r = j.req;
  try {
    psara_check_operator_args(r.n, r.M, j.uv.data(), 2, r.taps, r.precision);
    j.geo = psara::build_geometry(r.n, r.M, j.uv.data(), 2, r.taps);
  } catch (const psara::Error& e) {
    msg = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    msg = "host allocation failed";
    return PSARA_ENOMEM;
  }
  return PSARA_OK;
}

// Device half (worker thread): the context, data, prior, operator norm, gamma and steps.
psara_status prepare_device(psara_server* S, Job& j, std::string& msg) {
  psara_ctx* c = nullptr;
  psara_status st = psara_create(&c, S->device, nullptr);
  if (st != PSARA_OK) { msg = "context creation failed"; return st; }
  auto fail = [&](psara_status s) {
    msg = psara_last_error(c);
    psara_destroy(c);
    return s;
  };
  const psara_request& r = j.req;
  try {
    psara_bind_geometry(c, std::move(j.geo), r.precision);
  } catch (const psara::Error& e) {
    msg = e.msg;
    psara_destroy(c);
    return e.status;
  } catch (const std::exception& e) {
    msg = e.what();
    psara_destroy(c);
    return PSARA_EDEVICE;
  }
  j.geo = psara::Geometry();
  if ((st = psara_set_data(c, j.Y.data(), r.epsilon)) != PSARA_OK) return fail(st);
  if ((st = psara_set_prior(c, r.basis_mask, r.levels, nullptr, 1.0)) != PSARA_OK) return fail(st);
  double nrm = 0.0, g = 0.0;
  if ((st = psara_opnorm(c, r.opnorm_iters, r.opnorm_rtol, &nrm)) != PSARA_OK) return fail(st);
  if ((st = psara_data_gamma(c, r.gamma_factor, &g)) != PSARA_OK) return fail(st);
  if (!(g > 0.0)) { msg = "data-driven gamma is zero"; psara_destroy(c); return PSARA_EINVAL; }
  if ((st = psara_set_gamma(c, g)) != PSARA_OK) return fail(st);
  if ((st = psara_set_steps_auto(c, 0.99, nullptr)) != PSARA_OK) return fail(st);
  j.ctx = c;
  j.stage = 0;
  j.left = j.stages[0];
  try {
    begin_stage(j);
  } catch (const psara::Error& e) {
    msg = e.msg;
    psara_destroy(c);
    j.ctx = nullptr;
    return e.status;
  }
  return PSARA_OK;
}

void setup_loop(psara_server* S) {
  for (;;) {
    JobP j;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] { return S->stop || S->can_admit(); });
      if (S->stop) return;
      j = S->queue.front();
      S->queue.pop_front();
      S->used += j->foot;
      S->in_flight += 1;
      j->state = PSARA_REQ_RUNNING;
      j->t_start = S->now();
    }
    std::string msg;
    const psara_status st = prepare_host(*j, msg);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (st != PSARA_OK) retire(S, *j, PSARA_REQ_FAILED, st, msg);
      else S->ready.push_back(j);
    }
    S->cv.notify_all();
  }
}

// The admitted requests of one stage mode, precision, tap count and image side form a group; a
// group's batch runs on its own stream, so groups of different sizes overlap on the GPU, and
// each round gives a group as many iterations as fit in about kRoundSeconds of its measured
// iteration time (at most `quantum`): small problems then advance many iterations while a large
// one advances a few, instead of all moving in lockstep at the pace of the largest.
constexpr double kRoundSeconds = 0.01;
using GroupKey = std::tuple<int, int, int, int, int>;   // mode, precision, taps, side, check_every

struct Group {
  std::vector<psara_ctx*> key;          // members the cached batch was built for
  std::unique_ptr<psara::Batch<float>> bf;
  std::unique_ptr<psara::Batch<double>> bd;
  hipStream_t stream = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double t_iter = 0.0;                  // measured seconds per iteration (moving average)
  int k = 0;                            // iterations of the round in flight
  std::vector<JobP> mem;
  bool launched = false;
  Group() {
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) e0 = nullptr;
    if (hipEventCreate(&e1) != hipSuccess) e1 = nullptr;
  }
  ~Group() {
    drop_batch();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (stream) (void)hipStreamDestroy(stream);
  }
  Group(const Group&) = delete;
  Group& operator=(const Group&) = delete;
  void drop_batch() { bf.reset(); bd.reset(); key.clear(); }
  bool holds(const psara_ctx* c) const { return std::find(key.begin(), key.end(), c) != key.end(); }
};

// Rebuilds the group's batch when the membership changed and captures its graphs.  Called
// while the server has no GPU work in flight, so a capture never overlaps other work.
void prepare_round(Group& G, int mode) {
  if (!G.stream || !G.e0 || !G.e1) throw psara::Error(PSARA_EDEVICE, "group stream or events unavailable");
  std::vector<psara_ctx*> ctxs;
  for (auto& j : G.mem) ctxs.push_back(j->ctx);
  if (G.key != ctxs) {
    G.drop_batch();
    if (G.mem[0]->req.precision == PSARA_FP64) {
      std::vector<psara::Engine<double>*> e;
      for (auto* c : ctxs) e.push_back(c->f64.get());
      G.bd.reset(new psara::Batch<double>(e, G.stream));
    } else {
      std::vector<psara::Engine<float>*> e;
      for (auto* c : ctxs) e.push_back(c->f32.get());
      G.bf.reset(new psara::Batch<float>(e, G.stream));
    }
    G.key = ctxs;
  }
  const int ce = G.mem[0]->req.check_every;
  if (ce > 0) {
    if (G.bd) G.bd->capture_adaptive(mode, ce);
    else G.bf->capture_adaptive(mode, ce);
  } else if (G.bd) {
    G.bd->capture(mode);
  } else {
    G.bf->capture(mode);
  }
}

// Queues one round of the group: graph launches only.  An adaptive group runs whole chunks of
// check_every iterations (each followed by the check on the device); its members stop on the
// device, at their criteria or at their stage's bound.
void launch_round(Group& G, int mode, int quantum) {
  int left = 1 << 30;
  for (auto& j : G.mem) left = std::min(left, j->left);
  int k = G.t_iter > 0.0 ? (int)std::min<double>(quantum, std::max(1.0, kRoundSeconds / G.t_iter)) : std::min(quantum, 8);
  const int ce = G.mem[0]->req.check_every;
  psara::hip_check(hipEventRecord(G.e0, G.stream), "round start");
  if (ce > 0) {
    const int chunks = std::max(1, k / ce);
    G.k = chunks * ce;
    if (G.bd) G.bd->launch_adaptive(mode, chunks, ce);
    else G.bf->launch_adaptive(mode, chunks, ce);
  } else {
    G.k = std::max(1, std::min(k, left));
    if (G.bd) G.bd->run(mode, G.k);
    else G.bf->run(mode, G.k);
  }
  psara::hip_check(hipEventRecord(G.e1, G.stream), "round end");
  G.launched = true;
}

// Waits for the group's round and books the iterations.
void finish_round(Group& G) {
  psara::hip_check(hipEventSynchronize(G.e1), "round wait");
  float ms = 0.f;
  psara::hip_check(hipEventElapsedTime(&ms, G.e0, G.e1), "round time");
  const double t = 1e-3 * ms / G.k;
  G.t_iter = G.t_iter > 0.0 ? 0.5 * (G.t_iter + t) : t;
  for (auto& j : G.mem) {
    if (adaptive(*j)) {
      bool halted = false;
      int it = 0;
      stop_poll(*j, &halted, &it);
      j->ctx->iterations += it - j->it_seen;
      j->it_seen = it;
      j->left = halted ? 0 : std::max(1, j->stages[j->stage] - it);
    } else {
      j->left -= G.k;
      j->ctx->iterations += G.k;
    }
  }
  G.launched = false;
}

// Moves a job whose stage has ended to its next stage (reweighting it), or finishes it.
// Returns true when the job is finished (its result stored, its context released).
bool advance(psara_server* S, Job& j) {
  auto fail = [&](psara_status st, const std::string& m) {
    psara_destroy(j.ctx);
    j.ctx = nullptr;
    std::lock_guard<std::mutex> lk(S->mu);
    retire(S, j, PSARA_REQ_FAILED, st, m);
    return true;
  };
  try {
    if (j.left == 0 && adaptive(j)) stop_end(j);     // clears the halt flag
  } catch (const psara::Error& e) {
    return fail(e.status, e.msg);
  }
  while (j.left == 0) {
    if (j.stage == 0) {
      if (psara_coef_std(j.ctx, &j.delta) != PSARA_OK || !(j.delta > 0.0)) {
        const std::string m = j.delta > 0.0 ? psara_last_error(j.ctx) : "initial estimate is zero: no reweighting scale";
        psara_destroy(j.ctx);
        j.ctx = nullptr;
        std::lock_guard<std::mutex> lk(S->mu);
        retire(S, j, PSARA_REQ_FAILED, PSARA_EINVAL, m);
        return true;
      }
    }
    if (j.stage < j.req.cycles) {
      psara_status st = psara_reweight(j.ctx, j.delta);
      if (st != PSARA_OK) {
        const std::string m = psara_last_error(j.ctx);
        psara_destroy(j.ctx);
        j.ctx = nullptr;
        std::lock_guard<std::mutex> lk(S->mu);
        retire(S, j, PSARA_REQ_FAILED, st, m);
        return true;
      }
      j.delta /= j.req.delta_decay;
      j.stage += 1;
      j.left = j.stages[j.stage];
      try {
        begin_stage(j);
      } catch (const psara::Error& e) {
        return fail(e.status, e.msg);
      }
      continue;
    }
    psara_report rep;
    std::memset(&rep, 0, sizeof(rep));
    std::vector<double> img((size_t)j.req.n * j.req.n * 4);
    psara_status st = psara_report_now(j.ctx, &rep);
    if (st == PSARA_OK) st = psara_get_image(j.ctx, img.data());
    rep.iterations = j.ctx->iterations;
    const std::string m = st == PSARA_OK ? std::string() : std::string(psara_last_error(j.ctx));
    psara_destroy(j.ctx);
    j.ctx = nullptr;
    std::lock_guard<std::mutex> lk(S->mu);
    j.report = rep;
    j.image.swap(img);
    retire(S, j, st == PSARA_OK ? PSARA_REQ_DONE : PSARA_REQ_FAILED, st, m);
    return true;
  }
  return false;
}

void fail_jobs(psara_server* S, std::vector<JobP>& mem, psara_status st, const std::string& msg) {
  for (auto& j : mem) {
    if (j->ctx) psara_destroy(j->ctx);
    j->ctx = nullptr;
    j->left = -1;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  for (auto& j : mem) retire(S, *j, PSARA_REQ_FAILED, st, msg);
}

GroupKey key_of(const Job& j) {
  return std::make_tuple(stage_mode(j), (int)j.req.precision, j.req.taps, j.req.n, j.req.check_every);
}

void worker_loop(psara_server* S) {
  (void)hipSetDevice(S->device);
  std::vector<JobP> active, fresh;
  std::map<GroupKey, std::unique_ptr<Group>> groups;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (active.empty()) S->cv.wait(lk, [&] { return S->stop || !S->ready.empty(); });
      if (S->stop) break;
      while (!S->ready.empty()) {
        fresh.push_back(S->ready.front());
        S->ready.pop_front();
      }
    }
    // the round of every group, queued on the groups' streams
    std::map<GroupKey, std::vector<JobP>> members;
    for (auto& j : active) members[key_of(*j)].push_back(j);
    for (auto it = groups.begin(); it != groups.end();) {
      if (members.count(it->first)) ++it;
      else it = groups.erase(it);
    }
    // first every capture (nothing of the server runs on the GPU now), then every launch
    for (int phase = 0; phase < 2; ++phase) {
      for (auto& kv : members) {
        std::unique_ptr<Group>& G = groups[kv.first];
        if (!G) G.reset(new Group());
        if (phase == 0) G->mem = kv.second;
        else if (G->mem.empty() || G->mem[0]->left < 0) continue;
        try {
          if (phase == 0) prepare_round(*G, std::get<0>(kv.first));
          else launch_round(*G, std::get<0>(kv.first), S->quantum);
        } catch (const psara::Error& e) {
          G->drop_batch();
          G->launched = false;
          fail_jobs(S, G->mem, e.status, e.msg);
        } catch (const std::exception& e) {
          G->drop_batch();
          G->launched = false;
          fail_jobs(S, G->mem, PSARA_EDEVICE, e.what());
        }
      }
    }
    // device set-up of the newly admitted requests, overlapping the rounds on the GPU
    for (auto& j : fresh) {
      std::string msg;
      const psara_status st = prepare_device(S, *j, msg);
      if (st == PSARA_OK) {
        active.push_back(j);
      } else {
        std::lock_guard<std::mutex> lk(S->mu);
        retire(S, *j, PSARA_REQ_FAILED, st, msg);
      }
    }
    bool notify = !fresh.empty();
    fresh.clear();
    for (auto& kv : groups) {
      Group& G = *kv.second;
      if (!G.launched) continue;
      try {
        finish_round(G);
      } catch (const psara::Error& e) {
        G.drop_batch();
        G.launched = false;
        fail_jobs(S, G.mem, e.status, e.msg);
      }
    }
    // stage ends: reweighting or completion (a batch never outlives a member's context)
    std::vector<JobP> keep;
    for (auto& j : active) {
      if (j->left < 0) { notify = true; continue; }
      if (j->left == 0) {
        for (auto& kv : groups)
          if (kv.second->holds(j->ctx)) kv.second->drop_batch();
        if (advance(S, *j)) { notify = true; continue; }
      }
      keep.push_back(j);
    }
    active.swap(keep);
    if (notify) S->cv.notify_all();
  }
  groups.clear();
  for (auto& j : active)
    if (j->ctx) psara_destroy(j->ctx);
}

}  // namespace

extern "C" {

psara_status psara_server_create(psara_server** out, int device, size_t hbm_budget, int max_slots, int quantum,
                                 psara_serve_policy policy) {
  if (!out) return PSARA_EINVAL;
  *out = nullptr;
  if (max_slots < 1 || quantum < 1 || hbm_budget == 0) return PSARA_EINVAL;
  if (policy != PSARA_SERVE_BATCHED && policy != PSARA_SERVE_FIFO) return PSARA_EINVAL;
  if (psara_runtime_check(nullptr, nullptr) != PSARA_OK) return PSARA_EDEVICE;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return PSARA_EDEVICE;
  if (device < 0 || device >= count) return PSARA_EINVAL;
  std::unique_ptr<psara_server> S(new (std::nothrow) psara_server());
  if (!S) return PSARA_ENOMEM;
  S->device = device;
  S->budget = hbm_budget;
  S->policy = policy;
  S->max_slots = policy == PSARA_SERVE_FIFO ? 1 : max_slots;
  S->quantum = policy == PSARA_SERVE_FIFO ? (1 << 30) : quantum;
  S->t0 = std::chrono::steady_clock::now();
  try {
    const int nsetup = policy == PSARA_SERVE_FIFO ? 1 : 4;
    for (int i = 0; i < nsetup; ++i) S->setup_threads.emplace_back(setup_loop, S.get());
    S->worker = std::thread(worker_loop, S.get());
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv.notify_all();
    for (auto& t : S->setup_threads) if (t.joinable()) t.join();
    if (S->worker.joinable()) S->worker.join();
    return PSARA_ENOMEM;
  }
  *out = S.release();
  return PSARA_OK;
}

psara_status psara_server_submit(psara_server* S, const psara_request* r, uint64_t* ticket) {
  if (!S || !r || !ticket) return PSARA_EINVAL;
  auto bad = [&](const char* m) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->err = m;
    return PSARA_EINVAL;
  };
  if (!r->uv || !r->Y || r->M < 1 || r->n < 8) return bad("request: missing arrays or bad sizes");
  if (!(r->epsilon > 0.0) || r->cycles < 0 || !r->iters_per_stage) return bad("request: bad epsilon or stages");
  if (!(r->delta_decay > 1.0) || !(r->gamma_factor > 0.0) || r->opnorm_iters < 1) return bad("request: bad parameters");
  for (int l = 0; l <= r->cycles; ++l)
    if (r->iters_per_stage[l] < 0) return bad("request: negative iteration count");
  if (r->check_every < 0) return bad("request: negative check_every");
  if (r->check_every > 0) {
    if (!(r->stop.theta >= 0.0) || !(r->stop.rel_var >= 0.0) || std::isnan(r->stop.np_max))
      return bad("request: bad stopping criteria");
    for (int l = 0; l <= r->cycles; ++l)
      if (r->iters_per_stage[l] % r->check_every != 0) return bad("request: stage bounds must be multiples of check_every");
  }
  JobP j = std::make_shared<Job>();
  try {
    j->req = *r;
    j->uv.assign(r->uv, r->uv + 2 * r->M);
    j->Y.assign(r->Y, r->Y + 8 * r->M);
    j->stages.assign(r->iters_per_stage, r->iters_per_stage + r->cycles + 1);
  } catch (const std::bad_alloc&) {
    return PSARA_ENOMEM;
  }
  j->req.uv = nullptr;
  j->req.Y = nullptr;
  j->req.iters_per_stage = nullptr;
  j->foot = psara_footprint(r->n, r->M, r->taps, r->levels, r->basis_mask, r->precision);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    j->ticket = S->next_ticket++;
    j->t_submit = S->now();
    S->jobs[j->ticket] = j;
    S->queue.push_back(j);
    *ticket = j->ticket;
  }
  S->cv.notify_all();
  return PSARA_OK;
}

psara_status psara_server_poll(psara_server* S, uint64_t ticket, psara_result* out, double* image) {
  if (!S || !out) return PSARA_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return PSARA_EINVAL;
  Job& j = *it->second;
  out->state = j.state;
  out->status = j.status;
  out->t_submit = j.t_submit;
  out->t_start = j.t_start;
  out->t_done = j.t_done;
  out->n = j.req.n;
  out->report = j.report;
  if (j.state == PSARA_REQ_FAILED) {
    S->jobs.erase(it);
  } else if (j.state == PSARA_REQ_DONE && image) {
    std::memcpy(image, j.image.data(), j.image.size() * sizeof(double));
    S->jobs.erase(it);
  }
  return PSARA_OK;
}

psara_status psara_server_drain(psara_server* S) {
  if (!S) return PSARA_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv.wait(lk, [&] { return S->queue.empty() && S->ready.empty() && S->in_flight == 0; });
  return PSARA_OK;
}

double psara_server_clock(const psara_server* S) { return S ? S->now() : 0.0; }

const char* psara_server_last_error(const psara_server* S) { return S ? S->err.c_str() : "null server"; }

void psara_server_destroy(psara_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (auto& t : S->setup_threads) if (t.joinable()) t.join();
  if (S->worker.joinable()) S->worker.join();
  for (auto& j : S->ready)
    if (j->ctx) psara_destroy(j->ctx);
  delete S;
}

}  // extern "C"
