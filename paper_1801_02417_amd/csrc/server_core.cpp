// Scheduler of the request server: the psara_server_* entry points of include/psara.h on top of
// the Device interface (server_core.hpp).  Host only.
#include "server_core.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <tuple>

using psara::Error;
using psara::serve::Device;
using psara::serve::Job;
using psara::serve::JobP;
using psara::serve::Lane;

namespace {

// Books a job's end (mutex held by the caller): its state and status, and, for an admitted
// job, the release of its slot and footprint.
void retire(psara_server* S, Job& j, int state, psara_status st, const std::string& msg) {
  j.state = state;
  j.status = st;
  j.t_done = S->dev->now();
  if (st != PSARA_OK) {
    S->err = "request " + std::to_string(j.ticket) + ": " + msg;
    std::fprintf(stderr, "psara server: %s\n", S->err.c_str());
  }
  S->used -= j.foot;
  S->in_flight -= 1;
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
      j->t_start = S->dev->now();
    }
    psara_status st = PSARA_OK;
    std::string msg;
    try {
      S->dev->prepare_host(*j);
    } catch (const Error& e) {
      st = e.status;
      msg = e.msg;
    } catch (const std::bad_alloc&) {
      st = PSARA_ENOMEM;
      msg = "host allocation failed";
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (st != PSARA_OK) retire(S, *j, PSARA_REQ_FAILED, st, msg);
      else if (j->cancel) retire(S, *j, PSARA_REQ_CANCELLED, PSARA_OK, "");
      else S->ready.push_back(j);
    }
    S->cv.notify_all();
  }
}

// Each round gives a group as many iterations as fit in about kRoundSeconds of its measured
// iteration time (at most `quantum`): small problems then advance many iterations while a large
// one advances a few, instead of all moving in lockstep at the pace of the largest.
constexpr double kRoundSeconds = 0.01;
using GroupKey = std::tuple<int, int, int, int, int>;   // stage kind, precision, taps, side, check_every

GroupKey key_of(const Job& j) {
  return std::make_tuple(j.kind(), (int)j.req.precision, j.req.taps, j.req.n, j.req.check_every);
}

struct Group {
  std::unique_ptr<Lane> lane;
  std::vector<const Job*> key;   // members the lane's batch was made for (jobs stay alive meanwhile)
  double t_iter = 0.0;           // measured seconds per iteration (moving average)
  int k = 0;                     // iterations of the round in flight
  std::vector<JobP> mem;
  bool launched = false;
  void drop() {
    if (lane) lane->drop();
    key.clear();
  }
  bool holds(const Job* j) const { return std::find(key.begin(), key.end(), j) != key.end(); }
};

// Sets the device-side stopping state of an adaptive job's current stage: its criteria (the
// initialisation stage leaves N_p out, as psara_reweighted_solve_adaptive does) and its bound.
void begin_stage(psara_server* S, Job& j) {
  j.it_seen = 0;
  if (!j.adaptive() || j.left == 0) return;
  const double v[3] = {j.req.stop.theta, j.req.stop.rel_var, j.stage == 0 ? -1.0 : j.req.stop.np_max};
  S->dev->stop_begin(j, v, j.stages[j.stage]);
}

// Releases a job's solve and books its end (worker thread).
void close_job(psara_server* S, Job& j, int state, psara_status st, const std::string& msg) {
  j.solve.reset();
  j.left = -1;
  std::lock_guard<std::mutex> lk(S->mu);
  retire(S, j, state, st, msg);
}

// Device set-up of a newly admitted job (worker thread).
void open_job(psara_server* S, Job& j) {
  j.solve = S->dev->open(j);
  j.host.reset();
  j.stage = 0;
  j.left = j.stages[0];
  begin_stage(S, j);
}

// Moves a job whose stage has ended (left == 0) through its reweightings to its next stage
// with iterations left, or finishes it.  Returns true when the job has ended.
bool advance(psara_server* S, Job& j) {
  try {
    while (j.left == 0) {
      if (j.adaptive() && j.stages[j.stage] > 0) S->dev->stop_end(j);
      if (j.stage == 0) {
        j.delta = S->dev->coef_std(j);
        if (!(j.delta > 0.0)) throw Error(PSARA_EINVAL, "initial estimate is zero: no reweighting scale");
      }
      if (j.stage < j.req.cycles) {
        S->dev->reweight(j, j.delta);
        j.delta /= j.req.delta_decay;
        j.stage += 1;
        j.left = j.stages[j.stage];
        begin_stage(S, j);
        continue;
      }
      psara_report rep;
      std::memset(&rep, 0, sizeof(rep));
      std::vector<double> img;
      S->dev->finish(j, &rep, &img);
      rep.iterations = j.iterations;
      j.solve.reset();
      j.left = -1;
      std::lock_guard<std::mutex> lk(S->mu);
      j.report = rep;
      j.image.swap(img);
      retire(S, j, PSARA_REQ_DONE, PSARA_OK, "");
      return true;
    }
  } catch (const Error& e) {
    close_job(S, j, PSARA_REQ_FAILED, e.status, e.msg);
    return true;
  } catch (const std::bad_alloc&) {
    close_job(S, j, PSARA_REQ_FAILED, PSARA_ENOMEM, "host allocation failed");
    return true;
  }
  return false;
}

void fail_group(psara_server* S, Group& G, psara_status st, const std::string& msg) {
  G.drop();
  G.launched = false;
  for (auto& j : G.mem)
    if (j->left >= 0) close_job(S, *j, PSARA_REQ_FAILED, st, msg);
}

// Makes the group's batch current for its members and captures its round (nothing of the
// server runs on the device meanwhile).
void prepare_round(Group& G) {
  std::vector<const Job*> now;
  std::vector<Job*> members;
  for (auto& j : G.mem) {
    now.push_back(j.get());
    members.push_back(j.get());
  }
  const bool rebuild = now != G.key;
  if (rebuild) G.key.clear();
  G.lane->prepare(members, rebuild, G.mem[0]->kind(), G.mem[0]->req.check_every);
  G.key = now;
}

// Queues one round of the group.  An adaptive group runs whole chunks of check_every iterations
// (each followed by the stopping test on the device); its members stop on the device, at their
// criteria or at their stage's bound.
void launch_round(Group& G, int quantum) {
  int left = 1 << 30;
  for (auto& j : G.mem) left = std::min(left, j->left);
  const int k = G.t_iter > 0.0 ? (int)std::min<double>(quantum, std::max(1.0, kRoundSeconds / G.t_iter))
                               : std::min(quantum, 8);
  const int ce = G.mem[0]->req.check_every;
  G.k = ce > 0 ? std::max(1, k / ce) * ce : std::max(1, std::min(k, left));
  G.lane->launch(G.mem[0]->kind(), G.k, ce);
  G.launched = true;
}

// Waits for the group's round and books the iterations.
void finish_round(psara_server* S, Group& G) {
  const double t = G.lane->wait() / G.k;
  G.launched = false;
  G.t_iter = G.t_iter > 0.0 ? 0.5 * (G.t_iter + t) : t;
  for (auto& j : G.mem) {
    if (j->adaptive()) {
      bool halted = false;
      int it = 0;
      S->dev->stop_poll(*j, &halted, &it);
      j->iterations += it - j->it_seen;
      j->it_seen = it;
      j->left = halted ? 0 : std::max(1, j->stages[j->stage] - it);
    } else {
      j->left -= G.k;
      j->iterations += G.k;
    }
  }
}

void worker_loop(psara_server* S) {
  std::vector<JobP> active, fresh;
  std::map<GroupKey, Group> groups;
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
    // the round of every group, queued on the groups' lanes
    std::map<GroupKey, std::vector<JobP>> members;
    for (auto& j : active) members[key_of(*j)].push_back(j);
    for (auto it = groups.begin(); it != groups.end();) {
      if (members.count(it->first)) ++it;
      else it = groups.erase(it);
    }
    // first every capture (nothing of the server runs on the device now), then every launch
    for (int phase = 0; phase < 2; ++phase) {
      for (auto& kv : members) {
        Group& G = groups[kv.first];
        try {
          if (phase == 0) {
            if (!G.lane) G.lane = S->dev->lane();
            G.mem = kv.second;
            prepare_round(G);
          } else if (!G.mem.empty() && G.mem[0]->left > 0) {
            launch_round(G, S->quantum);
          }
        } catch (const Error& e) {
          fail_group(S, G, e.status, e.msg);
        } catch (const std::bad_alloc&) {
          fail_group(S, G, PSARA_ENOMEM, "host allocation failed");
        }
      }
    }
    // device set-up of the newly admitted requests, overlapping the rounds on the device
    for (auto& j : fresh) {
      bool cancelled;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        cancelled = j->cancel;
      }
      if (cancelled) {
        j->host.reset();
        std::lock_guard<std::mutex> lk(S->mu);
        retire(S, *j, PSARA_REQ_CANCELLED, PSARA_OK, "");
        continue;
      }
      try {
        open_job(S, *j);
        // a stage of zero iterations ends at once (advance reweights or finishes the job)
        if (j->left == 0 && advance(S, *j)) continue;
        active.push_back(j);
      } catch (const Error& e) {
        close_job(S, *j, PSARA_REQ_FAILED, e.status, e.msg);
      } catch (const std::bad_alloc&) {
        close_job(S, *j, PSARA_REQ_FAILED, PSARA_ENOMEM, "host allocation failed");
      }
    }
    bool notify = !fresh.empty();
    fresh.clear();
    for (auto& kv : groups) {
      Group& G = kv.second;
      if (!G.launched) continue;
      try {
        finish_round(S, G);
      } catch (const Error& e) {
        fail_group(S, G, e.status, e.msg);
      }
    }
    // cancellations, stage ends (reweighting or completion); a lane's batch never outlives a
    // member's solve
    std::vector<JobP> keep;
    for (auto& j : active) {
      if (j->left < 0) { notify = true; continue; }
      bool cancelled;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        cancelled = j->cancel;
      }
      if (cancelled || j->left == 0) {
        for (auto& kv : groups)
          if (kv.second.holds(j.get())) kv.second.drop();
      }
      if (cancelled) {
        close_job(S, *j, PSARA_REQ_CANCELLED, PSARA_OK, "");
        notify = true;
        continue;
      }
      if (j->left == 0 && advance(S, *j)) { notify = true; continue; }
      keep.push_back(j);
    }
    active.swap(keep);
    if (notify) S->cv.notify_all();
  }
  groups.clear();
  for (auto& j : active) j->solve.reset();
}

bool check_request(const psara_request* r, std::string* why) {
  auto bad = [&](const char* m) { *why = m; return false; };
  if (!r->uv || !r->Y || r->M < 1 || r->n < 8) return bad("request: missing arrays or bad sizes");
  if (!(r->epsilon > 0.0) || !std::isfinite(r->epsilon) || r->cycles < 0 || !r->iters_per_stage)
    return bad("request: bad epsilon or stages");
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
  return true;
}

}  // namespace

extern "C" {

psara_status psara_server_create(psara_server** out, int device, size_t hbm_budget, int max_slots, int quantum,
                                 psara_serve_policy policy) {
  if (!out) return PSARA_EINVAL;
  *out = nullptr;
  if (max_slots < 1 || quantum < 1 || hbm_budget == 0) return PSARA_EINVAL;
  if (policy != PSARA_SERVE_BATCHED && policy != PSARA_SERVE_FIFO) return PSARA_EINVAL;
  std::unique_ptr<psara_server> S(new (std::nothrow) psara_server());
  if (!S) return PSARA_ENOMEM;
  try {
    S->dev = psara::serve::make_device(device);
  } catch (const Error& e) {
    return e.status;
  } catch (const std::bad_alloc&) {
    return PSARA_ENOMEM;
  }
  S->budget = hbm_budget;
  S->policy = policy;
  S->max_slots = policy == PSARA_SERVE_FIFO ? 1 : max_slots;
  S->quantum = policy == PSARA_SERVE_FIFO ? (1 << 30) : quantum;
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
  std::string why;
  if (!check_request(r, &why)) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->err = why;
    return PSARA_EINVAL;
  }
  // the footprint test first: a request that could never be admitted is refused before its
  // arrays are read
  size_t foot = 0, cap = 0;
  try {
    foot = S->dev->footprint(*r);
    cap = S->dev->capacity();
  } catch (const Error& e) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->err = e.msg;
    return e.status;
  }
  if (foot == 0 || foot > cap) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->err = foot == 0 ? "request: no footprint for these sizes"
                       : "request: needs " + std::to_string(foot) + " bytes of device memory, more than the device's " +
                             std::to_string(cap);
    return foot == 0 ? PSARA_EINVAL : PSARA_ENOMEM;
  }
  JobP j;
  try {
    j = std::make_shared<Job>();
    j->req = *r;
    j->uv.assign(r->uv, r->uv + 2 * r->M);
    j->Y.assign(r->Y, r->Y + 8 * r->M);
    j->stages.assign(r->iters_per_stage, r->iters_per_stage + r->cycles + 1);
  } catch (const std::bad_alloc&) {
    return PSARA_ENOMEM;
  }
  j->foot = foot;
  j->req.uv = nullptr;
  j->req.Y = nullptr;
  j->req.iters_per_stage = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    j->ticket = S->next_ticket++;
    j->t_submit = S->dev->now();
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
  if (j.state == PSARA_REQ_FAILED || j.state == PSARA_REQ_CANCELLED) {
    S->jobs.erase(it);
  } else if (j.state == PSARA_REQ_DONE && image) {
    std::memcpy(image, j.image.data(), j.image.size() * sizeof(double));
    S->jobs.erase(it);
  }
  return PSARA_OK;
}

psara_status psara_server_cancel(psara_server* S, uint64_t ticket) {
  if (!S) return PSARA_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return PSARA_EINVAL;
    Job& j = *it->second;
    if (j.state == PSARA_REQ_QUEUED) {
      auto q = std::find(S->queue.begin(), S->queue.end(), it->second);
      if (q != S->queue.end()) S->queue.erase(q);
      j.state = PSARA_REQ_CANCELLED;
      j.t_done = S->dev->now();
    } else if (j.state == PSARA_REQ_RUNNING) {
      j.cancel = true;           // taken up by the thread that holds the job, at its next step
    } else {
      return PSARA_ESTATE;       // done, failed or cancelled already
    }
  }
  S->cv.notify_all();
  return PSARA_OK;
}

psara_status psara_server_drain(psara_server* S) {
  if (!S) return PSARA_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv.wait(lk, [&] { return S->queue.empty() && S->ready.empty() && S->in_flight == 0; });
  return PSARA_OK;
}

double psara_server_clock(const psara_server* S) { return S ? S->dev->now() : 0.0; }

const char* psara_server_last_error(const psara_server* S) {
  if (!S) return "null server";
  psara_server* m = const_cast<psara_server*>(S);
  std::lock_guard<std::mutex> lk(m->mu);
  m->err_copy = m->err;
  return m->err_copy.c_str();
}

void psara_server_destroy(psara_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (auto& t : S->setup_threads) if (t.joinable()) t.join();
  if (S->worker.joinable()) S->worker.join();
  for (auto& j : S->ready) j->solve.reset();
  S->jobs.clear();
  S->queue.clear();
  S->ready.clear();
  S->dev.reset();
  delete S;
}

}  // extern "C"
