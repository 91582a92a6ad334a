// Scheduler of the request server (declared in include/psara.h as psara_server_*): admission by
// device-memory footprint, host-side set-up on helper threads, and continuous batching of the
// admitted solves in rounds.  Host only: it reaches the GPU through the Device interface below,
// which the library implements with HIP (server.hip) and the host tests implement with a stub on
// a simulated clock, so the scheduling runs under the host sanitizers without a GPU.
//
// A request is Algorithm 2 on its own problem: the initialisation stage, then `cycles`
// reweighted stages.  While it runs it is a member of the group of its stage kind, precision,
// tap count, image side and check interval; a group advances all its members in one batched
// round at a time, and after a round the members that reached the end of a stage are reweighted
// (or finished) on their own and join the group of their next stage.
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "error.hpp"
#include "psara.h"

namespace psara {
namespace serve {

// Device-specific state of a request, owned by its job: what the set-up threads prepare on the
// host, and the request's solve on the device once it is admitted to the GPU.
struct HostPrep {
  virtual ~HostPrep() = default;
};
struct Solve {
  virtual ~Solve() = default;
};

// Stage kinds: the initialisation stage, a reweighted stage of the constrained problem, one of
// the unconstrained problem.
enum StageKind { SK_INIT = 0, SK_CONSTRAINED = 1, SK_UNCONSTRAINED = 2 };

struct Job {
  uint64_t ticket = 0;
  psara_request req{};             // the array pointers are cleared after the copy
  std::vector<double> uv, Y;
  std::vector<int> stages;
  size_t foot = 0;
  // owned by the thread that holds the job (a set-up thread, then the worker)
  std::unique_ptr<HostPrep> host;
  std::unique_ptr<Solve> solve;
  int stage = 0, left = 0;
  int it_seen = 0;                 // adaptive stages: iterations of the stage already booked
  double delta = 0.0;
  int64_t iterations = 0;
  // guarded by the server mutex
  bool cancel = false;
  int state = PSARA_REQ_QUEUED;
  psara_status status = PSARA_OK;
  double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
  psara_report report{};
  std::vector<double> image;

  bool adaptive() const { return req.check_every > 0; }
  int kind() const {
    if (stage == 0) return SK_INIT;
    return req.mode == PSARA_UNCONSTRAINED ? SK_UNCONSTRAINED : SK_CONSTRAINED;
  }
};
using JobP = std::shared_ptr<Job>;

// The device side of one group: the batch of its members and the stream its rounds run on.
struct Lane {
  virtual ~Lane() = default;
  // Makes the batch of `members` (rebuilding it when `rebuild`; the members' solves are live)
  // and captures what a round of stage kind `kind` launches (check_every > 0: chunks of that
  // many iterations, each followed by the stopping test).  Called while nothing of the server
  // runs on the device.
  virtual void prepare(const std::vector<Job*>& members, bool rebuild, int kind, int check_every) = 0;
  // Queues one round: `iters` iterations, or iters / check_every adaptive chunks.
  virtual void launch(int kind, int iters, int check_every) = 0;
  // Waits for the queued round; returns its duration on the device in seconds.
  virtual double wait() = 0;
  // Releases the batch (the members' solves stay).
  virtual void drop() = 0;
};

// The GPU as the scheduler sees it.  Every method may throw psara::Error.  Only the worker
// thread calls the methods marked (worker); the set-up threads call prepare_host.
class Device {
 public:
  virtual ~Device() = default;
  virtual double now() = 0;                                   // seconds since creation
  virtual size_t capacity() = 0;                              // bytes of device memory in all
  virtual size_t footprint(const psara_request& r) = 0;       // bytes one request holds
  virtual void prepare_host(Job& j) = 0;                      // argument checks, host set-up
  // (worker) the request's solve: operator, data, prior, operator norm, gamma, step sizes
  virtual std::unique_ptr<Solve> open(Job& j) = 0;
  // (worker) adaptive stages: criteria {theta, rel_var, np_max} and the stage's bound; the
  // halt flag and iterations so far; the end of the stage (clears the halt flag)
  virtual void stop_begin(Job& j, const double crit[3], int bound) = 0;
  virtual void stop_poll(Job& j, bool* halted, int* iters) = 0;
  virtual void stop_end(Job& j) = 0;
  virtual double coef_std(Job& j) = 0;                        // (worker) delta of the first reweighting
  virtual void reweight(Job& j, double delta) = 0;            // (worker)
  // (worker) the final report and image (n*n x 4) of a finished request
  virtual void finish(Job& j, psara_report* rep, std::vector<double>* image) = 0;
  virtual std::unique_ptr<Lane> lane() = 0;                   // (worker)
};

// The device layer of a server on GPU `device`: the library's HIP one, or the host tests' stub.
// Throws Error: PSARA_EDEVICE when no usable device (or a HIP runtime mismatch), PSARA_EINVAL
// for a bad ordinal.
std::unique_ptr<Device> make_device(int device);

}  // namespace serve
}  // namespace psara

struct psara_server {
  std::unique_ptr<psara::serve::Device> dev;
  size_t budget = 0;
  int max_slots = 1, quantum = 1;
  psara_serve_policy policy = PSARA_SERVE_BATCHED;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  size_t used = 0;            // footprint of the admitted, unfinished requests
  int in_flight = 0;          // admitted, unfinished
  std::deque<psara::serve::JobP> queue;     // submitted, not yet admitted
  std::deque<psara::serve::JobP> ready;     // set up on the host, waiting for the worker
  std::map<uint64_t, psara::serve::JobP> jobs;
  std::string err;            // guarded by mu
  std::string err_copy;       // the message psara_server_last_error returned last
  std::vector<std::thread> setup_threads;
  std::thread worker;

  bool can_admit() const {
    if (queue.empty() || in_flight >= max_slots) return false;
    return used + queue.front()->foot <= budget || in_flight == 0;
  }
};
