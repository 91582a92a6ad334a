// The request server's device layer on HIP (the scheduler is server_core.cpp): a request's
// solve is a psara context; a group's lane is a batch of those contexts advanced on a stream
// of its own, so groups of different sizes overlap on the GPU.  Only the server's worker thread
// calls into this layer's device methods (the set-up threads only build the host geometry),
// so no other thread makes a HIP call while the worker captures a graph.
#include <hip/hip_runtime.h>

#include <chrono>
#include <memory>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "engine.hpp"
#include "server_core.hpp"
#include "psara.h"

namespace psara {
namespace serve {
namespace {

struct HipHost : HostPrep {
  Geometry geo;
};

struct HipSolve : Solve {
  psara_ctx* c = nullptr;
  ~HipSolve() override {
    if (c) psara_destroy(c);
  }
};

psara_ctx* ctx_of(Job& j) {
  auto* s = static_cast<HipSolve*>(j.solve.get());
  if (!s || !s->c) throw Error(PSARA_ESTATE, "request has no device state");
  return s->c;
}

void ok(psara_ctx* c, psara_status st) {
  if (st != PSARA_OK) throw Error(st, psara_last_error(c));
}

int engine_mode(int kind) {
  if (kind == SK_INIT) return PM_INIT;
  return kind == SK_UNCONSTRAINED ? PM_UNCONSTRAINED : PM_CONSTRAINED;
}

struct HipLane : Lane {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::unique_ptr<Batch<float>> bf;
  std::unique_ptr<Batch<double>> bd;

  explicit HipLane(int dev) : device(dev) {
    hip_check(hipSetDevice(device), "hipSetDevice");
    hip_check(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking), "lane stream");
    hip_check(hipEventCreate(&e0), "lane event");
    hip_check(hipEventCreate(&e1), "lane event");
  }
  ~HipLane() override {
    (void)hipSetDevice(device);
    drop();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (stream) (void)hipStreamDestroy(stream);
  }
  void prepare(const std::vector<Job*>& members, bool rebuild, int kind, int check_every) override {
    hip_check(hipSetDevice(device), "hipSetDevice");
    if (rebuild || (!bf && !bd)) {
      drop();
      if (members[0]->req.precision == PSARA_FP64) {
        std::vector<Engine<double>*> e;
        for (Job* j : members) e.push_back(ctx_of(*j)->f64.get());
        bd.reset(new Batch<double>(e, stream));
      } else {
        std::vector<Engine<float>*> e;
        for (Job* j : members) e.push_back(ctx_of(*j)->f32.get());
        bf.reset(new Batch<float>(e, stream));
      }
    }
    const int mode = engine_mode(kind);
    if (check_every > 0) {
      if (bd) bd->capture_adaptive(mode, check_every);
      else bf->capture_adaptive(mode, check_every);
    } else if (bd) {
      bd->capture(mode);
    } else {
      bf->capture(mode);
    }
  }
  void launch(int kind, int iters, int check_every) override {
    hip_check(hipSetDevice(device), "hipSetDevice");
    const int mode = engine_mode(kind);
    hip_check(hipEventRecord(e0, stream), "round start");
    if (check_every > 0) {
      if (bd) bd->launch_adaptive(mode, iters / check_every, check_every);
      else bf->launch_adaptive(mode, iters / check_every, check_every);
    } else if (bd) {
      bd->run(mode, iters);
    } else {
      bf->run(mode, iters);
    }
    hip_check(hipEventRecord(e1, stream), "round end");
  }
  double wait() override {
    hip_check(hipEventSynchronize(e1), "round wait");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "round time");
    return 1e-3 * ms;
  }
  void drop() override {
    bf.reset();
    bd.reset();
  }
};

class HipDevice : public Device {
 public:
  explicit HipDevice(int device) : device_(device), t0_(std::chrono::steady_clock::now()) {
    int built = 0, running = 0;
    if (psara_runtime_check(&built, &running) != PSARA_OK)
      throw Error(PSARA_EDEVICE, "HIP runtime " + std::to_string(running) + " in this process, library built for " +
                                     std::to_string(built));
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) throw Error(PSARA_EDEVICE, "no device");
    if (device < 0 || device >= count) throw Error(PSARA_EINVAL, "bad device ordinal");
    hip_check(hipSetDevice(device), "hipSetDevice");
    size_t free_b = 0;
    hip_check(hipMemGetInfo(&free_b, &total_), "hipMemGetInfo");
  }
  double now() override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }
  size_t capacity() override { return total_; }
  size_t footprint(const psara_request& r) override {
    return psara_footprint(r.n, r.M, r.taps, r.levels, r.basis_mask, r.precision);
  }
  void prepare_host(Job& j) override {
    const psara_request& r = j.req;
    psara_check_operator_args(r.n, r.M, j.uv.data(), 2, r.taps, r.precision);
    std::unique_ptr<HipHost> h(new HipHost());
    h->geo = build_geometry(r.n, r.M, j.uv.data(), 2, r.taps);
    j.host = std::move(h);
  }
  std::unique_ptr<Solve> open(Job& j) override {
    const psara_request& r = j.req;
    auto* h = static_cast<HipHost*>(j.host.get());
    if (!h) throw Error(PSARA_ESTATE, "request was not set up on the host");
    std::unique_ptr<HipSolve> s(new HipSolve());
    psara_status st = psara_create(&s->c, device_, nullptr);
    if (st != PSARA_OK) throw Error(st, "context creation failed");
    psara_ctx* c = s->c;
    try {
      psara_bind_geometry(c, std::move(h->geo), r.precision);
    } catch (const std::exception& e) {
      throw Error(PSARA_EDEVICE, e.what());
    }
    ok(c, psara_set_data(c, j.Y.data(), r.epsilon));
    ok(c, psara_set_prior(c, r.basis_mask, r.levels, nullptr, 1.0));
    double nrm = 0.0, g = 0.0;
    ok(c, psara_opnorm(c, r.opnorm_iters, r.opnorm_rtol, &nrm));
    ok(c, psara_data_gamma(c, r.gamma_factor, &g));
    if (!(g > 0.0)) throw Error(PSARA_EINVAL, "data-driven gamma is zero");
    ok(c, psara_set_gamma(c, g));
    ok(c, psara_set_steps_auto(c, 0.99, nullptr));
    psara_tuning t;
    if (psara_tuning_lookup(r.n, r.M, r.taps, r.levels, r.basis_mask, r.precision, &t) == PSARA_OK)
      ok(c, psara_set_tuning(c, &t));
    return s;
  }
  void stop_begin(Job& j, const double crit[3], int bound) override {
    psara_ctx* c = ctx_of(j);
    hip_check(hipSetDevice(device_), "hipSetDevice");
    if (c->f64) c->f64->stop_begin(crit, bound);
    else c->f32->stop_begin(crit, bound);
  }
  void stop_poll(Job& j, bool* halted, int* iters) override {
    psara_ctx* c = ctx_of(j);
    hip_check(hipSetDevice(device_), "hipSetDevice");
    if (c->f64) c->f64->stop_poll(halted, iters);
    else c->f32->stop_poll(halted, iters);
  }
  void stop_end(Job& j) override {
    psara_ctx* c = ctx_of(j);
    hip_check(hipSetDevice(device_), "hipSetDevice");
    if (c->f64) (void)c->f64->stop_end();
    else (void)c->f32->stop_end();
  }
  double coef_std(Job& j) override {
    psara_ctx* c = ctx_of(j);
    double d = 0.0;
    ok(c, psara_coef_std(c, &d));
    return d;
  }
  void reweight(Job& j, double delta) override {
    psara_ctx* c = ctx_of(j);
    ok(c, psara_reweight(c, delta));
  }
  void finish(Job& j, psara_report* rep, std::vector<double>* image) override {
    psara_ctx* c = ctx_of(j);
    image->assign((size_t)j.req.n * j.req.n * 4, 0.0);
    ok(c, psara_report_now(c, rep));
    ok(c, psara_get_image(c, image->data()));
  }
  std::unique_ptr<Lane> lane() override { return std::unique_ptr<Lane>(new HipLane(device_)); }

 private:
  int device_ = 0;
  size_t total_ = 0;
  std::chrono::steady_clock::time_point t0_;
};

}  // namespace

std::unique_ptr<Device> make_device(int device) { return std::unique_ptr<Device>(new HipDevice(device)); }

}  // namespace serve
}  // namespace psara
