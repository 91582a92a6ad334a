// The autotuner of the C ABI (psara_autotune, psara_batch_autotune, psara_get/set_tuning,
// psara_tuning_lookup): it times the iteration of a solve (or of a batch) under candidate
// launch shapes -- gridding chunk size, de-gridding work-item size, analysis tile width, FFT
// cells per workgroup -- one parameter at a time, keeps the fastest, and can remember the
// choice per shape class for later solves of that class (the request server takes it from
// there).  The shapes change the launch geometry and the summation order of the gridding and
// of the de-gridding norm, not what is computed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ctx.hpp"
#include "engine.hpp"
#include "psara.h"

using psara::Batch;
using psara::Engine;
using psara::Error;
using psara::Tuning;

namespace {

psara::Tuning from_c(const psara_tuning& t) {
  Tuning u;
  u.grid_chunk = t.grid_chunk;
  u.degrid_item = t.degrid_item;
  u.ana_wide = t.analysis_wide;
  u.fft_cells = t.fft_cells;
  return u;
}

psara_tuning to_c(const Tuning& u) {
  psara_tuning t;
  t.grid_chunk = u.grid_chunk;
  t.degrid_item = u.degrid_item;
  t.analysis_wide = u.ana_wide;
  t.fft_cells = u.fft_cells;
  return t;
}

// ---- the per-class cache -----------------------------------------------------------------------
// shape class: precision, taps, image side, levels, basis mask, visibility count to the nearest
// power of two below
using ClassKey = std::tuple<int, int, int, int, uint32_t, int>;
std::mutex g_cache_mu;
std::map<ClassKey, Tuning> g_cache;

ClassKey class_of(int prec, int taps, int n, int levels, uint32_t mask, int64_t M) {
  int b = 0;
  while ((int64_t(2) << b) <= M) ++b;
  return std::make_tuple(prec, taps, n, levels, mask, b);
}

ClassKey class_of(const psara_ctx* c) {
  return class_of((int)c->prec, c->geo.T, c->geo.n, c->levels, c->mask, c->geo.M);
}

template <class F>
psara_status guarded(psara_ctx* c, F&& f) {
  if (!c) return PSARA_EINVAL;
  try {
    if (hipSetDevice(c->device) != hipSuccess) throw Error(PSARA_EDEVICE, "hipSetDevice failed");
    f();
    c->err.clear();
    return PSARA_OK;
  } catch (const Error& e) {
    c->err = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return PSARA_ENOMEM;
  } catch (const std::exception& e) {
    c->err = e.what();
    return PSARA_EDEVICE;
  }
}

int engine_mode(const psara_ctx* c, psara_mode m) {
  int pm = m == PSARA_NNLS_INIT ? psara::PM_INIT : (m == PSARA_UNCONSTRAINED ? psara::PM_UNCONSTRAINED : psara::PM_CONSTRAINED);
  if (m != PSARA_CONSTRAINED && m != PSARA_NNLS_INIT && m != PSARA_UNCONSTRAINED) throw Error(PSARA_EINVAL, "unknown mode");
  if (c->tv_kind) {
    if (pm == psara::PM_INIT) throw Error(PSARA_EINVAL, "the TV priors have no initialisation stage");
    pm = pm == psara::PM_CONSTRAINED ? psara::PM_TV_CONSTRAINED : psara::PM_TV_UNCONSTRAINED;
  }
  return pm;
}

void require_ready(const psara_ctx* c, int pm) {
  if (!(c->op_set && c->data_set && c->steps_set)) throw Error(PSARA_ESTATE, "operator, data and step sizes must be set");
  if (pm != psara::PM_INIT && !c->prior_set) throw Error(PSARA_ESTATE, "prior must be set for this mode");
}

// Seconds per iteration of `run`, which queues `iters` iterations on `stream`: the best of three
// timed runs after one untimed run (which also captures the graphs).
template <class F>
double time_runs(F&& run, hipStream_t stream, int iters) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  psara::hip_check(hipEventCreate(&e0), "event");
  psara::hip_check(hipEventCreate(&e1), "event");
  double best = 1e30;
  try {
    run();
    psara::hip_check(hipStreamSynchronize(stream), "tuning warm-up");
    for (int r = 0; r < 3; ++r) {
      psara::hip_check(hipEventRecord(e0, stream), "event");
      run();
      psara::hip_check(hipEventRecord(e1, stream), "event");
      psara::hip_check(hipEventSynchronize(e1), "event");
      float ms = 0.f;
      psara::hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
      best = std::min(best, 1e-3 * ms / iters);
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

// Coordinate search over the four parameters from `start`, each candidate timed by `measure`
// (which applies it); a candidate must beat the incumbent by 1 % to replace it.  Returns the
// choice and writes the time of `start` and of the choice.
template <class M>
Tuning search(const Tuning& start, int K, bool fp32, M&& measure, double* t_start, double* t_best) {
  Tuning best = start;
  double tb = measure(best);
  *t_start = tb;
  auto consider = [&](Tuning cand) {
    try {
      psara::check_tuning(cand, K);
    } catch (const Error&) {
      return;
    }
    const double t = measure(cand);
    if (t < 0.99 * tb) {
      tb = t;
      best = cand;
    }
  };
  for (int v : {1024, 512, 256})
    if (v != best.grid_chunk) { Tuning c = best; c.grid_chunk = v; consider(c); }
  for (int v : {256, 128, 512})
    if (v != best.degrid_item) { Tuning c = best; c.degrid_item = v; consider(c); }
  // (FP64 analysis tiles are 8 wide either way, so there only the all-bases bit is a candidate)
  for (int v : {1, 0, 3, 2})
    if (v != best.ana_wide && (fp32 || v == (best.ana_wide ^ psara::kAnaAllBases))) {
      Tuning c = best;
      c.ana_wide = v;
      consider(c);
    }
  for (int v : {0, 1024, 2048})
    if (v != best.fft_cells && (v == 0 || v > std::max(512, K))) { Tuning c = best; c.fft_cells = v; consider(c); }
  measure(best);        // leaves the choice applied
  *t_best = tb;
  return best;
}

template <typename R>
Engine<R>* engine_of(psara_ctx* c);
template <> Engine<float>* engine_of<float>(psara_ctx* c) { return c->f32.get(); }
template <> Engine<double>* engine_of<double>(psara_ctx* c) { return c->f64.get(); }

constexpr int kTrialIters = 8;   // iterations per timed run (one captured chain)

template <typename R>
Tuning tune_one(psara_ctx* c, int pm, double* t0, double* t1) {
  Engine<R>* e = engine_of<R>(c);
  const size_t nb = psara_state_bytes(c);
  std::vector<double> keep(nb / sizeof(double));
  e->get_state(keep.data());
  Tuning best;
  try {
    auto measure = [&](const Tuning& t) {
      e->set_tuning(t);
      return time_runs([&] { e->run(pm, kTrialIters); }, e->stream(), kTrialIters);
    };
    best = search(e->tuning(), c->geo.K, std::is_same<R, float>::value, measure, t0, t1);
  } catch (...) {
    e->set_state(keep.data());
    throw;
  }
  e->set_state(keep.data());
  return best;
}

template <typename R>
Tuning tune_batch(psara_ctx* const* ctxs, int count, int pm, double* t0, double* t1) {
  std::vector<Engine<R>*> m;
  std::vector<std::vector<double>> keep(count);
  for (int i = 0; i < count; ++i) {
    m.push_back(engine_of<R>(ctxs[i]));
    keep[i].resize(psara_state_bytes(ctxs[i]) / sizeof(double));
    m[i]->get_state(keep[i].data());
  }
  int Kmax = 0;
  for (auto* e : m) Kmax = std::max(Kmax, e->geometry().K);
  auto restore = [&] {
    for (int i = 0; i < count; ++i) m[i]->set_state(keep[i].data());
  };
  Tuning best;
  try {
    auto measure = [&](const Tuning& t) {
      for (auto* e : m) e->set_tuning(t);
      Batch<R> b(m, ctxs[0]->stream);
      return time_runs([&] { b.run(pm, kTrialIters); }, b.stream(), kTrialIters);
    };
    best = search(m[0]->tuning(), Kmax, std::is_same<R, float>::value, measure, t0, t1);
  } catch (...) {
    restore();
    throw;
  }
  restore();
  return best;
}

}  // namespace

extern "C" {

psara_status psara_get_tuning(const psara_ctx* c, psara_tuning* out) {
  if (!c || !out) return PSARA_EINVAL;
  if (!c->op_set) return PSARA_ESTATE;
  *out = to_c(c->f64 ? c->f64->tuning() : c->f32->tuning());
  return PSARA_OK;
}

psara_status psara_set_tuning(psara_ctx* c, const psara_tuning* t) {
  return guarded(c, [&] {
    if (!c->op_set) throw Error(PSARA_ESTATE, "operator not set");
    const Tuning u = t ? from_c(*t) : Tuning();
    psara::check_tuning(u, c->geo.K);
    if (c->f64) c->f64->set_tuning(u);
    else c->f32->set_tuning(u);
  });
}

psara_status psara_autotune(psara_ctx* c, psara_mode mode, int flags, psara_tuning* chosen, double* ms_per_iter) {
  return guarded(c, [&] {
    const int pm = engine_mode(c, mode);
    require_ready(c, pm);
    if (flags & ~(PSARA_TUNE_USE_CACHE | PSARA_TUNE_STORE)) throw Error(PSARA_EINVAL, "unknown tuning flags");
    if (flags & PSARA_TUNE_USE_CACHE) {
      Tuning hit;
      bool found = false;
      {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(class_of(c));
        if (it != g_cache.end()) { hit = it->second; found = true; }
      }
      if (found) {
        if (c->f64) c->f64->set_tuning(hit);
        else c->f32->set_tuning(hit);
        if (chosen) *chosen = to_c(hit);
        if (ms_per_iter) ms_per_iter[0] = ms_per_iter[1] = 0.0;
        return;
      }
    }
    double t0 = 0.0, t1 = 0.0;
    const Tuning best = c->f64 ? tune_one<double>(c, pm, &t0, &t1) : tune_one<float>(c, pm, &t0, &t1);
    if (flags & PSARA_TUNE_STORE) {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      g_cache[class_of(c)] = best;
    }
    if (chosen) *chosen = to_c(best);
    if (ms_per_iter) {
      ms_per_iter[0] = 1e3 * t0;
      ms_per_iter[1] = 1e3 * t1;
    }
  });
}

psara_status psara_batch_autotune(psara_ctx* const* ctxs, int count, psara_mode mode, psara_tuning* chosen,
                                  double* ms_per_iter) {
  if (!ctxs || count <= 0) return PSARA_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!ctxs[i]) return PSARA_EINVAL;
  return guarded(ctxs[0], [&] {
    const int pm = engine_mode(ctxs[0], mode);
    for (int i = 0; i < count; ++i) {
      if (ctxs[i]->tv_kind) throw Error(PSARA_EINVAL, "batches take the SARA prior only");
      require_ready(ctxs[i], pm);
      if (ctxs[i]->prec != ctxs[0]->prec || ctxs[i]->device != ctxs[0]->device || ctxs[i]->geo.T != ctxs[0]->geo.T)
        throw Error(PSARA_EINVAL, "batch members must share device, precision and tap count");
      for (int j = 0; j < i; ++j)
        if (ctxs[j] == ctxs[i]) throw Error(PSARA_EINVAL, "a context appears twice in the batch");
    }
    double t0 = 0.0, t1 = 0.0;
    const Tuning best = ctxs[0]->f64 ? tune_batch<double>(ctxs, count, pm, &t0, &t1)
                                     : tune_batch<float>(ctxs, count, pm, &t0, &t1);
    if (chosen) *chosen = to_c(best);
    if (ms_per_iter) {
      ms_per_iter[0] = 1e3 * t0;
      ms_per_iter[1] = 1e3 * t1;
    }
  });
}

psara_status psara_tuning_lookup(int n, int64_t M, int taps, int levels, uint32_t basis_mask, psara_precision precision,
                                 psara_tuning* out) {
  if (!out) return PSARA_EINVAL;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(class_of((int)precision, taps, n, levels, basis_mask, M));
  if (it == g_cache.end()) return PSARA_ESTATE;
  *out = to_c(it->second);
  return PSARA_OK;
}

}  // extern "C"
