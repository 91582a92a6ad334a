// C ABI of the library (declared in include/psara.h): argument validation, the context,
// and the reweighting driver of Algorithm 2.  Every call catches all C++ exceptions and
// returns a status; the message is kept in the context.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "engine.hpp"
#include "psara.h"

using psara::Engine;
using psara::Error;


namespace {

template <class F>
void with_engine(psara_ctx* c, F&& f) {
  if (c->f32) f(*c->f32);
  else if (c->f64) f(*c->f64);
  else throw Error(PSARA_ESTATE, "operator not set");
}

template <class F>
psara_status guard(psara_ctx* c, F&& f) {
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

void require(bool cond, psara_status st, const char* msg) {
  if (!cond) throw Error(st, msg);
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int primal_mode(psara_mode m) {
  switch (m) {
    case PSARA_CONSTRAINED: return psara::PM_CONSTRAINED;
    case PSARA_NNLS_INIT: return psara::PM_INIT;
    case PSARA_UNCONSTRAINED: return psara::PM_UNCONSTRAINED;
  }
  throw Error(PSARA_EINVAL, "unknown mode");
}

// Engine mode of a solve: the TV priors run Algorithm 3 (no initialisation stage)
int solve_mode(const psara_ctx* c, psara_mode m) {
  const int pm = primal_mode(m);
  if (!c->tv_kind) return pm;
  require(pm != psara::PM_INIT, PSARA_EINVAL, "the TV priors have no initialisation stage");
  return pm == psara::PM_CONSTRAINED ? psara::PM_TV_CONSTRAINED : psara::PM_TV_UNCONSTRAINED;
}

void require_sara(const psara_ctx* c) {
  require(!c->tv_kind, PSARA_EINVAL, "not defined for the TV priors (Algorithm 3)");
}

size_t coef_count(const psara_ctx* c) {
  if (c->tv_kind) return (size_t)(c->tv_kind == 2 ? 3 : 2) * c->geo.n * c->geo.n;
  int nb = 0;
  for (int b = 0; b <= 8; ++b) nb += (c->mask >> b) & 1u;
  return (size_t)nb * c->geo.n * c->geo.n;
}

void run_stage(psara_ctx* c, int mode, int iters, int check_every, psara_report* out) {
  require(c->op_set && c->data_set, PSARA_ESTATE, "operator and data must be set before solving");
  require(c->steps_set, PSARA_ESTATE, "step sizes must be set before solving");
  require(mode == psara::PM_INIT || c->prior_set, PSARA_ESTATE, "prior must be set for this mode");
  require(iters >= 0, PSARA_EINVAL, "iters must be >= 0");
  int left = iters;
  const int chunk = check_every > 0 ? check_every : iters;
  psara_report rep;
  std::memset(&rep, 0, sizeof(rep));
  while (left > 0) {
    const int k = std::min(left, std::max(chunk, 1));
    with_engine(c, [&](auto& e) { e.run(mode, k); });
    c->iterations += k;
    left -= k;
    if (check_every > 0) with_engine(c, [&](auto& e) { e.report(&rep); });
  }
  if (out) {
    with_engine(c, [&](auto& e) { e.report(out); });
    out->iterations = c->iterations;
  }
  with_engine(c, [&](auto& e) { psara::hip_check(hipStreamSynchronize(e.stream()), "solve sync"); });
}


// Runs f() for a batch of contexts; an error is recorded in every context.
template <class F>
psara_status batch_guard(psara_ctx* const* ctxs, int count, F&& f) {
  if (!ctxs || count <= 0) return PSARA_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!ctxs[i]) return PSARA_EINVAL;
  auto fail = [&](const std::string& m) { for (int i = 0; i < count; ++i) ctxs[i]->err = m; };
  try {
    if (hipSetDevice(ctxs[0]->device) != hipSuccess) throw Error(PSARA_EDEVICE, "hipSetDevice failed");
    f();
    for (int i = 0; i < count; ++i) ctxs[i]->err.clear();
    return PSARA_OK;
  } catch (const Error& e) {
    fail(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    fail("host allocation failed");
    return PSARA_ENOMEM;
  } catch (const std::exception& e) {
    fail(e.what());
    return PSARA_EDEVICE;
  }
}

void check_batch(psara_ctx* const* ctxs, int count, int mode) {
  for (int i = 0; i < count; ++i) require_sara(ctxs[i]);
  for (int i = 0; i < count; ++i) {
    psara_ctx* c = ctxs[i];
    require(c->op_set && c->data_set, PSARA_ESTATE, "batch member without operator or data");
    require(c->steps_set, PSARA_ESTATE, "batch member without step sizes");
    require(mode == psara::PM_INIT || c->prior_set, PSARA_ESTATE, "batch member without a prior");
    require(c->device == ctxs[0]->device, PSARA_EINVAL, "batch members must share one device");
    require(c->prec == ctxs[0]->prec, PSARA_EINVAL, "batch members must share the precision");
    for (int j = 0; j < i; ++j) require(ctxs[j] != c, PSARA_EINVAL, "a context appears twice in the batch");
  }
}

template <typename R> Engine<R>* engine_of(psara_ctx* c);
template <> Engine<float>* engine_of<float>(psara_ctx* c) { return c->f32.get(); }
template <> Engine<double>* engine_of<double>(psara_ctx* c) { return c->f64.get(); }

template <typename R>
void batch_reweighted(psara_ctx* const* ctxs, int count, int mode, int cycles, const int* iters, double decay,
                      psara_report* reports) {
  std::vector<Engine<R>*> m;
  for (int i = 0; i < count; ++i) m.push_back(engine_of<R>(ctxs[i]));
  psara::Batch<R> b(m, ctxs[0]->stream);
  auto stage = [&](int pm, int k) {
    b.run(pm, k);
    psara::hip_check(hipStreamSynchronize(b.stream()), "batch sync");
    for (int i = 0; i < count; ++i) ctxs[i]->iterations += k;
  };
  if (cycles < 0) {                       // a plain batched stage
    stage(mode, iters[0]);
  } else {
    stage(psara::PM_INIT, iters[0]);
    std::vector<double> delta(count);
    for (int i = 0; i < count; ++i) {
      delta[i] = m[i]->coef_std();
      require(delta[i] > 0.0, PSARA_EINVAL, "initial estimate is zero: no reweighting scale");
    }
    for (int l = 1; l <= cycles; ++l) {
      for (int i = 0; i < count; ++i) m[i]->reweight(delta[i]);
      stage(mode, iters[l]);
      for (int i = 0; i < count; ++i) delta[i] /= decay;
    }
  }
  if (reports)
    for (int i = 0; i < count; ++i) {
      m[i]->report(&reports[i]);
      reports[i].iterations = ctxs[i]->iterations;
    }
}
}  // namespace

void psara_check_operator_args(int n, int64_t M, const double* uv, int oversample, int taps, psara_precision precision) {
  require(is_pow2(n) && n >= 8 && n <= 1024, PSARA_EINVAL, "n must be a power of two in [8, 1024]");
  require(M >= 1 && M < (int64_t(1) << 31), PSARA_EINVAL, "M must be in [1, 2^31)");
  require(uv != nullptr, PSARA_EINVAL, "uv is NULL");
  require(oversample == 2, PSARA_EINVAL, "oversample must be 2");
  require(taps == 4 || taps == 6 || taps == 8, PSARA_EINVAL, "taps must be 4, 6 or 8");
  require(precision == PSARA_FP64 || precision == PSARA_FP32_MIXED, PSARA_EINVAL, "unknown precision");
  for (int64_t i = 0; i < 2 * M; ++i) require(std::isfinite(uv[i]), PSARA_ENAN, "non-finite uv");
}

void psara_bind_geometry(psara_ctx* c, psara::Geometry&& g, psara_precision precision) {
  if (hipSetDevice(c->device) != hipSuccess) throw Error(PSARA_EDEVICE, "hipSetDevice failed");
  c->f32.reset();
  c->f64.reset();
  c->op_set = c->data_set = c->prior_set = c->steps_set = c->norm_set = false;
  c->iterations = 0;
  c->geo = std::move(g);
  c->prec = precision;
  if (precision == PSARA_FP64) c->f64.reset(new Engine<double>(c->geo, c->stream));
  else c->f32.reset(new Engine<float>(c->geo, c->stream));
  c->op_set = true;
}

extern "C" {

const char* psara_status_string(psara_status s) {
  switch (s) {
    case PSARA_OK: return "ok";
    case PSARA_EINVAL: return "invalid argument";
    case PSARA_ENOMEM: return "out of device memory";
    case PSARA_EDEVICE: return "device error";
    case PSARA_ESTATE: return "call out of order";
    case PSARA_ENAN: return "non-finite input";
  }
  return "unknown status";
}

psara_status psara_runtime_check(int* built, int* running) {
  int rt = 0;
  const hipError_t e = hipRuntimeGetVersion(&rt);
  if (built) *built = HIP_VERSION;
  if (running) *running = e == hipSuccess ? rt : 0;
  if (e != hipSuccess) return PSARA_EDEVICE;
  // major * 10^7 + minor * 10^5 + patch: the major and minor versions must agree
  return rt / 100000 == HIP_VERSION / 100000 ? PSARA_OK : PSARA_EDEVICE;
}

psara_status psara_step_sizes(int prior, double phi_norm_sq, double margin, double* out) {
  if (!out || prior < 0 || prior > 2 || !std::isfinite(phi_norm_sq) || !(phi_norm_sq > 0.0) ||
      !std::isfinite(margin) || !(margin > 0.0) || margin > 1.0)
    return PSARA_EINVAL;
  if (prior == 0) {
    // Algorithm 1 with ||Psi|| = 1: rho1 = rho3 = 1, rho2 = 1 / ||phi||^2, and tau at `margin` of
    // the largest value the condition 1/tau >= rho1 ||Psi||^2 + rho2 ||phi||^2 + rho3 allows
    out[1] = 1.0;
    out[2] = 1.0 / phi_norm_sq;
    out[3] = 1.0;
    out[0] = margin / (out[1] + 1.0 + out[3]);          // rho2 ||phi||^2 = 1 exactly

  } else {
    // Algorithm 3: rho1 = 1 / ||Psi||^2 with ||Psi||^2 <= 8 (TV) or 9 (l1 + TV), rho3 = 1, and the
    // data term's gradient Lipschitz constant ||phi||^2 / 2 entering the condition as its half
    const double psi2 = prior == 2 ? 9.0 : 8.0;
    out[1] = 1.0 / psi2;
    out[2] = 1.0;
    out[3] = 1.0;
    out[0] = margin / (0.25 * phi_norm_sq + out[1] * psi2 + out[3]);
  }
  return PSARA_OK;
}

psara_status psara_set_steps_auto(psara_ctx* c, double margin, double* out) {
  if (!c) return PSARA_EINVAL;
  double st[4];
  psara_status s = PSARA_OK;
  s = guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(c->norm_set, PSARA_ESTATE, "run psara_opnorm before setting steps");
    require(psara_step_sizes(c->tv_kind, c->phi_norm_sq, margin, st) == PSARA_OK, PSARA_EINVAL,
            "margin must be in (0, 1]");
  });
  if (s != PSARA_OK) return s;
  s = psara_set_steps(c, st[0], st[1], st[2], st[3]);
  if (s == PSARA_OK && out)
    for (int i = 0; i < 4; ++i) out[i] = st[i];
  return s;
}

psara_status psara_create(psara_ctx** out, int device, void* hip_stream) {
  if (!out) return PSARA_EINVAL;
  *out = nullptr;
  if (psara_runtime_check(nullptr, nullptr) != PSARA_OK) return PSARA_EDEVICE;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return PSARA_EDEVICE;
  if (device < 0 || device >= count) return PSARA_EINVAL;
  std::unique_ptr<psara_ctx> c(new (std::nothrow) psara_ctx());
  if (!c) return PSARA_ENOMEM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) return PSARA_EDEVICE;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return PSARA_EDEVICE;
    c->own_stream = true;
  }
  *out = c.release();
  return PSARA_OK;
}

void psara_destroy(psara_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  c->f32.reset();
  c->f64.reset();
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* psara_last_error(const psara_ctx* c) { return c ? c->err.c_str() : "null context"; }

psara_status psara_set_operator(psara_ctx* c, int n, int64_t M, const double* uv, int oversample, int taps,
                                psara_precision precision) {
  return guard(c, [&] {
    psara_check_operator_args(n, M, uv, oversample, taps, precision);
    psara_bind_geometry(c, psara::build_geometry(n, M, uv, oversample, taps), precision);
  });
}

psara_status psara_set_data(psara_ctx* c, const double* Y, double epsilon) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(Y != nullptr, PSARA_EINVAL, "Y is NULL");
    require(std::isfinite(epsilon) && epsilon > 0.0, PSARA_EINVAL, "epsilon must be finite and > 0");
    const int64_t M = c->geo.M;
    std::vector<double> ys((size_t)M * 8);
    for (int64_t p = 0; p < M; ++p) {
      const double* s = Y + 8 * c->geo.perm[p];
      for (int k = 0; k < 8; ++k) {
        require(std::isfinite(s[k]), PSARA_ENAN, "non-finite visibility");
        ys[8 * p + k] = s[k];
      }
    }
    with_engine(c, [&](auto& e) { e.set_data(ys.data(), epsilon); });
    c->eps = epsilon;
    c->data_set = true;
  });
}

// Whether p is device (or managed) memory of this context's device.
static bool device_buffer(const void* p, int device) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == device;
}

psara_status psara_set_data_dev(psara_ctx* c, const double* Y, double epsilon) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(Y != nullptr, PSARA_EINVAL, "Y is NULL");
    require(std::isfinite(epsilon) && epsilon > 0.0, PSARA_EINVAL, "epsilon must be finite and > 0");
    require(device_buffer(Y, c->device), PSARA_EINVAL, "Y is not device memory of the context's device");
    bool ok = false;
    with_engine(c, [&](auto& e) { ok = e.set_data_dev(Y, epsilon); });
    require(ok, PSARA_ENAN, "non-finite visibility");
    c->eps = epsilon;
    c->data_set = true;
  });
}

psara_status psara_set_mueller(psara_ctx* c, const double* D) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(!(D && c->tv_kind), PSARA_EINVAL, "the TV priors take the data per Stokes map: no Mueller matrices");
    std::vector<double> mix;
    if (D) {
      const int64_t M = c->geo.M;
      mix.resize((size_t)M * 32);
      // L: rows the Stokes maps I, Q, U, V, columns the brightness products (eq. RIME)
      static const double Lre[4][4] = {{1, 0, 0, 1}, {1, 0, 0, -1}, {0, 1, 1, 0}, {0, 0, 0, 0}};
      static const double Lim[4][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 1, -1, 0}};
      for (int64_t p = 0; p < M; ++p) {
        const double* d = D + 32 * c->geo.perm[p];          // D_m[j][k] at d[2 (4 j + k)]
        for (int k = 0; k < 32; ++k) require(std::isfinite(d[k]), PSARA_ENAN, "non-finite Mueller matrix");
        for (int s = 0; s < 4; ++s)
          for (int j = 0; j < 4; ++j) {
            double re = 0.0, im = 0.0;                       // (L D_m^T)[s][j] = sum_k L[s][k] D_m[j][k]
            for (int k = 0; k < 4; ++k) {
              const double dr = d[2 * (4 * j + k)], di = d[2 * (4 * j + k) + 1];
              re += Lre[s][k] * dr - Lim[s][k] * di;
              im += Lre[s][k] * di + Lim[s][k] * dr;
            }
            mix[(size_t)p * 32 + 2 * (4 * s + j)] = re;
            mix[(size_t)p * 32 + 2 * (4 * s + j) + 1] = im;
          }
      }
    }
    with_engine(c, [&](auto& e) { e.set_mixing(D ? mix.data() : nullptr); });
    c->mueller = D != nullptr;
    c->norm_set = false;        // the operator changed: its norm and the step sizes are stale
    c->steps_set = false;
  });
}

psara_status psara_set_prior(psara_ctx* c, uint32_t basis_mask, int levels, const double* weights, double gamma) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(basis_mask != 0 && basis_mask < (1u << 9), PSARA_EINVAL, "basis_mask must select bits 0..8");
    const int n = c->geo.n;
    require(levels >= 1 && levels <= psara::kMaxLevels && (n >> levels) >= 1 && n % (1 << levels) == 0,
            PSARA_EINVAL, "levels must satisfy n divisible by 2^levels");
    require(std::isfinite(gamma) && gamma > 0.0, PSARA_EINVAL, "gamma must be > 0");
    c->mask = basis_mask;
    c->tv_kind = 0;
    const size_t J4 = coef_count(c) * 4;
    if (weights)
      for (size_t i = 0; i < J4; ++i) {
        require(std::isfinite(weights[i]), PSARA_ENAN, "non-finite weight");
        require(weights[i] >= 0.0, PSARA_EINVAL, "weights must be >= 0");
      }
    with_engine(c, [&](auto& e) { e.set_prior(basis_mask, levels, weights, gamma); });
    c->levels = levels;
    c->gamma = gamma;
    c->prior_set = true;
  });
}

psara_status psara_set_prior_tv(psara_ctx* c, int l1, const double* tv_weight, const double* l1_weight) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(!c->mueller, PSARA_EINVAL, "the TV priors take the data per Stokes map: no Mueller matrices");
    require(tv_weight != nullptr && (!l1 || l1_weight != nullptr), PSARA_EINVAL, "weights are NULL");
    for (int i = 0; i < 4; ++i) {
      require(std::isfinite(tv_weight[i]) && tv_weight[i] > 0.0, PSARA_EINVAL, "TV weights must be > 0");
      if (l1) require(std::isfinite(l1_weight[i]) && l1_weight[i] > 0.0, PSARA_EINVAL, "l1 weights must be > 0");
    }
    with_engine(c, [&](auto& e) { e.set_prior_tv(l1 ? 2 : 1, tv_weight, l1 ? l1_weight : nullptr); });
    c->tv_kind = l1 ? 2 : 1;
    c->mask = 0;
    c->levels = 0;
    c->gamma = 1.0;
    c->prior_set = true;
    c->steps_set = false;      // Algorithm 3 has its own step-size condition
  });
}

psara_status psara_set_steps(psara_ctx* c, double tau, double rho1, double rho2, double rho3) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(c->norm_set, PSARA_ESTATE, "run psara_opnorm before setting steps");
    require(tau > 0 && rho1 > 0 && rho2 > 0 && rho3 > 0 && std::isfinite(tau) && std::isfinite(rho1) &&
                std::isfinite(rho2) && std::isfinite(rho3),
            PSARA_EINVAL, "step sizes must be finite and > 0");
    if (c->tv_kind) {
      // the condition with the smooth data term of Algorithm 3: its gradient is
      // ||phi~||^2 = ||phi||^2 / 2 Lipschitz (L L^H = 2 I), ||Psi||^2 <= 8 (TV) or 9 (l1 + TV)
      const double psi2 = c->tv_kind == 2 ? 9.0 : 8.0;
      const double cond = 1.0 / tau - rho1 * psi2 - rho3 - 0.25 * c->phi_norm_sq;
      require(cond >= -1e-12 / tau, PSARA_EINVAL,
              "step sizes violate 1/tau - rho1 ||Psi||^2 - rho3 >= ||phi~||^2 / 2 (Algorithm 3)");
    } else {
      const double cond = 1.0 / tau - rho1 * 1.0 - rho2 * c->phi_norm_sq - rho3;
      require(cond >= -1e-12 / tau, PSARA_EINVAL, "step sizes violate 1/tau - rho1 ||Psi||^2 - rho2 ||phi||^2 - rho3 >= 0");
    }
    with_engine(c, [&](auto& e) { e.set_steps(tau, rho1, rho2, rho3); });
    c->tau = tau; c->rho1 = rho1; c->rho2 = rho2; c->rho3 = rho3;
    c->steps_set = true;
  });
}

psara_status psara_opnorm(psara_ctx* c, int max_iter, double rtol, double* phi_norm_sq) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(max_iter >= 1 && rtol >= 0.0, PSARA_EINVAL, "bad power-iteration parameters");
    double lam = 0.0;
    int its = 0;
    if (c->f64) {
      lam = c->f64->opnorm(max_iter, rtol, &its);
    } else {
      Engine<double> tmp(c->geo, c->stream);
      lam = tmp.opnorm(max_iter, rtol, &its);
    }
    require(std::isfinite(lam) && lam > 0.0, PSARA_EDEVICE, "power iteration did not produce a positive norm");
    c->phi_norm_sq = lam;
    c->norm_set = true;
    c->steps_set = false;
    if (phi_norm_sq) *phi_norm_sq = lam;
  });
}

psara_status psara_solve(psara_ctx* c, psara_mode mode, int iters, int check_every, psara_report* out) {
  return guard(c, [&] { run_stage(c, solve_mode(c, mode), iters, check_every, out); });
}

// ---- the allocation-free iteration ------------------------------------------------------------
// The iteration's scratch buffers (gridding partial slots and FP64 partial sums) of
// psara_solve_noalloc live in this array, one copy per device for the life of the process.  In
// host code `scratch` names a host-side stand-in, not device memory: its device address comes
// from hipGetSymbolAddress, once per device, and only that address is handed to kernels.
constexpr size_t kNoallocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;      // device ordinal -> address of `scratch` on it

// The current device's copy of `scratch` (the caller has made `device` current).
void* scratch_on(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(PSARA_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch_addr[device] = p;
  return p;
}
}  // namespace

psara_status psara_solve_noalloc(psara_ctx* c, psara_mode mode, int iters) {
  return guard(c, [&] {
    const int pm = solve_mode(c, mode);
    require(c->op_set && c->data_set, PSARA_ESTATE, "operator and data must be set before solving");
    require(c->steps_set, PSARA_ESTATE, "step sizes must be set before solving");
    require(pm == psara::PM_INIT || c->prior_set, PSARA_ESTATE, "prior must be set for this mode");
    require(iters >= 0, PSARA_EINVAL, "iters must be >= 0");
    void* scr = scratch_on(c->device);
    with_engine(c, [&](auto& e) { e.run_in_scratch(pm, iters, scr, kNoallocScratchBytes); });
    c->iterations += iters;
  });
}

psara_status psara_capture(psara_ctx* c, psara_mode mode, int iters, int check_every) {
  return guard(c, [&] {
    const int pm = solve_mode(c, mode);
    require(c->op_set && c->data_set && c->steps_set, PSARA_ESTATE, "operator, data and step sizes must be set");
    require(pm == psara::PM_INIT || c->prior_set, PSARA_ESTATE, "prior must be set for this mode");
    require(iters >= 0 && check_every >= 0, PSARA_EINVAL, "iters and check_every must be >= 0");
    // the run lengths psara_solve uses: check_every at a time (the last one shorter), or all
    const int chunk = check_every > 0 ? std::min(check_every, iters) : iters;
    with_engine(c, [&](auto& e) {
      if (chunk > 0) e.capture(pm, chunk);
      if (chunk > 0 && iters % chunk) e.capture(pm, iters % chunk);
    });
  });
}

namespace {
void check_stop(const psara_stop* stop, int max_iters, int check_every) {
  require(stop != nullptr, PSARA_EINVAL, "stop is NULL");
  require(std::isfinite(stop->theta) && stop->theta >= 0.0, PSARA_EINVAL, "stop->theta must be >= 0");
  require(std::isfinite(stop->rel_var) && stop->rel_var >= 0.0, PSARA_EINVAL, "stop->rel_var must be >= 0");
  require(!std::isnan(stop->np_max), PSARA_EINVAL, "stop->np_max is NaN");
  require(max_iters >= 0, PSARA_EINVAL, "max_iters must be >= 0");
  require(check_every >= 1, PSARA_EINVAL, "check_every must be >= 1");
}

int run_stage_adaptive(psara_ctx* c, int mode, int max_iters, int check_every, const psara_stop* stop) {
  require(c->op_set && c->data_set, PSARA_ESTATE, "operator and data must be set before solving");
  require(c->steps_set, PSARA_ESTATE, "step sizes must be set before solving");
  require(mode == psara::PM_INIT || c->prior_set, PSARA_ESTATE, "prior must be set for this mode");
  const double v[3] = {stop->theta, stop->rel_var, stop->np_max};
  int it = 0;
  with_engine(c, [&](auto& e) { it = e.run_adaptive(mode, max_iters, check_every, v); });
  c->iterations += it;
  return it;
}
}  // namespace

psara_status psara_solve_adaptive(psara_ctx* c, psara_mode mode, int max_iters, int check_every,
                                  const psara_stop* stop, int* iters_run, psara_report* out) {
  return guard(c, [&] {
    check_stop(stop, max_iters, check_every);
    const int it = run_stage_adaptive(c, solve_mode(c, mode), max_iters, check_every, stop);
    if (iters_run) *iters_run = it;
    if (out) {
      with_engine(c, [&](auto& e) { e.report(out); });
      out->iterations = c->iterations;
    }
  });
}

psara_status psara_reweighted_solve_adaptive(psara_ctx* c, psara_mode mode, int cycles, int max_iters_per_stage,
                                             int check_every, const psara_stop* stop, double delta_decay,
                                             int* iters_run, psara_report* out) {
  return guard(c, [&] {
    require_sara(c);
    check_stop(stop, max_iters_per_stage, check_every);
    require(cycles >= 0, PSARA_EINVAL, "cycles must be >= 0");
    require(delta_decay > 1.0 && std::isfinite(delta_decay), PSARA_EINVAL, "delta_decay must be > 1");
    require(c->prior_set, PSARA_ESTATE, "prior not set");
    const int pm = primal_mode(mode);
    psara_stop init = *stop;
    init.np_max = -1.0;
    int it = run_stage_adaptive(c, psara::PM_INIT, max_iters_per_stage, check_every, &init);
    if (iters_run) iters_run[0] = it;
    double delta = 0.0;
    with_engine(c, [&](auto& e) { delta = e.coef_std(); });
    require(delta > 0.0, PSARA_EINVAL, "initial estimate is zero: no reweighting scale");
    for (int l = 1; l <= cycles; ++l) {
      with_engine(c, [&](auto& e) { e.reweight(delta); });
      it = run_stage_adaptive(c, pm, max_iters_per_stage, check_every, stop);
      if (iters_run) iters_run[l] = it;
      delta /= delta_decay;
    }
    if (out) {
      with_engine(c, [&](auto& e) { e.report(out); });
      out->iterations = c->iterations;
    }
  });
}

psara_status psara_reweight(psara_ctx* c, double delta) {
  return guard(c, [&] {
    require_sara(c);
    require(c->prior_set, PSARA_ESTATE, "prior not set");
    require(std::isfinite(delta) && delta > 0.0, PSARA_EINVAL, "delta must be > 0");
    with_engine(c, [&](auto& e) { e.reweight(delta); });
  });
}

psara_status psara_coef_std(psara_ctx* c, double* out) {
  return guard(c, [&] {
    require_sara(c);
    require(c->prior_set, PSARA_ESTATE, "prior not set");
    require(out != nullptr, PSARA_EINVAL, "out is NULL");
    with_engine(c, [&](auto& e) { *out = e.coef_std(); });
  });
}

psara_status psara_reweighted_solve(psara_ctx* c, psara_mode mode, int cycles, const int* iters_per_stage,
                                    double delta_decay, psara_report* out) {
  return guard(c, [&] {
    require_sara(c);
    require(cycles >= 0 && iters_per_stage != nullptr, PSARA_EINVAL, "bad stage list");
    require(delta_decay > 1.0 && std::isfinite(delta_decay), PSARA_EINVAL, "delta_decay must be > 1");
    require(c->prior_set, PSARA_ESTATE, "prior not set");
    for (int l = 0; l <= cycles; ++l) require(iters_per_stage[l] >= 0, PSARA_EINVAL, "negative iteration count");
    const int pm = primal_mode(mode);
    run_stage(c, psara::PM_INIT, iters_per_stage[0], 0, nullptr);
    double delta = 0.0;
    with_engine(c, [&](auto& e) { delta = e.coef_std(); });
    require(delta > 0.0, PSARA_EINVAL, "initial estimate is zero: no reweighting scale");
    for (int l = 1; l <= cycles; ++l) {
      with_engine(c, [&](auto& e) { e.reweight(delta); });
      run_stage(c, pm, iters_per_stage[l], 0, (l == cycles) ? out : nullptr);
      delta /= delta_decay;
    }
    if (cycles == 0 && out) {
      with_engine(c, [&](auto& e) { e.report(out); });
      out->iterations = c->iterations;
    }
  });
}

psara_status psara_data_gamma(psara_ctx* c, double factor, double* gamma) {
  return guard(c, [&] {
    require_sara(c);
    require(c->op_set && c->data_set && c->prior_set, PSARA_ESTATE, "operator, data and prior must be set");
    require(c->norm_set, PSARA_ESTATE, "run psara_opnorm first");
    require(gamma != nullptr && std::isfinite(factor) && factor > 0.0, PSARA_EINVAL, "bad arguments");
    double m = 0.0;
    with_engine(c, [&](auto& e) { m = e.data_max_coef(); });
    *gamma = factor * m / c->phi_norm_sq;
  });
}

psara_status psara_set_gamma(psara_ctx* c, double gamma) {
  return guard(c, [&] {
    require_sara(c);
    require(c->prior_set, PSARA_ESTATE, "prior not set");
    require(std::isfinite(gamma) && gamma > 0.0, PSARA_EINVAL, "gamma must be > 0");
    with_engine(c, [&](auto& e) { e.set_gamma(gamma); });
    c->gamma = gamma;
  });
}

psara_status psara_batch_solve(psara_ctx* const* ctxs, int count, psara_mode mode, int iters, psara_report* reports) {
  return batch_guard(ctxs, count, [&] {
    const int pm = primal_mode(mode);
    require(iters >= 0, PSARA_EINVAL, "iters must be >= 0");
    check_batch(ctxs, count, pm);
    if (ctxs[0]->prec == PSARA_FP64) batch_reweighted<double>(ctxs, count, pm, -1, &iters, 10.0, reports);
    else batch_reweighted<float>(ctxs, count, pm, -1, &iters, 10.0, reports);
  });
}

psara_status psara_batch_reweighted_solve(psara_ctx* const* ctxs, int count, psara_mode mode, int cycles,
                                          const int* iters_per_stage, double delta_decay, psara_report* reports) {
  return batch_guard(ctxs, count, [&] {
    const int pm = primal_mode(mode);
    require(cycles >= 0 && iters_per_stage != nullptr, PSARA_EINVAL, "bad stage list");
    require(delta_decay > 1.0 && std::isfinite(delta_decay), PSARA_EINVAL, "delta_decay must be > 1");
    for (int l = 0; l <= cycles; ++l) require(iters_per_stage[l] >= 0, PSARA_EINVAL, "negative iteration count");
    check_batch(ctxs, count, pm);
    for (int i = 0; i < count; ++i) require(ctxs[i]->prior_set, PSARA_ESTATE, "batch member without a prior");
    if (ctxs[0]->prec == PSARA_FP64) batch_reweighted<double>(ctxs, count, pm, cycles, iters_per_stage, delta_decay, reports);
    else batch_reweighted<float>(ctxs, count, pm, cycles, iters_per_stage, delta_decay, reports);
  });
}

psara_status psara_batch_solve_adaptive(psara_ctx* const* ctxs, int count, psara_mode mode, int max_iters,
                                        int check_every, const psara_stop* stop, int* iters_run,
                                        psara_report* reports) {
  return batch_guard(ctxs, count, [&] {
    const int pm = primal_mode(mode);
    check_stop(stop, max_iters, check_every);
    check_batch(ctxs, count, pm);
    const double v[3] = {stop->theta, stop->rel_var, stop->np_max};
    std::vector<int> its(count, 0);
    auto go = [&](auto tag) {
      using R = decltype(tag);
      std::vector<Engine<R>*> m;
      for (int i = 0; i < count; ++i) m.push_back(engine_of<R>(ctxs[i]));
      psara::Batch<R> b(m, ctxs[0]->stream);
      b.run_adaptive(pm, max_iters, check_every, v, its.data());
      for (int i = 0; i < count; ++i) {
        ctxs[i]->iterations += its[i];
        if (iters_run) iters_run[i] = its[i];
        if (reports) {
          m[i]->report(&reports[i]);
          reports[i].iterations = ctxs[i]->iterations;
        }
      }
    };
    if (ctxs[0]->prec == PSARA_FP64) go(double(0));
    else go(float(0));
  });
}

psara_status psara_batch_profile_passes(psara_ctx* const* ctxs, int count, psara_mode mode, int iters,
                                        double* ms_per_pass) {
  return batch_guard(ctxs, count, [&] {
    const int pm = primal_mode(mode);
    require(iters >= 0, PSARA_EINVAL, "iters must be >= 0");
    require(ms_per_pass != nullptr, PSARA_EINVAL, "ms_per_pass is NULL");
    check_batch(ctxs, count, pm);
    auto go = [&](auto tag) {
      using R = decltype(tag);
      std::vector<Engine<R>*> m;
      for (int i = 0; i < count; ++i) m.push_back(engine_of<R>(ctxs[i]));
      psara::Batch<R> b(m, ctxs[0]->stream);
      b.profile(pm, iters, ms_per_pass);
      for (int i = 0; i < count; ++i) ctxs[i]->iterations += 2 * iters;
    };
    if (ctxs[0]->prec == PSARA_FP64) go(double(0));
    else go(float(0));
  });
}

psara_status psara_report_now(psara_ctx* c, psara_report* out) {
  return guard(c, [&] {
    require(c->op_set && c->data_set, PSARA_ESTATE, "operator and data must be set");
    require(out != nullptr, PSARA_EINVAL, "out is NULL");
    with_engine(c, [&](auto& e) { e.report(out); });
    out->iterations = c->iterations;
  });
}

psara_status psara_synchronize(psara_ctx* c) {
  return guard(c, [&] { psara::hip_check(hipStreamSynchronize(c->stream), "synchronize"); });
}

psara_status psara_get_image(psara_ctx* c, double* S) {
  return guard(c, [&] {
    require(S != nullptr, PSARA_EINVAL, "S is NULL");
    with_engine(c, [&](auto& e) { e.get_img(psara::IMG_S, S, 4); });
  });
}

psara_status psara_get_image_dev(psara_ctx* c, double* S) {
  return guard(c, [&] {
    require(S != nullptr, PSARA_EINVAL, "S is NULL");
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(device_buffer(S, c->device), PSARA_EINVAL, "S is not device memory of the context's device");
    with_engine(c, [&](auto& e) { e.get_img_dev(psara::IMG_S, S, 4); });
  });
}

size_t psara_state_bytes(const psara_ctx* c) {
  if (!c || !c->op_set) return 0;
  const size_t N = (size_t)c->geo.n * c->geo.n;
  const size_t J = c->prior_set ? coef_count(c) : 0;
  return sizeof(double) * (N * 4 + N * 2 + J * 4 + (size_t)c->geo.M * 8 + N * 4 + N * 2);
}

psara_status psara_get_state(psara_ctx* c, void* buf, size_t bytes) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(buf != nullptr && bytes >= psara_state_bytes(c), PSARA_EINVAL, "state buffer too small");
    with_engine(c, [&](auto& e) { e.get_state((double*)buf); });
  });
}

psara_status psara_set_state(psara_ctx* c, const void* buf, size_t bytes) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(buf != nullptr && bytes >= psara_state_bytes(c), PSARA_EINVAL, "state buffer too small");
    const double* d = (const double*)buf;
    const size_t cnt = psara_state_bytes(c) / sizeof(double);
    for (size_t i = 0; i < cnt; ++i) require(std::isfinite(d[i]), PSARA_ENAN, "non-finite state");
    with_engine(c, [&](auto& e) { e.set_state(d); });
  });
}

psara_status psara_reset_state(psara_ctx* c) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    with_engine(c, [&](auto& e) { e.zero_state(); });
    c->iterations = 0;
  });
}

size_t psara_footprint(int n, int64_t M, int taps, int levels, uint32_t basis_mask, psara_precision precision) {
  if (!is_pow2(n) || M < 1 || levels < 1) return 0;
  const size_t R = precision == PSARA_FP64 ? 8 : 4;
  const size_t N = (size_t)n * n, K = 2 * (size_t)n;
  const size_t ts = psara::degrid_tile((int)K), ntiles = (K / ts) * (K / ts);
  int nb = 0, nwav = 0;
  for (int b = 0; b <= 8; ++b) nb += (basis_mask >> b) & 1u;
  nwav = nb - (int)(basis_mask & 1u);
  size_t llst = 0;
  for (int l = 1; l < levels; ++l) llst += (size_t)(n >> l) * (n >> l);
  const double spill = (1.0 + (taps - 1.0) / ts) * (1.0 + (taps - 1.0) / ts);
  size_t b = 0;
  b += N * 36 * R;                                   // 8 four-channel and 2 two-channel images
  b += (size_t)M * (24 * R + 4 + 2 * R);             // Y, Bv, R; window starts; offsets
  b += K * K * 8 * R + K * (size_t)n * 8 * R;        // grid and FFT intermediate
  b += (2 * ntiles + 2) * 4 + (size_t)(spill * (double)M + 1) * 4;
  b += 3 * (size_t)nb * N * 4 * R + (size_t)std::max(nwav, 1) * std::max<size_t>(llst, 1) * 4 * R;
  // gridding chunks: at most one per 16 x 16 tile plus one per 256 rows (the smallest chunk the
  // launch shapes allow; runs end a chunk early by at most a run each); each holds a
  // (16 + T - 1)^2 partial slot and a pair of FP64 partials
  const size_t ntg = (K / 16) * (K / 16), rg = 16 + (size_t)taps - 1;
  const size_t chunks = ntg + 2 * ((size_t)M / 256 + 1);
  b += chunks * rg * rg * 8 * R;
  const size_t parts = (size_t)M / 64 + ntiles + 8 * (N / 64 + 64) + chunks;   // de-grid items of >= 64 rows
  b += 2 * parts * 8 + 64 * 8;
  return b;
}

psara_status psara_apply_phi(psara_ctx* c, const double* S, double* Y) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(S && Y, PSARA_EINVAL, "NULL argument");
    with_engine(c, [&](auto& e) { e.apply_phi(S, Y); });
  });
}

psara_status psara_apply_phi_adjoint(psara_ctx* c, const double* B, double* S) {
  return guard(c, [&] {
    require(c->op_set, PSARA_ESTATE, "operator not set");
    require(S && B, PSARA_EINVAL, "NULL argument");
    with_engine(c, [&](auto& e) { e.apply_phi_adjoint(B, S); });
  });
}

psara_status psara_apply_psi_adjoint(psara_ctx* c, const double* S, double* A) {
  return guard(c, [&] {
    require(c->prior_set, PSARA_ESTATE, "prior not set");
    require(S && A, PSARA_EINVAL, "NULL argument");
    with_engine(c, [&](auto& e) { e.apply_psi_adjoint(S, A); });
  });
}

psara_status psara_apply_psi(psara_ctx* c, const double* A, double* S) {
  return guard(c, [&] {
    require(c->prior_set, PSARA_ESTATE, "prior not set");
    require(S && A, PSARA_EINVAL, "NULL argument");
    with_engine(c, [&](auto& e) { e.apply_psi(A, S); });
  });
}

int psara_layout(const psara_ctx* c, int64_t* perm) {
  if (!c || !c->op_set) return PSARA_ESTATE;
  if (perm)
    for (int64_t p = 0; p < c->geo.M; ++p) perm[p] = c->geo.perm[p];
  return c->geo.ts;
}

psara_status psara_profile_passes(psara_ctx* c, psara_mode mode, int iters, double* ms_per_pass) {
  return guard(c, [&] {
    require_sara(c);
    const int pm = primal_mode(mode);
    require(c->op_set && c->data_set && c->steps_set, PSARA_ESTATE, "solve set-up incomplete");
    require(pm == psara::PM_INIT || c->prior_set, PSARA_ESTATE, "prior not set");
    require(iters >= 1 && ms_per_pass != nullptr, PSARA_EINVAL, "bad iteration count or output");
    with_engine(c, [&](auto& e) { e.profile(pm, iters, ms_per_pass); });
    c->iterations += iters;
  });
}

}  // extern "C"
