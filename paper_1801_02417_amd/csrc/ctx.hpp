// The context behind the C ABI's opaque psara_ctx (shared by the C entry points and the
// request server).
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>

#include "engine.hpp"
#include "psara.h"

struct psara_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  psara::Geometry geo;
  bool op_set = false, data_set = false, prior_set = false, steps_set = false, norm_set = false;
  psara_precision prec = PSARA_FP32_MIXED;
  std::unique_ptr<psara::Engine<float>> f32;
  std::unique_ptr<psara::Engine<double>> f64;
  double eps = 0.0, gamma = 0.0, phi_norm_sq = 0.0;
  double tau = 0.0, rho1 = 0.0, rho2 = 0.0, rho3 = 0.0;
  uint32_t mask = 0;
  int levels = 0;
  int tv_kind = 0;            // 0: SARA prior; 1: TV, 2: l1 + TV (Algorithm 3)
  bool mueller = false;       // per-row Mueller matrices in phi
  int64_t iterations = 0;
};

// Binds a host-built geometry (psara::build_geometry) to the context and creates its engine;
// the device half of psara_set_operator.  Throws psara::Error.
void psara_bind_geometry(psara_ctx* c, psara::Geometry&& g, psara_precision precision);
// The argument checks of psara_set_operator.  Throws psara::Error.
void psara_check_operator_args(int n, int64_t M, const double* uv, int oversample, int taps, psara_precision precision);
