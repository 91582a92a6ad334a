"""Assemble an imaging problem from a workload (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

Measurements follow eq. RIME_disc, Y = phi(S_true) + E, with E i.i.d. circular
complex Gaussian of variance sigma^2 per entry (sigma^2/2 per real and
imaginary part, Sec. 4.1).  The paper fixes sigma = 5e-3 for its M87 models; the
synthetic workloads instead fix an input SNR, sigma = ||phi(S_true)||_F /
sqrt(4M) * 10^(-ISNR/20) (a reading).  The l2 bound is the chi-square rule of
Sec. 4.1 with 8M real degrees of freedom:
    epsilon^2 = (8M + 2 sqrt(2 * 8M)) sigma^2 / 2.
The free parameter gamma (Sec. 3.3.1, "only affects the convergence speed") is
set from the data, gamma = 1e-3 ||Psi^dagger Re phi^dagger(Y)||_inf / ||phi||^2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .nufft import NUFFT, MeasurementOp
from .sara import SARA, BASES
from .pd import Problem, step_sizes, phi_norm_sq


def chi2_epsilon(M: int, sigma: float) -> float:
    return math.sqrt((8 * M + 2 * math.sqrt(2 * 8 * M)) * sigma * sigma / 2.0)


@dataclass
class Built:
    pb: Problem
    mop: MeasurementOp
    sara: SARA
    truth: np.ndarray      # (N, 4)
    sigma: float
    phi_norm_sq: float
    gamma: float


def build(wl, bases=BASES, levels=None, phi_norm=None, gamma=None, norm_rtol=1e-12, norm_max_iter=1000,
          mueller=None) -> Built:
    """mueller: None, or (M, 4, 4) known direction-independent Mueller matrices of the rows."""
    n = wl.n
    nu = NUFFT(wl.uv, n, wl.oversample, wl.taps)
    mop = MeasurementOp(nu, mueller)
    sara = SARA(n, wl.levels if levels is None else levels, bases)
    truth = wl.truth.reshape(n * n, 4)
    y0 = mop.phi(truth)
    sigma = np.linalg.norm(y0) / math.sqrt(4 * wl.M) * 10.0 ** (-wl.isnr_db / 20.0)
    Y = y0 + sigma * wl.noise
    eps = chi2_epsilon(wl.M, sigma)
    if phi_norm is None:
        phi_norm, _ = phi_norm_sq(mop, n * n, max_iter=norm_max_iter, rtol=norm_rtol)
    tau, r1, r2, r3 = step_sizes(phi_norm)
    if gamma is None:
        gamma = 1e-3 * float(np.max(np.abs(sara.adjoint(np.real(mop.phi_adj(Y)))))) / phi_norm
    pb = Problem(mop.phi, mop.phi_adj, sara.forward, sara.adjoint, Y, eps, tau, r1, r2, r3)
    return Built(pb, mop, sara, truth, sigma, phi_norm, gamma)
