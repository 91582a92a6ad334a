"""Kaiser-Bessel interpolation kernel (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

The paper's measurement operator interpolates the oversampled FFT grid with
compact-support kernels (Sec. 4.1, eq. meas_op, citing Fessler & Sutton 2003)
without naming the kernel.  Reading: Kaiser-Bessel of width T taps with the
shape parameter of Beatty, Nishimura & Pauly (2005),

    beta = pi * sqrt((T/alpha)^2 (alpha - 1/2)^2 - 0.8),
    psi(t) = I0(beta sqrt(1 - (2t/T)^2)) / I0(beta)   for |t| <= T/2, else 0,

and the scaling of the zero-padding operator Z is 1/psi_hat, with psi_hat the
exact continuous Fourier transform of psi:

    psi_hat(nu) = (T / I0(beta)) sinh(sqrt(beta^2 - (pi T nu)^2)) / sqrt(beta^2 - (pi T nu)^2).

Pinned by numerical quadrature of psi (tests/test_oracle_nufft.py).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import i0


def kb_beta(taps: int, alpha: float) -> float:
    return math.pi * math.sqrt((taps / alpha) ** 2 * (alpha - 0.5) ** 2 - 0.8)


def kb_psi(t, taps: int, beta: float):
    """Kernel value at offset t (grid cells); zero outside |t| <= T/2."""
    t = np.asarray(t, dtype=np.float64)
    u = 1.0 - (2.0 * t / taps) ** 2
    inside = u >= 0.0
    val = i0(beta * np.sqrt(np.where(inside, u, 0.0))) / i0(beta)
    return np.where(inside, val, 0.0)


def kb_psi_hat(nu, taps: int, beta: float):
    """Continuous Fourier transform of kb_psi at frequency nu (cycles per cell)."""
    nu = np.asarray(nu, dtype=np.float64)
    z2 = beta * beta - (math.pi * taps * nu) ** 2
    z = np.sqrt(z2.astype(np.complex128))
    with np.errstate(invalid="ignore", divide="ignore"):
        val = np.where(np.abs(z) > 1e-12, np.sinh(z) / np.where(np.abs(z) > 1e-12, z, 1.0), 1.0)
    return (taps / i0(beta) * val).real
