"""Evaluation and stopping quantities (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

* SNR = 20 log10(||s_true|| / ||s - s_true||)  (Sec. 4.7, the printed definition;
  the values of Table 1 were evidently computed with a natural log, so they
  are not compared with);
* NRMSE = sqrt(sum |s - s_true|^2 / sum |s_true|^2)  (Sec. 4.6);
* polarisation error image p and N_p (Sec. 4.2): p_n = ||S_{n,2:4}|| - S_{n,1}
  where that exceeds zeta, zeta = 3 x rms of the Stokes-I residual image.
  Readings: V is included in the norm (all four Stokes maps are solved); the
  residual image is Re phi^dagger(Y - phi(S)) / (2M), 2M approximating the
  peak of the point-spread function of Re phi^dagger phi;
* stopping quantities of Sec. 4.6: residual ||phi(S) - Y||, the maximum over
  Stokes maps of the relative variation between consecutive iterates, and the
  objective ||Psi^dagger S||_{W,1} (eq. g_l1).
"""
from __future__ import annotations

import math

import numpy as np


def snr_db(est: np.ndarray, truth: np.ndarray) -> float:
    return 20.0 * math.log10(np.linalg.norm(truth) / np.linalg.norm(est - truth))


def nrmse(est: np.ndarray, truth: np.ndarray) -> float:
    return float(np.sqrt(np.sum(np.abs(est - truth) ** 2) / np.sum(np.abs(truth) ** 2)))


def residual_norm(mop, S: np.ndarray, Y: np.ndarray) -> float:
    return float(np.linalg.norm(mop.phi(S) - Y))


def relative_variation(S_new: np.ndarray, S_old: np.ndarray) -> np.ndarray:
    """Per Stokes column ||S_new - S_old|| / ||S_old|| (inf where ||S_old|| = 0)."""
    num = np.linalg.norm(S_new - S_old, axis=0)
    den = np.linalg.norm(S_old, axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(den > 0, num / np.where(den > 0, den, 1.0), np.inf)


def weighted_l1(psi_adj, S: np.ndarray, W: np.ndarray) -> float:
    return float(np.sum(W * np.abs(psi_adj(S))))


def polarization_error(mop, S: np.ndarray, Y: np.ndarray):
    """(p image, zeta, N_p in percent)."""
    M = Y.shape[0]
    res = np.real(mop.phi_adj(Y - mop.phi(S))) / (2.0 * M)
    zeta = 3.0 * float(np.sqrt(np.mean(res[:, 0] ** 2)))
    v = np.linalg.norm(S[:, 1:4], axis=1) - S[:, 0]
    p = np.where(v > zeta, v, 0.0)
    return p, zeta, 100.0 * float(np.count_nonzero(p)) / S.shape[0]


def cone_violation(S: np.ndarray) -> float:
    return float(np.max(np.maximum(np.linalg.norm(S[:, 1:4], axis=1) - S[:, 0], 0.0)))
