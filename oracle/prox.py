"""Closed-form projections and thresholding of Polarized SARA (oracle, FP64).

TEST INFRASTRUCTURE ONLY.  Sec. 3.3 ("Primal updates", "Dual updates").
Readings:
  * soft-thresholding: the printed first case carries a sign typo; the standard
    prox of the weighted l1 norm sign(a) max(|a| - t, 0) of the cited Chaux et
    al. (2007) is used (eq. soft_thresh);
  * l2 ball in the dual B step: the radius is epsilon (Moreau identity for the
    indicator of B(Y, epsilon)), not epsilon/rho_2 as printed in Algorithm 1 /
    the data-fidelity paragraph; the printed form would make the fixed point
    satisfy ||phi(S) - Y|| <= epsilon/rho_2, contradicting the stopping rule of
    Sec. 4.6;
  * P_E2 case boundaries: "||r|| <= d keep; else ||r|| <= -d zero; else scale"
    (continuous, and r = 0, d = 0 maps to 0 instead of dividing by zero);
  * P_V and P_E1 keep points on the boundary (both branches agree there).
"""
from __future__ import annotations

import numpy as np


def proj_U(X: np.ndarray) -> np.ndarray:
    """Projection onto real matrices (eq. real_proj)."""
    return np.real(X).astype(np.float64)


def proj_U_prime(X: np.ndarray) -> np.ndarray:
    """Projection onto U' (eq. pos_set): real part, then Stokes I clipped at 0 (Sec. 4.2)."""
    S = np.real(X).astype(np.float64).copy()
    S[:, 0] = np.maximum(S[:, 0], 0.0)
    return S


def proj_V(U: np.ndarray) -> np.ndarray:
    """Projection onto V = {z1 + z2 <= 0} per row (eq. set_V, Proposition 2.1 of Chierchia et al.)."""
    U = np.asarray(U, dtype=np.float64)
    out = U.copy()
    viol = U[:, 0] + U[:, 1] > 0.0
    out[viol, 0] = 0.5 * (U[viol, 0] - U[viol, 1])
    out[viol, 1] = 0.5 * (U[viol, 1] - U[viol, 0])
    return out


def soft_threshold(A: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Component-wise prox of sum t |a| (eq. soft_thresh, sign typo corrected)."""
    return np.sign(A) * np.maximum(np.abs(A) - t, 0.0)


def proj_ball(X: np.ndarray, Y: np.ndarray, radius: float) -> np.ndarray:
    """Projection of X onto the Frobenius ball of centre Y and given radius (data-fidelity paragraph)."""
    diff = X - Y
    nrm = np.sqrt(np.sum(np.abs(diff) ** 2))
    if nrm > radius:
        return radius * diff / nrm + Y
    return X.copy()


def proj_E1(c: np.ndarray, d: np.ndarray):
    """Projection onto the epigraph of h1(s) = -s, pointwise (eq. proj_e1)."""
    c = np.asarray(c, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    keep = c + d >= 0.0
    cc = np.where(keep, c, 0.5 * (c - d))
    dd = np.where(keep, d, 0.5 * (d - c))
    return cc, dd


def proj_E2(R: np.ndarray, d: np.ndarray):
    """Projection onto the epigraph of h2(r) = ||r||_2 (a Lorentz cone), per row (eq. proj_e2_def)."""
    R = np.asarray(R, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    nr = np.sqrt(np.sum(R * R, axis=1))
    keep = nr <= d
    zero = ~keep & (nr <= -d)
    scale = ~keep & ~zero
    a = np.where(scale, 0.5 * (1.0 + d / np.where(scale, nr, 1.0)), 0.0)
    outR = np.where(keep[:, None], R, a[:, None] * R)
    outd = np.where(keep, d, a * nr)
    return outR, outd


def proj_polarization_cone(S: np.ndarray) -> np.ndarray:
    """Direct projection onto P = {||S_{n,2:4}|| <= S_{n,1}} (eq. flux_cons), per pixel.

    P is a product of Lorentz cones, so this is proj_E2 with d = S_{:,1}.  Used
    only as an independent cross-check of the epigraphical splitting.
    """
    R, d = proj_E2(S[:, 1:4], S[:, 0])
    out = np.empty_like(np.asarray(S, dtype=np.float64))
    out[:, 0] = d
    out[:, 1:4] = R
    return out
