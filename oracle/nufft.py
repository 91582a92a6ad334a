"""Measurement operator phi (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

phi(S) = Phi S L with Phi = G F Z (Sec. 4.1, eq. meas_op; the no-DDE case of
eq. RIME).  Phi acts identically on every column of S L, so it is applied per
Stokes column and the rows are then mixed by L (Sec. 2.1: S^T L =
[I+Q, U+iV, U-iV, I-Q]).  The adjoint is phi^dagger(B) = Phi^dagger(B L^H);
the projection onto the real set U (eq. real_proj) takes its real part.

Readings (the paper is silent on these):
  * alpha is the oversampling per dimension, so the grid has (alpha n)^2 cells;
  * pixel (r, c) has centred coordinates (r - n/2, c - n/2) and sits at grid
    index ((r - n/2) mod K, (c - n/2) mod K), K = alpha n;
  * F is the unnormalised forward DFT, and Phi x approximates the direct
    transform  sum_n x_n exp(-i omega . n)  (the sign of eq. RIME);
  * G row m holds psi(t - k) psi(t' - k') over the T x T cells with
    k in [ceil(t - T/2), ceil(t - T/2) + T - 1], t = K omega / (2 pi), indices
    wrapped mod K; G is an explicit CSR matrix so G^H is exact.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .kb import kb_beta, kb_psi, kb_psi_hat

# Stokes -> brightness mixing (Sec. 2.1): row vector [I, Q, U, V] times L.
L_MIX = np.array([[1, 0, 0, 1],
                  [1, 0, 0, -1],
                  [0, 1, 1, 0],
                  [0, 1j, -1j, 0]], dtype=np.complex128)


class NUFFT:
    """Phi = G F Z for single n x n image columns (vectorised row-major, length N = n^2)."""

    def __init__(self, uv: np.ndarray, n: int, oversample: int = 2, taps: int = 6, kernel: str = "kb"):
        uv = np.asarray(uv, dtype=np.float64)
        self.n, self.K, self.T, self.M = n, oversample * n, taps, uv.shape[0]
        K, T = self.K, taps
        if kernel == "kb":
            beta = kb_beta(taps, oversample)
            psi = lambda x: kb_psi(x, taps, beta)
            j = np.arange(n) - n // 2
            s1 = 1.0 / kb_psi_hat(j / K, taps, beta)
        elif kernel == "nearest":
            # delta kernel: weight 1 on the single cell of the window (T = 1), no scaling
            if taps != 1:
                raise ValueError("nearest kernel needs taps == 1")
            psi = lambda x: np.ones_like(x)
            s1 = np.ones(n)
        else:
            raise ValueError(kernel)
        t = K * uv / (2.0 * math.pi)                      # (M, 2) grid coordinates
        k0 = np.ceil(t - T / 2.0).astype(np.int64)        # window starts
        offs = np.arange(T)
        w1 = psi(t[:, 0:1] - (k0[:, 0:1] + offs))         # (M, T)
        w2 = psi(t[:, 1:2] - (k0[:, 1:2] + offs))
        cols = (((k0[:, 0, None, None] + offs[None, :, None]) % K) * K
                + (k0[:, 1, None, None] + offs[None, None, :]) % K)
        data = w1[:, :, None] * w2[:, None, :]
        rows = np.repeat(np.arange(self.M), T * T)
        self.G = sp.csr_matrix((data.ravel(), (rows, cols.ravel())), shape=(self.M, K * K))
        self.GT = self.G.T.tocsr()
        self.k0, self.frac = k0, t - k0
        self.scale = s1[:, None] * s1[None, :]            # Z's scaling, (n, n)
        self.pos = (np.arange(n) - n // 2) % K            # Z's embedding rows / cols

    # Phi: C^N -> C^M, several columns at once ((N,) or (N, c))
    def forward(self, x: np.ndarray) -> np.ndarray:
        n, K = self.n, self.K
        xs = np.asarray(x).reshape(n, n, -1) * self.scale[:, :, None]
        grid = np.zeros((K, K, xs.shape[2]), dtype=np.complex128)
        grid[np.ix_(self.pos, self.pos)] = xs                   # Z
        xf = np.fft.fft2(grid, axes=(0, 1))                     # F
        y = self.G @ xf.reshape(K * K, -1)                      # G
        return y if np.ndim(x) == 2 else y[:, 0]

    # Phi^dagger: C^M -> C^N
    def adjoint(self, y: np.ndarray) -> np.ndarray:
        n, K = self.n, self.K
        yy = np.asarray(y).reshape(self.M, -1)
        g = (self.GT @ yy).reshape(K, K, -1)                    # G^H (G is real)
        z = np.fft.ifft2(g, axes=(0, 1)) * (K * K)              # F^H
        x = z[np.ix_(self.pos, self.pos)] * self.scale[:, :, None]   # Z^H
        x = x.reshape(n * n, -1)
        return x if np.ndim(y) == 2 else x[:, 0]


def direct_dft(x: np.ndarray, uv: np.ndarray, n: int) -> np.ndarray:
    """sum_{r,c} x[r,c] exp(-i (w0 (r - n/2) + w1 (c - n/2))) for each uv row (slow, exact)."""
    j = np.arange(n) - n // 2
    e0 = np.exp(-1j * np.outer(uv[:, 0], j))      # (M, n)
    e1 = np.exp(-1j * np.outer(uv[:, 1], j))
    X = np.asarray(x).reshape(n, n)
    return np.einsum("mr,rc,mc->m", e0, X, e1)


class MeasurementOp:
    """phi(S) = Phi(S) L and phi^dagger(B) = Phi^dagger(B L^H) on N x 4 Stokes matrices.

    With known direction-independent Mueller matrices D_m (eq. RIME, its D with no dependence
    on the sky position), row m of the visibilities is y_m = (Phi S)_m L D_m^T (the transposed
    form of y = D (S^T L)^T), and the adjoint mixes row m of B by (L D_m^T)^H."""

    def __init__(self, nufft: NUFFT, mueller: np.ndarray = None):
        self.nufft = nufft
        self.mix = None if mueller is None else L_MIX @ np.transpose(np.asarray(mueller), (0, 2, 1))

    def phi(self, S: np.ndarray) -> np.ndarray:
        V = self.nufft.forward(np.asarray(S, dtype=np.complex128))
        if self.mix is None:
            return V @ L_MIX
        return np.einsum("ms,msj->mj", V, self.mix)

    def phi_adj(self, B: np.ndarray) -> np.ndarray:
        """Complex N x 4 result; Algorithm 1 applies P_U = Re afterwards."""
        if self.mix is None:
            return self.nufft.adjoint(np.asarray(B) @ L_MIX.conj().T)
        return self.nufft.adjoint(np.einsum("mj,msj->ms", np.asarray(B), self.mix.conj()))
