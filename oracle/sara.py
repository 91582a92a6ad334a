"""SARA sparsity dictionary (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

Psi is the concatenation of the Dirac basis and the first eight Daubechies
wavelet bases (Sec. 3.1, "Sparsifying regularization"; SARA of Carrillo et al.).
Readings (the paper is silent on normalisation, levels, boundaries, phase):
  * Psi = (1/sqrt(nb)) [I, W_1, ..., W_8] with nb = 9 bases, so that
    Psi Psi^dagger = I (a tight frame with ||Psi|| = 1);
  * each W_b is an orthonormal periodised 2-D DWT with a per-problem level
    count; analysis of a length-m signal is
        a_k = sum_j h[j] x[(2k + j) mod m],   d_k = sum_j g[j] x[(2k + j) mod m],
    with g[j] = (-1)^j h[F-1-j], wrap-around summed even when F > m;
  * 2-D: rows first, then columns, recursing on the low-low block; Mallat
    layout  [[LL, HL], [LH, HH]]  in place;  synthesis is the exact transpose;
  * Db_p low-pass filters come from Daubechies' spectral factorisation of
    P(y) = sum_{k<p} C(p-1+k, k) y^k keeping the roots inside the unit circle
    (minimum phase), ordered so that Db2 = (1+r3, 3+r3, 3-r3, 1-r3)/(4 r2).
Coefficient matrices are J x 4 with J = nb N: basis blocks stacked, each block
the n x n Mallat array vectorised row-major.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

BASES = ("dirac", "db1", "db2", "db3", "db4", "db5", "db6", "db7", "db8")


def daubechies_lowpass(p: int) -> np.ndarray:
    """Orthonormal Daubechies low-pass filter with p vanishing moments (length 2p)."""
    if p < 1:
        raise ValueError(p)
    Pk = [math.comb(p - 1 + k, k) for k in range(p)]            # P(y) coefficients, y^0 first
    yroots = np.roots(Pk[::-1]) if p > 1 else np.array([])
    zs = []
    for y in yroots:
        # y = (2 - z - 1/z)/4  <=>  z^2 - (2 - 4y) z + 1 = 0 ; keep the root inside the circle
        b = 2.0 - 4.0 * y
        z1 = (b + np.sqrt(b * b - 4.0 + 0j)) / 2.0
        z2 = (b - np.sqrt(b * b - 4.0 + 0j)) / 2.0
        zs.append(z1 if abs(z1) < 1.0 else z2)
    q = np.poly(zs) if zs else np.array([1.0])                 # highest power first
    binom = np.array([math.comb(p, k) for k in range(p + 1)], dtype=np.float64)   # (1+z)^p
    h = np.real(np.polymul(q, binom))
    return h * (math.sqrt(2.0) / h.sum())


def highpass(h: np.ndarray) -> np.ndarray:
    F = len(h)
    return np.array([(-1) ** j * h[F - 1 - j] for j in range(F)])


@lru_cache(maxsize=None)
def filterbank_matrix(m: int, h_key: tuple) -> np.ndarray:
    """Explicit one-level periodised analysis matrix of size m x m.

    Row k < m/2 holds h[j] at column (2k + j) mod m (approximation a_k);
    row m/2 + k holds g[j] there (detail d_k).  Wrap-around entries add up
    when the filter is longer than m.  The matrix is orthogonal.
    """
    h = np.array(h_key)
    g = highpass(h)
    W = np.zeros((m, m))
    for k in range(m // 2):
        for j in range(len(h)):
            W[k, (2 * k + j) % m] += h[j]
            W[m // 2 + k, (2 * k + j) % m] += g[j]
    return W


def analysis_1d(x: np.ndarray, h: np.ndarray, axis: int):
    """Periodised one-level analysis along `axis`: returns (approx, detail)."""
    xm = np.moveaxis(x, axis, -1)
    m = xm.shape[-1]
    c = xm @ filterbank_matrix(m, tuple(h)).T
    return np.moveaxis(c[..., : m // 2], -1, axis), np.moveaxis(c[..., m // 2:], -1, axis)


def synthesis_1d(a: np.ndarray, d: np.ndarray, h: np.ndarray, axis: int) -> np.ndarray:
    """Exact transpose of analysis_1d."""
    c = np.concatenate([np.moveaxis(a, axis, -1), np.moveaxis(d, axis, -1)], axis=-1)
    m = c.shape[-1]
    return np.moveaxis(c @ filterbank_matrix(m, tuple(h)), -1, axis)


def dwt2(x: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """Multi-level periodised 2-D DWT of the leading two axes (n x n x ...), Mallat layout.

    Each level transforms the rows of the current low-low block (along axis 1),
    then its columns (along axis 0), with the explicit matrix of
    ``filterbank_matrix``.
    """
    c = np.array(x, dtype=np.float64, copy=True)
    m = c.shape[0]
    hk = tuple(h)
    for _ in range(levels):
        W = filterbank_matrix(m, hk)
        blk = c[:m, :m]
        rows = np.matmul(W, blk.reshape(m, m, -1))                  # rows[r] = W @ blk[r]
        c[:m, :m] = (W @ rows.reshape(m, -1)).reshape(blk.shape)    # then columns
        m //= 2
    return c


def idwt2(c: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """Inverse of dwt2 (its transpose, the DWT being orthonormal): columns, then rows."""
    x = np.array(c, dtype=np.float64, copy=True)
    n = x.shape[0]
    hk = tuple(h)
    for lev in reversed(range(levels)):
        m = n >> lev
        W = filterbank_matrix(m, hk)
        blk = x[:m, :m]
        cols = (W.T @ blk.reshape(m, -1)).reshape(m, m, -1)
        x[:m, :m] = np.matmul(W.T, cols).reshape(blk.shape)
    return x


class SARA:
    """Psi and Psi^dagger on N x 4 matrices for a chosen set of bases and level count."""

    def __init__(self, n: int, levels: int, bases=BASES):
        if n % (1 << levels):
            raise ValueError("n must be divisible by 2^levels")
        self.n, self.levels, self.bases = n, levels, tuple(bases)
        self.nb = len(self.bases)
        self.norm = 1.0 / math.sqrt(self.nb)
        self.filters = {b: daubechies_lowpass(int(b[2:])) for b in self.bases if b != "dirac"}

    @property
    def J(self) -> int:
        return self.nb * self.n * self.n

    def adjoint(self, S: np.ndarray) -> np.ndarray:
        """Psi^dagger S: (N, 4) -> (J, 4)."""
        n = self.n
        img = np.asarray(S, dtype=np.float64).reshape(n, n, -1)
        blocks = []
        for b in self.bases:
            cb = img if b == "dirac" else dwt2(img, self.filters[b], self.levels)
            blocks.append(cb.reshape(n * n, -1))
        out = np.concatenate(blocks, axis=0) * self.norm
        return out if np.ndim(S) == 2 else out[:, 0]

    def forward(self, A: np.ndarray) -> np.ndarray:
        """Psi A: (J, 4) -> (N, 4)."""
        n, N = self.n, self.n * self.n
        AA = np.asarray(A, dtype=np.float64).reshape(self.nb * N, -1)
        acc = np.zeros((n, n, AA.shape[1]))
        for i, b in enumerate(self.bases):
            blk = AA[i * N:(i + 1) * N].reshape(n, n, -1)
            acc += blk if b == "dirac" else idwt2(blk, self.filters[b], self.levels)
        out = (acc * self.norm).reshape(N, -1)
        return out if np.ndim(A) == 2 else out[:, 0]
