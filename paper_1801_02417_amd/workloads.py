"""Seeded synthetic workloads shaped like the paper's polarimetric VLBI imaging runs.

This module only draws random inputs: ground-truth Stokes maps, uv sampling
points and unit-variance noise.  It contains none of the imaging method's
arithmetic (no measurement operator, no wavelets, no projections), so both the
FP64 CPU oracle and the HIP library can consume it.

Shapes follow the paper's simulation setup (Sec. 4.1, "Simulation Setup"):
compact, non-negative total-intensity emission with a smooth linear polarisation
fraction and angle (the polarisation cone of eq. flux_bound holds pixel-wise),
sparse VLBI coverage made of Earth-rotation arcs from a handful of stations, and
i.i.d. complex Gaussian noise per correlation column (eq. RIME_disc).  The
paper's own EHT coverage and M87 models are not available, so the recipes below
stand in for them.

Conventions shared with every consumer:
  * images are ``(n, n, 4)`` float64 arrays, axis 0 = rows, axis 1 = columns,
    last axis = Stokes (I, Q, U, V); pixel (r, c) has centred coordinates
    (r - n/2, c - n/2);
  * ``uv`` is ``(M, 2)`` float64 in radians per pixel, each component in
    [-pi, pi); component 0 pairs with the row axis, component 1 with columns;
  * ``noise`` is ``(M, 4)`` complex128 with E|e|^2 = 1 (variance 1/2 per real
    and imaginary part).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import gaussian_filter

BASE_SEED = 2417


@dataclass
class Workload:
    """One imaging problem: ground truth, sampling and noise draws."""
    name: str
    n: int
    M: int
    taps: int
    oversample: int
    levels: int
    isnr_db: float
    iters: int
    cycles: int
    truth: np.ndarray          # (n, n, 4) float64
    uv: np.ndarray             # (M, 2) float64, rad/pixel
    noise: np.ndarray          # (M, 4) complex128, unit variance
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# smooth random fields and polarisation
# ----------------------------------------------------------------------------
def smooth_field(rng: np.random.Generator, n: int) -> np.ndarray:
    """Gaussian-filtered white noise (sigma = n/8, periodic), min-max scaled to [0, 1]."""
    f = gaussian_filter(rng.standard_normal((n, n)), sigma=n / 8.0, mode="wrap")
    lo, hi = f.min(), f.max()
    return (f - lo) / (hi - lo)


def add_polarisation(rng: np.random.Generator, I: np.ndarray, max_fraction: float = 0.6) -> np.ndarray:
    """Stokes cube from I: m ~ smooth in [0, max_fraction], chi smooth in [-pi/2, pi/2], V = 0.01 I."""
    n = I.shape[0]
    m = max_fraction * smooth_field(rng, n)
    chi = 0.5 * math.pi * (2.0 * smooth_field(rng, n) - 1.0)
    S = np.empty((n, n, 4))
    S[..., 0] = I
    S[..., 1] = m * I * np.cos(2.0 * chi)
    S[..., 2] = m * I * np.sin(2.0 * chi)
    S[..., 3] = 0.01 * I
    return S


def _coords(n: int):
    r = np.arange(n, dtype=np.float64)[:, None] * np.ones((1, n))
    c = np.ones((n, 1)) * np.arange(n, dtype=np.float64)[None, :]
    return r, c


def blobs_image(rng: np.random.Generator, n: int, count: int = 3) -> np.ndarray:
    """Sum of `count` isotropic Gaussian blobs (amplitude U(0.5,1), width U(1.5,4) px)."""
    r, c = _coords(n)
    I = np.zeros((n, n))
    for _ in range(count):
        a = rng.uniform(0.5, 1.0)
        s = rng.uniform(1.5, 4.0)
        cr, cc = rng.uniform(0.25 * n, 0.75 * n, size=2)
        I += a * np.exp(-((r - cr) ** 2 + (c - cc) ** 2) / (2.0 * s * s))
    return I


def ring_jet_image(rng: np.random.Generator, n: int) -> np.ndarray:
    """Thin asymmetric annulus plus an elliptical Gaussian jet (black-hole-shadow-like)."""
    r, c = _coords(n)
    dy, dx = r - n / 2.0, c - n / 2.0
    rad = np.hypot(dy, dx)
    th = np.arctan2(dy, dx)
    r0, w = 0.22 * n, 0.025 * n
    th0 = rng.uniform(0.0, 2.0 * math.pi)
    ring = np.exp(-((rad - r0) ** 2) / (2.0 * w * w)) * (1.0 + 0.6 * np.cos(th - th0))
    peak = ring.max()
    thj = rng.uniform(0.0, 2.0 * math.pi)
    jy, jx = 0.25 * n * math.sin(thj), 0.25 * n * math.cos(thj)
    ey, ex = dy - jy, dx - jx
    along = ex * math.cos(thj) + ey * math.sin(thj)
    across = -ex * math.sin(thj) + ey * math.cos(thj)
    smaj, smin = 0.12 * n, 0.02 * n
    jet = 0.3 * peak * np.exp(-0.5 * ((along / smaj) ** 2 + (across / smin) ** 2))
    return ring + jet


def add_knots(rng: np.random.Generator, I: np.ndarray, count: int = 20) -> np.ndarray:
    n = I.shape[0]
    r, c = _coords(n)
    peak = I.max()
    out = I.copy()
    for _ in range(count):
        s = rng.uniform(0.5, 1.5)
        a = rng.uniform(0.05, 0.3) * peak
        cr, cc = rng.uniform(0.1 * n, 0.9 * n, size=2)
        out += a * np.exp(-((r - cr) ** 2 + (c - cc) ** 2) / (2.0 * s * s))
    return out


# ----------------------------------------------------------------------------
# uv coverage
# ----------------------------------------------------------------------------
def gaussian_uv(rng: np.random.Generator, M: int, sigma: float = math.pi / 4) -> np.ndarray:
    """Isotropic Gaussian density, each draw resampled until inside [-pi, pi)^2."""
    out = np.empty((0, 2))
    while out.shape[0] < M:
        d = rng.normal(0.0, sigma, size=(2 * (M - out.shape[0]) + 16, 2))
        ok = np.all((d >= -math.pi) & (d < math.pi), axis=1)
        out = np.concatenate([out, d[ok]], axis=0)
    return out[:M].copy()


def arc_uv(rng: np.random.Generator, M: int, stations: int = 8, max_omega: float = math.pi / 2) -> np.ndarray:
    """Earth-rotation synthesis arcs (Thompson, Moran & Swenson projection), 12 h track.

    Stations sit at random points of the unit sphere; the source declination is
    drawn in [20, 60] degrees.  Each baseline traces an ellipse as the hour
    angle sweeps [-6 h, 6 h]; the time sampling is chosen so that the total
    number of samples reaches M (then truncated to exactly M).  The coverage is
    scaled so that its largest |omega| component equals ``max_omega``.
    """
    pos = rng.standard_normal((stations, 3))
    pos /= np.linalg.norm(pos, axis=1, keepdims=True)
    dec = math.radians(rng.uniform(20.0, 60.0))
    pairs = [(a, b) for a in range(stations) for b in range(a + 1, stations)]
    nt = -(-M // len(pairs))
    H = np.linspace(-0.5 * math.pi, 0.5 * math.pi, nt)
    uu, vv = [], []
    for a, b in pairs:
        bx, by, bz = pos[a] - pos[b]
        u = bx * np.sin(H) + by * np.cos(H)
        v = -bx * math.sin(dec) * np.cos(H) + by * math.sin(dec) * np.sin(H) + bz * math.cos(dec)
        uu.append(u)
        vv.append(v)
    uv = np.stack([np.concatenate(vv), np.concatenate(uu)], axis=1)[:M]
    uv *= max_omega / np.max(np.abs(uv))
    return np.clip(uv, -math.pi, math.pi - 1e-12)


def unit_noise(rng: np.random.Generator, M: int) -> np.ndarray:
    """(M, 4) circular complex Gaussian with E|e|^2 = 1."""
    return (rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4))) / math.sqrt(2.0)


def station_mueller(rng: np.random.Generator, M: int, stations: int = 8, gain_spread: float = 0.1,
                    leakage: float = 0.05) -> np.ndarray:
    """(M, 4, 4) complex direction-independent Mueller matrices D_m = J_a kron conj(J_b) of the
    station pair (a, b) of each row (drawn uniformly, a != b), from per-station 2 x 2 Jones
    matrices J = [[g1, d1], [d2, g2]] with complex gains g ~ 1 + gain_spread CN(0, 1) and
    polarization leakage d ~ leakage CN(0, 1).  D_m acts on the brightness vector
    [I+Q, U+iV, U-iV, I-Q] of a row, taken as the row-major 2 x 2 coherency matrix."""
    def cn(size):
        return (rng.standard_normal(size) + 1j * rng.standard_normal(size)) / math.sqrt(2.0)
    J = np.empty((stations, 2, 2), dtype=np.complex128)
    J[:, 0, 0] = 1.0 + gain_spread * cn(stations)
    J[:, 1, 1] = 1.0 + gain_spread * cn(stations)
    J[:, 0, 1] = leakage * cn(stations)
    J[:, 1, 0] = leakage * cn(stations)
    a = rng.integers(0, stations, size=M)
    b = (a + rng.integers(1, stations, size=M)) % stations
    return np.einsum("mij,mkl->mikjl", J[a], np.conj(J[b])).reshape(M, 4, 4)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------
def blobs32(seed: int = BASE_SEED + 0) -> Workload:
    """32x32, 3 blobs, 600 Gaussian-density uv points, KB 6x6, 30 dB, 3 levels."""
    rng = np.random.default_rng(seed)
    n, M = 32, 600
    S = add_polarisation(rng, blobs_image(rng, n, 3))
    uv = gaussian_uv(rng, M)
    return Workload("blobs32", n, M, taps=6, oversample=2, levels=3, isnr_db=30.0,
                    iters=300, cycles=2, truth=S, uv=uv, noise=unit_noise(rng, M))


def ring128(seed: int = BASE_SEED + 1) -> Workload:
    """128x128 ring+jet, 8-station arcs with 12000 samples, KB 8x8, 20 dB, 4 levels."""
    rng = np.random.default_rng(seed)
    n, M = 128, 12000
    S = add_polarisation(rng, ring_jet_image(rng, n))
    uv = arc_uv(rng, M)
    return Workload("ring128", n, M, taps=8, oversample=2, levels=4, isnr_db=20.0,
                    iters=2000, cycles=5, truth=S, uv=uv, noise=unit_noise(rng, M))


def ring256(seed: int = BASE_SEED + 2) -> Workload:
    """256x256 ring+jet+20 knots, 1e5 Gaussian + 1e5 arc uv points, KB 8x8, 20 dB, 4 levels."""
    rng = np.random.default_rng(seed)
    n, M = 256, 200000
    S = add_polarisation(rng, add_knots(rng, ring_jet_image(rng, n), 20))
    uv = np.concatenate([gaussian_uv(rng, M // 2), arc_uv(rng, M - M // 2)], axis=0)
    return Workload("ring256", n, M, taps=8, oversample=2, levels=4, isnr_db=20.0,
                    iters=300, cycles=2, truth=S, uv=uv, noise=unit_noise(rng, M))


def batch_request(index: int, sides=(64, 128, 256), m_range=(3.0, 5.0),
                  isnr_range=(15.0, 35.0), big_side: int = 512, big_M: int = 1_000_000) -> Workload:
    """One request of the batched / served mixes (per-request seed 2417*1000 + index).

    Side uniform over ``sides``; M log-uniform over 10**m_range (side ``big_side``
    uses ``big_M``); input SNR uniform in ``isnr_range``; ground truth follows the
    ring+jet recipe (plus knots at 256 and above); uv mixes Gaussian and arcs.
    """
    rng = np.random.default_rng(BASE_SEED * 1000 + index)
    n = int(sides[rng.integers(0, len(sides))])
    M = big_M if n == big_side else int(round(10.0 ** rng.uniform(*m_range)))
    isnr = float(rng.uniform(*isnr_range))
    I = ring_jet_image(rng, n)
    if n >= 256:
        I = add_knots(rng, I, 20)
    S = add_polarisation(rng, I)
    half = M // 2
    uv = np.concatenate([gaussian_uv(rng, half), arc_uv(rng, M - half)], axis=0)
    return Workload(f"req{index}", n, M, taps=8, oversample=2, levels=4, isnr_db=isnr,
                    iters=300, cycles=2, truth=S, uv=uv, noise=unit_noise(rng, M))


def tiny(n: int = 16, M: int = 150, taps: int = 6, levels: int = 2, seed: int = 7,
         isnr_db: float = 30.0) -> Workload:
    """Small problem for convergence and parity tests (blob image, Gaussian uv)."""
    rng = np.random.default_rng(seed)
    S = add_polarisation(rng, blobs_image(rng, n, 2))
    uv = gaussian_uv(rng, M)
    return Workload(f"tiny{n}", n, M, taps=taps, oversample=2, levels=levels, isnr_db=isnr_db,
                    iters=300, cycles=2, truth=S, uv=uv, noise=unit_noise(rng, M))


def near_cone(n: int = 32, M: int = 1000, isnr_db: float = 35.0, seed: int = BASE_SEED + 12,
              stations: int = 6, blobs: int = 3) -> Workload:
    """Polarization close to the cone: Gaussian blobs with polarization fraction 0.97 at every
    pixel (chi smooth, V = 0.01 I), so sqrt(Q^2 + U^2 + V^2) sits 3 % below I, with sparse
    coverage (`stations`-station arcs out to 0.9 pi).  Estimates made without the polarization
    constraint leave the cone on a sizeable share of pixels.  KB 6 and 3 levels for n <= 32,
    KB 8 and 4 levels above."""
    rng = np.random.default_rng(seed)
    I = blobs_image(rng, n, blobs)
    chi = 0.5 * math.pi * (2.0 * smooth_field(rng, n) - 1.0)
    m = 0.97
    S = np.stack([I, m * I * np.cos(2.0 * chi), m * I * np.sin(2.0 * chi), 0.01 * I], axis=-1)
    uv = arc_uv(rng, M, stations=stations, max_omega=0.9 * math.pi)
    small = n <= 32
    return Workload(f"near_cone{n}", n, M, taps=6 if small else 8, oversample=2, levels=3 if small else 4,
                    isnr_db=isnr_db, iters=300, cycles=2, truth=S, uv=uv, noise=unit_noise(rng, M))


def np_study() -> Workload:
    """The polarization-error study: the near-cone workload (32x32 blobs, fraction 0.97, 6-station
    arcs with 1000 rows, 35 dB) on the 300-iteration schedule of the blob workload
    (initialisation + 2 reweighting cycles)."""
    wl = near_cone()
    wl.name = "np_study"
    return wl


WORKLOADS = {"blobs32": blobs32, "ring128": ring128, "ring256": ring256}


def poisson_arrivals(count: int, rate: float, seed: int = BASE_SEED * 1000 + 999) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: cumulative exponential gaps of mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
