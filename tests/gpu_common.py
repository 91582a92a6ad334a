"""Shared set-up for the GPU parity tests: seeded problems built by the oracle, and the
same inputs handed to the HIP library through its C ABI."""
from __future__ import annotations

import math
import sys

import numpy as np

from oracle import problem as oproblem
from oracle.nufft import NUFFT, MeasurementOp
from oracle.sara import SARA, BASES
from paper_1801_02417_amd import psara as P
from paper_1801_02417_amd import workloads as wk

PREC = {"fp64": P.PSARA_FP64, "fp32": P.PSARA_FP32_MIXED}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def random_uv(rng, M, spread=math.pi / 3):
    uv = rng.normal(0, spread, size=(M, 2))
    return np.clip(uv, -math.pi, math.pi - 1e-9)


def mask_of(bases) -> int:
    m = 0
    for b in bases:
        m |= 1 << (0 if b == "dirac" else int(b[2:]))
    return m


def solver_for(wl_or_uv, n, taps, prec, levels=None, bases=BASES, gamma=1.0, weights=None):
    uv = wl_or_uv.uv if hasattr(wl_or_uv, "uv") else wl_or_uv
    s = P.Solver(n, uv, taps=taps, precision=PREC[prec])
    if levels is not None:
        s.set_prior(levels, gamma, mask_of(bases), weights)
    return s
