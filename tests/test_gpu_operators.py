"""GPU parity of the measurement operator phi / phi^dagger and the SARA frame Psi / Psi^dagger
(HIP kernels through the C ABI) against the FP64 oracle on identical seeded inputs."""
import math

import numpy as np
import pytest

from oracle.nufft import NUFFT, MeasurementOp
from oracle.sara import SARA, BASES
from oracle.pd import phi_norm_sq
from paper_1801_02417_amd import workloads as wk
from tests.gpu_common import P, say, rel_err, random_uv, solver_for, mask_of

pytestmark = pytest.mark.gpu

# (n, M, taps, levels): tiny, config-0-like, coarse levels of size 1, T = 8 at 64 and 128
CASES = [(16, 150, 6, 2), (32, 600, 6, 3), (8, 40, 4, 3), (64, 3000, 8, 4), (128, 12000, 8, 4)]
TOL = {"fp64": 1e-11, "fp32": 3e-6}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_M%d_T%d" % (c[0], c[1], c[2]))
def test_phi_and_adjoint(case, prec):
    n, M, T, L = case
    say(f"[phi] n={n} M={M} T={T} prec={prec}")
    rng = np.random.default_rng(n * 7 + T)
    uv = random_uv(rng, M)
    mop = MeasurementOp(NUFFT(uv, n, 2, T))
    S = rng.standard_normal((n * n, 4))
    B = rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4))
    s = solver_for(uv, n, T, prec)
    try:
        y = s.phi(S)
        x = s.phi_adjoint(B)
    finally:
        s.close()
    e1 = rel_err(y, mop.phi(S))
    e2 = rel_err(x, np.real(mop.phi_adj(B)))
    say(f"   phi rel err {e1:.2e}  adjoint rel err {e2:.2e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_identity_on_device(prec):
    n, M, T = 32, 500, 8
    rng = np.random.default_rng(99)
    uv = random_uv(rng, M)
    s = solver_for(uv, n, T, prec)
    try:
        X = rng.standard_normal((n * n, 4))
        Y = rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4))
        lhs = np.real(np.vdot(s.phi(X), Y))
        rhs = np.sum(X * s.phi_adjoint(Y))
    finally:
        s.close()
    assert abs(lhs - rhs) <= (1e-12 if prec == "fp64" else 2e-6) * abs(lhs)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", [(16, 2, BASES), (32, 3, BASES), (8, 3, BASES), (64, 4, BASES),
                                  (256, 4, BASES), (32, 2, ("dirac",)), (32, 1, ("db1", "db8")),
                                  (16, 4, ("db3", "db8"))],
                         ids=lambda c: "n%d_L%d_%s" % (c[0], c[1], "-".join(c[2]) if len(c[2]) < 9 else "sara"))
def test_psi_and_adjoint(case, prec):
    n, L, bases = case
    say(f"[psi] n={n} L={L} bases={bases} prec={prec}")
    rng = np.random.default_rng(n + L)
    sara = SARA(n, L, bases)
    S = rng.standard_normal((n * n, 4))
    A = rng.standard_normal((sara.J, 4))
    s = solver_for(random_uv(rng, 10), n, 6, prec, levels=L, bases=bases)
    try:
        a = s.psi_adjoint(S)
        x = s.psi(A)
        rt = s.psi(a)
    finally:
        s.close()
    tol = {"fp64": 1e-12, "fp32": 2e-6}[prec]
    ea, ex = rel_err(a, sara.adjoint(S)), rel_err(x, sara.forward(A))
    say(f"   analysis {ea:.2e} synthesis {ex:.2e} roundtrip {rel_err(rt, S):.2e}")
    assert ea <= tol and ex <= tol
    assert rel_err(rt, S) <= tol            # Psi Psi^dagger = I on the device


def test_wavelet_filters_match_oracle():
    from oracle.sara import daubechies_lowpass
    for p in range(1, 9):
        assert np.max(np.abs(P.psara_wavelet_filter(p) - daubechies_lowpass(p))) < 1e-14


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_power_iteration(prec):
    n, M, T = 32, 600, 6
    rng = np.random.default_rng(5)
    uv = random_uv(rng, M)
    mop = MeasurementOp(NUFFT(uv, n, 2, T))
    ref, _ = phi_norm_sq(mop, n * n, max_iter=3000, rtol=1e-13)
    s = solver_for(uv, n, T, prec)
    try:
        got = s.opnorm(3000, 1e-13)
    finally:
        s.close()
    say(f"[opnorm] {prec} gpu {got:.12e} oracle {ref:.12e}")
    assert abs(got - ref) <= 1e-8 * ref      # FP64 on the device in both precisions


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_phi_with_mueller_matrices(prec):
    """Known direction-independent Mueller matrices per row (psara_set_mueller): phi and its
    adjoint against the oracle's operator with the same matrices, the adjoint identity on the
    device, and psara_set_mueller(None) restoring the plain operator bit for bit."""
    n, M, T = 32, 700, 8
    rng = np.random.default_rng(71)
    uv = random_uv(rng, M)
    D = wk.station_mueller(rng, M, leakage=0.2)
    mop = MeasurementOp(NUFFT(uv, n, 2, T), D)
    S = rng.standard_normal((n * n, 4))
    B = rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4))
    s = solver_for(uv, n, T, prec)
    try:
        y_plain = s.phi(S)
        s.set_mueller(D)
        y = s.phi(S)
        x = s.phi_adjoint(B)
        lhs = np.real(np.vdot(y, B))
        rhs = float(np.sum(S * x))
        s.set_mueller(None)
        assert np.array_equal(s.phi(S), y_plain)
    finally:
        s.close()
    e1 = rel_err(y, mop.phi(S))
    e2 = rel_err(x, np.real(mop.phi_adj(B)))
    say(f"[mueller] {prec}: phi rel err {e1:.2e}, adjoint rel err {e2:.2e}, <phi S, B> - <S, phi^t B> "
        f"{abs(lhs - rhs) / abs(lhs):.2e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec]
    assert abs(lhs - rhs) <= 10 * TOL[prec] * abs(lhs)
