"""Edge cases of the measurement operator and the iteration on the device against the oracle:
a single visibility row at the corner of the band (its window wraps across both grid edges),
many rows at one uv point (runs split at their maximum length, one gridding tile split into
several chunks whose partial slots the column inverse FFT sums), and inputs the boundary must
reject (no rows, rows outside the band, a side that is not a power of two)."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import pd, problem
from oracle.nufft import NUFFT, MeasurementOp
from paper_1801_02417_amd import workloads as wk
from tests.gpu_common import P, say, rel_err, random_uv, solver_for
from tests.test_gpu_iteration import _compare, _oracle_steps, _random_state

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 3e-6}


def _phi_parity(uv, n, T, prec, seed):
    rng = np.random.default_rng(seed)
    M = uv.shape[0]
    mop = MeasurementOp(NUFFT(uv, n, 2, T))
    S = rng.standard_normal((n * n, 4))
    B = rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4))
    s = solver_for(uv, n, T, prec)
    try:
        y = s.phi(S)
        x = s.phi_adjoint(B)
    finally:
        s.close()
    return rel_err(y, mop.phi(S)), rel_err(x, np.real(mop.phi_adj(B)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("corner", [(-math.pi, -math.pi), (math.pi - 1e-9, -math.pi), (math.pi - 1e-9, math.pi - 1e-9)],
                         ids=["low-low", "high-low", "high-high"])
def test_single_row_at_band_corner(corner, prec):
    uv = np.array([corner], dtype=np.float64)
    e1, e2 = _phi_parity(uv, 16, 8, prec, seed=3)
    say(f"[edge] one row at {corner} {prec}: phi {e1:.2e} adjoint {e2:.2e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


def _clustered_uv(rng, M_same, M_rest):
    """M_same rows at one uv point, the rest spread over the band."""
    same = np.tile(np.array([[0.3, -0.7]]), (M_same, 1))
    return np.concatenate([same, random_uv(rng, M_rest)], axis=0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_many_rows_at_one_point(prec):
    uv = _clustered_uv(np.random.default_rng(5), 2600, 400)
    e1, e2 = _phi_parity(uv, 32, 8, prec, seed=6)
    say(f"[edge] 2600 rows at one point {prec}: phi {e1:.2e} adjoint {e2:.2e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
def test_iterations_with_many_rows_at_one_point(prec, tol):
    """Initialisation-stage iterations (which run the fused de-grid + grid pass) and constrained
    ones (separate passes) on the clustered coverage, from a random state."""
    n, T, L = 32, 8, 2
    base = wk.tiny(n=n, M=3000, taps=T, levels=L, seed=41)
    wl = dataclasses.replace(base, uv=_clustered_uv(np.random.default_rng(7), 2600, 400))
    b = problem.build(wl, norm_rtol=1e-8, norm_max_iter=300)
    rng = np.random.default_rng(8)
    W = rng.uniform(0.2, 1.0, size=(b.sara.J, 4))
    gW = b.gamma * W
    s = solver_for(wl, n, T, prec, levels=L, gamma=b.gamma, weights=W)
    try:
        s.set_data(b.pb.Y, b.pb.eps)
        s.opnorm(200, 1e-8)
        s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
        for mode in ("init", "polsara"):
            st = _random_state(rng, n * n, b.sara.J, wl.M, gW)
            if mode == "init":
                st.Z[:] = 0; st.A[:] = 0; st.C[:] = 0; st.D[:] = 0
            s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
            scale = {}
            ref = _oracle_steps(st.copy(), b.pb, gW, mode, 3, scale)
            s.solve(P.PSARA_NNLS_INIT if mode == "init" else P.PSARA_CONSTRAINED, 3, report=False)
            w = _compare(s.state(), ref, tol, f"clustered {mode}", scale if prec == "fp32" else None)
            say(f"[edge] clustered coverage, {mode}, {prec}: worst rel err {w:.2e}")
    finally:
        s.close()


def test_boundary_rejects_bad_inputs():
    with pytest.raises(P.PsaraError):
        P.Solver(16, np.zeros((0, 2)), taps=8, precision=P.PSARA_FP32_MIXED)
    with pytest.raises(P.PsaraError):
        P.Solver(16, np.array([[math.pi, 0.0]]), taps=8, precision=P.PSARA_FP32_MIXED)
    with pytest.raises(P.PsaraError):
        P.Solver(24, np.array([[0.1, 0.2]]), taps=8, precision=P.PSARA_FP32_MIXED)
    with pytest.raises(P.PsaraError):
        P.Solver(16, np.array([[0.1, float("nan")]]), taps=8, precision=P.PSARA_FP32_MIXED)
