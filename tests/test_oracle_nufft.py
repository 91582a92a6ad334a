"""Pins of the oracle's measurement operator (Sec. 4.1 eq. meas_op, Sec. 2.1 L)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle.kb import kb_beta, kb_psi, kb_psi_hat
from oracle.nufft import NUFFT, MeasurementOp, direct_dft, L_MIX
from oracle.pd import phi_norm_sq, power_iteration
from paper_1801_02417_amd import workloads as wk


def _rand_uv(rng, M, spread=math.pi / 3):
    return np.clip(rng.normal(0, spread, size=(M, 2)), -math.pi, math.pi - 1e-9)


@pytest.mark.parametrize("taps", [6, 8])
def test_kb_fourier_transform_matches_quadrature(taps):
    beta = kb_beta(taps, 2.0)
    for nu in (0.0, 0.05, 0.13, 0.25):
        q = quad(lambda x: float(kb_psi(x, taps, beta)) * math.cos(2 * math.pi * nu * x),
                 -taps / 2, taps / 2, epsabs=1e-13, epsrel=1e-13, limit=400)[0]
        assert abs(q - float(kb_psi_hat(nu, taps, beta))) <= 1e-12 * abs(q)


def test_kb_shape_parameter_values():
    # Beatty et al. (2005) beta for alpha = 2 (Sec. 4.1 leaves the kernel open)
    assert abs(kb_beta(6, 2.0) - 13.8551003) < 1e-6
    assert abs(kb_beta(8, 2.0) - 18.6389397) < 1e-6
    assert float(kb_psi(0.0, 8, kb_beta(8, 2.0))) == 1.0
    assert float(kb_psi(4.0001, 8, kb_beta(8, 2.0))) == 0.0


@pytest.mark.parametrize("n,taps", [(8, 6), (16, 8), (32, 6)])
def test_adjoint_identity(n, taps):
    """<Phi x, y> = <x, Phi^dagger y> for complex x, y."""
    rng = np.random.default_rng(n + taps)
    nu = NUFFT(_rand_uv(rng, 77), n, 2, taps)
    x = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    y = rng.standard_normal(77) + 1j * rng.standard_normal(77)
    lhs = np.vdot(nu.forward(x), y)
    rhs = np.vdot(x, nu.adjoint(y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_identity_full_phi_real_inner_product():
    """<phi(X), Y>_R = <X, Re phi^dagger Y> for real X (the map Algorithm 1 uses)."""
    rng = np.random.default_rng(3)
    n, M = 16, 90
    mop = MeasurementOp(NUFFT(_rand_uv(rng, M), n, 2, 8))
    X = rng.standard_normal((n * n, 4))
    Y = rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4))
    lhs = np.real(np.vdot(mop.phi(X), Y))
    rhs = np.sum(X * np.real(mop.phi_adj(Y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_brightness_mixing():
    """S^T L = [I+Q, U+iV, U-iV, I-Q] (Sec. 2.1) and L L^H = 2 I."""
    s = np.array([1.5, -0.25, 0.75, 0.125])
    b = s @ L_MIX
    assert np.allclose(b, [1.25, 0.75 + 0.125j, 0.75 - 0.125j, 1.75], atol=0, rtol=0)
    assert np.array_equal(L_MIX @ L_MIX.conj().T, 2 * np.eye(4))


def test_phi_adj_phi_is_twice_Phi_adj_Phi():
    rng = np.random.default_rng(4)
    n, M = 8, 40
    nu = NUFFT(_rand_uv(rng, M), n, 2, 6)
    mop = MeasurementOp(nu)
    X = rng.standard_normal((n * n, 4))
    lhs = mop.phi_adj(mop.phi(X))
    rhs = 2 * nu.adjoint(nu.forward(X.astype(complex)))
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))


@pytest.mark.parametrize("n", [8, 16])
def test_nufft_matches_direct_dft_and_improves_with_taps(n):
    """NUFFT vs the direct transform on tiny grids."""
    rng = np.random.default_rng(10 + n)
    uv = rng.uniform(-math.pi, math.pi, size=(50, 2))
    x = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    ref = direct_dft(x, uv, n)
    errs = {}
    for taps in (4, 6, 8):
        y = NUFFT(uv, n, 2, taps).forward(x)
        errs[taps] = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    # measured: T=6 5.2e-6 / 5.5e-6, T=8 6.4e-8 / 4.9e-8 relative; bound at twice the measurement
    assert errs[6] < 1.1e-5
    assert errs[8] < 1.3e-7
    assert errs[8] < errs[6] < errs[4]


def test_nearest_kernel_on_grid_is_centred_fft2():
    """alpha = 1, T = 1, omega on the grid: Phi x = fft2 of the centred image (sign, centring, wrap)."""
    rng = np.random.default_rng(21)
    n = 8
    k = rng.integers(-n // 2, n // 2, size=(30, 2))
    uv = 2 * math.pi * k / n
    nu = NUFFT(uv, n, 1, 1, kernel="nearest")
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    ref = np.fft.fft2(np.fft.ifftshift(x))[k[:, 0] % n, k[:, 1] % n]
    assert np.max(np.abs(nu.forward(x.ravel()) - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(direct_dft(x, uv, n) - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_window_wraps_across_grid_edge():
    """A frequency near 0 puts taps on both ends of the grid (index wrap mod K); the weights
    equal those of the same fractional offset shifted into the interior."""
    n = 16
    K = 2 * n
    shift = 2 * math.pi * 8 / K
    uv = np.array([[0.01, 0.3], [0.01 + shift, 0.3]])
    nu = NUFFT(uv, n, 2, 8)
    rows0 = set(int(c) // K for c in nu.G[0].indices)
    assert 0 in rows0 and K - 1 in rows0
    assert nu.G[0].nnz == 64 and nu.G[1].nnz == 64
    assert np.allclose(np.sort(nu.G[0].data), np.sort(nu.G[1].data), rtol=1e-12, atol=0)


def test_power_iteration_matches_explicit_matrix_norm():
    """||phi||^2 of X -> Re phi^dagger phi X equals the squared spectral norm of the explicit real matrix."""
    rng = np.random.default_rng(8)
    n, M = 8, 30
    mop = MeasurementOp(NUFFT(_rand_uv(rng, M), n, 2, 6))
    N = n * n
    # explicit real matrix of X -> [Re phi(X); Im phi(X)] on the N x 4 real space
    cols = []
    for j in range(N * 4):
        e = np.zeros(N * 4)
        e[j] = 1.0
        y = mop.phi(e.reshape(N, 4)).ravel()
        cols.append(np.concatenate([y.real, y.imag]))
    Mat = np.array(cols).T
    ref = np.linalg.norm(Mat, 2) ** 2
    lam, its = phi_norm_sq(mop, N, rtol=1e-13, max_iter=5000)
    assert abs(lam - ref) <= 1e-9 * ref


def test_power_iteration_generic():
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((6, 6)))
    A = Q @ np.diag([5.0, 3.0, 1.0, 0.5, 0.1, 0.0]) @ Q.T
    lam, _ = power_iteration(lambda x: A @ x, np.ones(6), 10000, 1e-15)
    assert abs(lam - 5.0) < 1e-12


def test_workload_uv_inside_band_and_truth_in_cone():
    for wl in (wk.blobs32(), wk.tiny()):
        assert np.all(wl.uv >= -math.pi) and np.all(wl.uv < math.pi)
        S = wl.truth
        assert np.all(np.linalg.norm(S[..., 1:], axis=-1) <= S[..., 0] + 1e-15)
        assert abs(np.mean(np.abs(wl.noise) ** 2) - 1.0) < 0.1


def test_mueller_operator_pins():
    """Measurement operator with known direction-independent Mueller matrices D_m (eq. RIME
    with D constant over the sky): identity matrices give the plain operator; the column form
    y_m = D_m (L^T v_m) of the equation, written out row by row, equals the operator; the
    adjoint is exact; Mueller matrices built from unitary Jones matrices preserve norms."""
    wl = wk.tiny(n=16, M=120, taps=6, levels=2, seed=21)
    rng = np.random.default_rng(4)
    nu = NUFFT(wl.uv, wl.n, 2, 6)
    plain = MeasurementOp(nu)
    eye = MeasurementOp(nu, np.broadcast_to(np.eye(4, dtype=np.complex128), (wl.M, 4, 4)))
    S = rng.standard_normal((wl.n * wl.n, 4))
    B = rng.standard_normal((wl.M, 4)) + 1j * rng.standard_normal((wl.M, 4))
    assert np.allclose(eye.phi(S), plain.phi(S), rtol=0, atol=1e-13 * np.abs(plain.phi(S)).max())
    assert np.allclose(eye.phi_adj(B), plain.phi_adj(B), rtol=0, atol=1e-13 * np.abs(plain.phi_adj(B)).max())
    D = wk.station_mueller(rng, wl.M, leakage=0.2)
    op = MeasurementOp(nu, D)
    V = nu.forward(S.astype(np.complex128))
    L = np.array([[1, 0, 0, 1], [1, 0, 0, -1], [0, 1, 1, 0], [0, 1j, -1j, 0]])
    rows = np.stack([D[m] @ (L.T @ V[m]) for m in range(wl.M)])
    assert np.allclose(op.phi(S), rows, rtol=0, atol=1e-12 * np.abs(rows).max())
    lhs = np.real(np.vdot(op.phi(S), B))
    rhs = float(np.sum(S * np.real(op.phi_adj(B))))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # unitary Jones matrices: D_m = J_a kron conj(J_b) is unitary, so each row keeps its norm
    q = np.linalg.qr(rng.standard_normal((8, 2, 2)) + 1j * rng.standard_normal((8, 2, 2)))[0]
    a, b = rng.integers(0, 8, wl.M), rng.integers(0, 8, wl.M)
    Du = np.einsum("mij,mkl->mikjl", q[a], np.conj(q[b])).reshape(wl.M, 4, 4)
    yu, y0 = MeasurementOp(nu, Du).phi(S), plain.phi(S)
    assert np.allclose(np.linalg.norm(yu, axis=1), np.linalg.norm(y0, axis=1), rtol=1e-12, atol=0)
