"""Pins of the oracle's Algorithm 3 (the TV-based problems eq. Akiyama and eq. Akiyama_2)."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import pd, tv
from oracle.nufft import NUFFT, MeasurementOp
from paper_1801_02417_amd import workloads as wk


def test_difference_operators_adjoint_and_norm():
    """d1, d2 and their adjoints are exact transposes, and ||grad||^2 has the closed form of
    the Neumann difference operator, 8 sin^2(pi (n - 1) / (2n)) (the largest eigenvalue of the
    1-D second difference with the zero-difference boundary is 4 sin^2(pi (n - 1) / (2n)))."""
    rng = np.random.default_rng(1)
    for n in (3, 8, 16):
        U = rng.standard_normal((n * n, 4))
        G = rng.standard_normal((n * n, 4))
        assert abs(np.sum(tv.d1(U, n) * G) - np.sum(U * tv.d1_adj(G, n))) < 1e-12 * np.sum(np.abs(U))
        assert abs(np.sum(tv.d2(U, n) * G) - np.sum(U * tv.d2_adj(G, n))) < 1e-12 * np.sum(np.abs(U))
        A = tv.psi_adj(U, n, "l1tv")
        assert abs(np.sum(A * np.concatenate([G, G, G])) - np.sum(U * tv.psi(np.concatenate([G, G, G]), n, "l1tv"))) \
            < 1e-11 * np.sum(np.abs(U))
        # power iteration on grad^T grad for one map
        x = rng.standard_normal((n * n, 1))
        for _ in range(3000):
            x = tv.d1_adj(tv.d1(x, n), n) + tv.d2_adj(tv.d2(x, n), n)
            x /= np.linalg.norm(x)
        lam = float(np.sum(x * (tv.d1_adj(tv.d1(x, n), n) + tv.d2_adj(tv.d2(x, n), n))))
        assert abs(lam - 8 * math.sin(math.pi * (n - 1) / (2 * n)) ** 2) < 1e-6
    # the difference at the last row / column is zero, the others are plain differences
    U = np.arange(9.0).reshape(9, 1)
    assert np.array_equal(tv.d1(U, 3).ravel(), [3, 3, 3, 3, 3, 3, 0, 0, 0])
    assert np.array_equal(tv.d2(U, 3).ravel(), [1, 1, 0, 1, 1, 0, 1, 1, 0])


def test_group_soft_threshold():
    """The l2,1 proximity operator: pairs of norm at most t vanish, others shrink by t along
    themselves; it matches a numerical minimisation, and the dual step it induces is the
    projection of each pair on the ball of radius t (Moreau)."""
    a, b = tv.group_soft_threshold(np.array([3.0, 0.3, 0.0]), np.array([4.0, 0.4, 0.0]), np.array([1.0, 1.0, 1.0]))
    assert np.allclose(a, [2.4, 0, 0]) and np.allclose(b, [3.2, 0, 0])
    rng = np.random.default_rng(2)
    for _ in range(5):
        v = rng.standard_normal(2) * 2
        t = rng.uniform(0.1, 2.0)
        r = minimize(lambda x: t * np.linalg.norm(x) + 0.5 * np.sum((x - v) ** 2), v, method="Nelder-Mead",
                     options={"xatol": 1e-10, "fatol": 1e-14, "maxiter": 20000})
        p1, p2 = tv.group_soft_threshold(v[:1], v[1:], np.array([t]))
        assert np.allclose([p1[0], p2[0]], r.x, atol=1e-6)
        rho = rng.uniform(0.1, 2.0)
        At = v * 3
        T1, T2 = tv.group_soft_threshold(At[:1] / rho, At[1:] / rho, np.array([t / rho]))
        dual = At - rho * np.array([T1[0], T2[0]])
        proj = At * min(1.0, t / np.linalg.norm(At))
        assert np.allclose(dual, proj, atol=1e-12)


def _brute_force_problem(constrained: bool, kind: str):
    rng = np.random.default_rng(5)
    n, N, M = 4, 16, 24
    uv = np.clip(rng.normal(0, 1.0, size=(M, 2)), -math.pi, math.pi - 1e-9)
    nu = NUFFT(uv, n, 2, 6)
    mop = MeasurementOp(nu)
    I = rng.uniform(0.2, 1, size=N)
    chi = rng.uniform(0, np.pi, N)
    S = np.stack([I, 0.9 * I * np.cos(2 * chi), 0.9 * I * np.sin(2 * chi), 0.05 * I], 1)
    y0 = mop.phi(S)
    Y = y0 + 0.05 * np.linalg.norm(y0) / math.sqrt(4 * M) * (rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4)))
    beta, _ = pd.phi_norm_sq(mop, N, rtol=1e-12)
    pb = tv.build(nu, Y, n, kind, [0.05, 0.03, 0.03, 0.02], [0.02, 0.01, 0.01, 0.01] if kind == "l1tv" else None,
                  beta / 2.0)
    return pb, n, N


@pytest.mark.parametrize("constrained", [False, True])
@pytest.mark.parametrize("kind", ["tv", "l1tv"])
def test_alg3_matches_brute_force_on_4x4(constrained, kind):
    """4x4 Stokes images, 24 rows: a general-purpose solver on the explicit problem, with the
    norms smoothed by delta = 1e-9 (sqrt(x^2 + delta^2), moving the objective by < 1e-7):
    L-BFGS-B with I >= 0 without the constraint, SLSQP with the polarization cone with it,
    started from zero, reaches the objective Algorithm 3 converges to."""
    pb, n, N = _brute_force_problem(constrained, kind)
    delta = 1e-9
    D1 = tv.d1(np.eye(N), n)
    D2 = tv.d2(np.eye(N), n)

    def f(z):
        S = z.reshape(N, 4)
        r = pb.phit(S) - pb.Yt
        g1, g2 = D1 @ S, D2 @ S
        q = np.sqrt(g1 ** 2 + g2 ** 2 + delta ** 2)
        val = 0.5 * np.sum(np.abs(r) ** 2) + np.sum(q * pb.tv_weight)
        grad = np.real(pb.phit_adj(r)) + D1.T @ (g1 / q * pb.tv_weight) + D2.T @ (g2 / q * pb.tv_weight)
        if kind == "l1tv":
            a = np.sqrt(S ** 2 + delta ** 2)
            val += np.sum(a * pb.l1_weight)
            grad = grad + S / a * pb.l1_weight
        return val, grad.ravel()

    z0 = np.zeros(4 * N)
    if constrained:
        def cone(z):
            S = z.reshape(N, 4)
            return np.concatenate([S[:, 0] ** 2 - np.sum(S[:, 1:] ** 2, 1), S[:, 0]])

        def cone_jac(z):
            S = z.reshape(N, 4)
            J = np.zeros((2 * N, 4 * N))
            for p in range(N):
                J[p, 4 * p] = 2 * S[p, 0]
                J[p, 4 * p + 1:4 * p + 4] = -2 * S[p, 1:]
                J[N + p, 4 * p] = 1.0
            return J
        z0[0::4] = 0.1
        r = minimize(lambda z: f(z)[0], z0, jac=lambda z: f(z)[1], method="SLSQP",
                     constraints=[{"type": "ineq", "fun": cone, "jac": cone_jac}],
                     options={"maxiter": 3000, "ftol": 1e-15})
    else:
        bounds = [(0, None) if k % 4 == 0 else (None, None) for k in range(4 * N)]
        r = minimize(f, z0, jac=True, method="L-BFGS-B", bounds=bounds,
                     options={"maxiter": 20000, "ftol": 1e-16, "gtol": 1e-12})
    brute = tv.objective(pb, r.x.reshape(N, 4))
    st = tv.run_alg3(tv.zeros(n, pb.Yt.shape[0], kind), pb, 5000, constrained)
    got = tv.objective(pb, st.S)
    assert abs(got - brute) <= 1e-6 * brute, (got, brute)
    if constrained:
        assert np.all(st.S[:, 0] >= np.linalg.norm(st.S[:, 1:], axis=1) - 1e-9)
    else:
        assert np.all(st.S[:, 0] >= 0)
