"""Pins of the oracle's projections and thresholding (Sec. 3.3)."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

from oracle.prox import (proj_U, proj_U_prime, proj_V, soft_threshold, proj_ball, proj_E1, proj_E2,
                         proj_polarization_cone)

RNG = np.random.default_rng(1234)


def _pts(k, dim, scale=2.0):
    return RNG.standard_normal((k, dim)) * scale


def test_idempotence_and_fixed_points():
    X = _pts(500, 4)
    for P in (proj_polarization_cone,):
        Y = P(X)
        assert np.max(np.abs(P(Y) - Y)) < 1e-15
    U = _pts(500, 2)
    V = proj_V(U)
    assert np.array_equal(proj_V(V), V)
    c, d = proj_E1(U[:, 0], U[:, 1])
    c2, d2 = proj_E1(c, d)
    assert np.max(np.abs(c2 - c)) == 0 and np.max(np.abs(d2 - d)) == 0
    R, dd = proj_E2(X[:, 1:], X[:, 0])
    R2, dd2 = proj_E2(R, dd)
    assert np.max(np.abs(R2 - R)) < 1e-15 and np.max(np.abs(dd2 - dd)) < 1e-15


def test_points_inside_are_unchanged():
    U = _pts(300, 2)
    inside = U[U[:, 0] + U[:, 1] <= 0]
    assert np.array_equal(proj_V(inside), inside)
    c, d = U[:, 0], U[:, 1]
    keep = c + d >= 0
    cc, dd = proj_E1(c[keep], d[keep])
    assert np.array_equal(cc, c[keep]) and np.array_equal(dd, d[keep])
    X = _pts(300, 4)
    inn = X[np.linalg.norm(X[:, 1:], axis=1) <= X[:, 0]]
    assert len(inn) > 10
    assert np.array_equal(proj_polarization_cone(inn), inn)


def test_lorentz_cone_moreau_decomposition():
    """Self-dual cone K: x = P_K(x) - P_K(-x) and <P_K(x), P_K(-x)> = 0."""
    X = _pts(1000, 4)
    P = proj_polarization_cone(X)
    Q = proj_polarization_cone(-X)
    assert np.max(np.abs(X - (P - Q))) < 1e-14
    assert np.max(np.abs(np.sum(P * Q, axis=1))) < 1e-13


def test_e2_boundary_readings():
    R, d = proj_E2(np.zeros((1, 3)), np.zeros(1))            # r = 0, d = 0 -> 0 (no division)
    assert np.array_equal(R, np.zeros((1, 3))) and d[0] == 0
    R, d = proj_E2(np.array([[3.0, 4.0, 0.0]]), np.array([5.0]))   # on the cone: kept
    assert np.array_equal(R, [[3.0, 4.0, 0.0]]) and d[0] == 5.0
    R, d = proj_E2(np.array([[3.0, 4.0, 0.0]]), np.array([-5.0]))  # on the polar cone: 0
    assert np.array_equal(R, np.zeros((1, 3))) and d[0] == 0.0
    R, d = proj_E2(np.array([[3.0, 4.0, 0.0]]), np.array([1.0]))   # alpha = (1 + 1/5)/2 = 0.6
    assert np.allclose(R, [[1.8, 2.4, 0.0]], rtol=1e-15) and abs(d[0] - 3.0) < 1e-15


def _brute_from(x, x0, cons):
    r = minimize(lambda u: np.sum((u - x) ** 2), x0, jac=lambda u: 2 * (u - x), constraints=cons,
                 method="SLSQP", options={"ftol": 1e-16, "maxiter": 500})
    return r.x


def _brute(x, cons):
    return _brute_from(x, x, cons)


@pytest.mark.parametrize("which", ["V", "E1", "E2"])
def test_projections_are_distance_minimisers(which):
    """Brute-force SLSQP minimisation of ||u - x||^2 over each set, 300 random points."""
    pts = _pts(300, 4 if which == "E2" else 2)
    worst = 0.0
    for x in pts:
        if which == "V":
            want = proj_V(x[None])[0]
            cons = [{"type": "ineq", "fun": lambda u: -(u[0] + u[1]), "jac": lambda u: np.array([-1.0, -1.0])}]
        elif which == "E1":
            c, d = proj_E1(x[:1], x[1:])
            want = np.array([c[0], d[0]])
            cons = [{"type": "ineq", "fun": lambda u: u[0] + u[1], "jac": lambda u: np.array([1.0, 1.0])}]
        else:
            if np.linalg.norm(x[:3]) <= -x[3]:
                continue          # polar-cone points map to 0: checked by the Moreau test
            R, d = proj_E2(x[None, :3], x[3:])
            want = np.concatenate([R[0], d])
            cons = [{"type": "ineq", "fun": lambda u: u[3] - np.linalg.norm(u[:3]),
                     "jac": lambda u: np.concatenate([-u[:3] / max(np.linalg.norm(u[:3]), 1e-300), [1.0]])}]
            x0 = np.array([0.0, 0.0, 0.0, np.linalg.norm(x) + 1.0])
            got = _brute_from(x, x0, cons)
            worst = max(worst, np.max(np.abs(got - want)))
            continue
        got = _brute(x, cons)
        worst = max(worst, np.max(np.abs(got - want)))
    assert worst < 1e-7


def test_soft_threshold_is_prox_of_weighted_l1():
    for a, t in [(2.5, 1.0), (-2.5, 1.0), (0.3, 1.0), (-0.3, 0.5), (0.0, 0.2)]:
        ref = minimize_scalar(lambda u: t * abs(u) + 0.5 * (u - a) ** 2, bounds=(-10, 10),
                              method="bounded", options={"xatol": 1e-12}).x
        # a 1-D minimiser search resolves the argmin to about sqrt(machine eps)
        assert abs(soft_threshold(np.array(a), np.array(t)) - ref) < 1e-7


def test_dual_sparsity_update_is_clip():
    """A - rho1 T_{gW/rho1}(A/rho1) = clip(A, -gW, gW) (Moreau identity)."""
    A = _pts(2000, 4, 3.0)
    gW = np.abs(_pts(2000, 4, 1.0))
    for rho1 in (1.0, 0.37, 5.0):
        upd = A - rho1 * soft_threshold(A / rho1, gW / rho1)
        assert np.max(np.abs(upd - np.clip(A, -gW, gW))) < 1e-15 * 8


def test_ball_projection():
    rng = np.random.default_rng(9)
    Y = rng.standard_normal((20, 4)) + 1j * rng.standard_normal((20, 4))
    X = Y + 3.0 * (rng.standard_normal((20, 4)) + 1j * rng.standard_normal((20, 4)))
    P = proj_ball(X, Y, 2.0)
    assert abs(np.linalg.norm(P - Y) - 2.0) < 1e-14
    d1 = (X - Y) / np.linalg.norm(X - Y)
    d2 = (P - Y) / np.linalg.norm(P - Y)
    assert np.max(np.abs(d1 - d2)) < 1e-15
    inside = Y + 0.01 * (X - Y)
    assert np.array_equal(proj_ball(inside, Y, 2.0), inside)


def test_real_and_positive_sets():
    X = _pts(50, 4) + 1j * _pts(50, 4)
    assert np.array_equal(proj_U(X), X.real)
    P = proj_U_prime(X)
    assert np.array_equal(P[:, 1:], X.real[:, 1:])
    assert np.array_equal(P[:, 0], np.maximum(X.real[:, 0], 0))
