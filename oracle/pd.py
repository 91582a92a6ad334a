"""Algorithm 1 (primal-dual) and Algorithm 2 (reweighting) of Polarized SARA.

TEST INFRASTRUCTURE ONLY.  FP64 restatement of Sec. 3.3 with the readings
listed in ``oracle.prox``.  Variables follow the paper: primal S (N x 4) and Z
(N x 2); duals A (J x 4, sparsity), B (M x 4 complex, data fidelity -- complex
as in eq. min_gen2_dual, although Algorithm 1's header lists it as real),
C (N x 4) and D (N x 2) (epigraphs).

Stages / modes:
  * ``"init"``     : the initialisation of Sec. 3.3.4 -- g = 0, no polarization
                     constraint, S projected on U' (Stokes I >= 0); only S and B
                     are updated, all other variables stay zero;
  * ``"polsara"``  : problem eq. min_gen2 (all terms: U, weighted l1, l2 ball, V,
                     E1, E2);
  * ``"nocons"``   : "Polarized SARA without constraint", eq.
                     min_gen_matrix_no_flux (U', weighted l1, l2 ball; Sec. 4.2);
  * ``"plain"``    : U, weighted l1, l2 ball only (used by closed-form tests);
  * ``"cone"``     : test-only cross-check replacing the epigraphical split by a
                     dual variable on the direct Lorentz-cone projection.
Step sizes (the paper gives only the condition of Sec. 3.3.3): rho1 = rho3 = 1,
rho2 = 1/||phi||^2, tau = 0.99 / (rho1 ||Psi||^2 + rho2 ||phi||^2 + rho3).
Initial variables are zero (the paper does not fix them).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

from . import metrics
from .prox import (proj_E1, proj_E2, proj_U, proj_U_prime, proj_V, soft_threshold, proj_ball,
                   proj_polarization_cone)

MODES = ("init", "polsara", "nocons", "plain", "cone")


@dataclass
class State:
    S: np.ndarray
    Z: np.ndarray
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    D: np.ndarray

    @staticmethod
    def zeros(N: int, J: int, M: int) -> "State":
        return State(np.zeros((N, 4)), np.zeros((N, 2)), np.zeros((J, 4)),
                     np.zeros((M, 4), dtype=np.complex128), np.zeros((N, 4)), np.zeros((N, 2)))

    def copy(self) -> "State":
        return State(*(np.array(v, copy=True) for v in (self.S, self.Z, self.A, self.B, self.C, self.D)))


@dataclass
class Problem:
    """Operators and constants of one solve.  phi/phi_adj/psi/psi_adj are callables on matrices."""
    phi: object
    phi_adj: object
    psi: object
    psi_adj: object
    Y: np.ndarray
    eps: float
    tau: float
    rho1: float
    rho2: float
    rho3: float


def step_sizes(phi_norm_sq: float, psi_norm_sq: float = 1.0, margin: float = 0.99):
    """(tau, rho1, rho2, rho3) meeting 1/tau - rho1||Psi||^2 - rho2||phi||^2 - rho3 >= 0 (Sec. 3.3.3)."""
    rho1, rho3 = 1.0, 1.0
    rho2 = 1.0 / phi_norm_sq
    tau = margin / (rho1 * psi_norm_sq + rho2 * phi_norm_sq + rho3)
    return tau, rho1, rho2, rho3


def alg1_iteration(st: State, pb: Problem, gammaW: np.ndarray, mode: str = "polsara") -> State:
    """One iteration k -> k+1 of Algorithm 1, steps in the paper's order."""
    tau, r1, r2, r3 = pb.tau, pb.rho1, pb.rho2, pb.rho3
    use_l1 = mode in ("polsara", "nocons", "plain", "cone")
    use_epi = mode == "polsara"
    use_cone = mode == "cone"

    # -- primal updates ------------------------------------------------------
    grad = pb.phi_adj(st.B)
    if use_l1:
        grad = grad + pb.psi(st.A)
    if use_epi or use_cone:
        grad = grad + st.C
    arg = st.S - tau * grad
    S1 = proj_U_prime(arg) if mode in ("init", "nocons") else proj_U(arg)
    Z1 = proj_V(st.Z - tau * st.D) if use_epi else st.Z
    X = 2.0 * S1 - st.S

    # -- dual updates: sparsity --------------------------------------------
    if use_l1:
        At = st.A + r1 * pb.psi_adj(X)
        A1 = At - r1 * soft_threshold(At / r1, gammaW / r1)
    else:
        A1 = st.A

    # -- dual updates: l2 ball ---------------------------------------------
    Bt = st.B + r2 * pb.phi(X)
    B1 = Bt - r2 * proj_ball(Bt / r2, pb.Y, pb.eps)

    # -- dual updates: epigraphical projections --------------------------------
    C1, D1 = st.C, st.D
    if use_epi:
        Ct = st.C + r3 * X
        Dt = st.D + r3 * (2.0 * Z1 - st.Z)
        c1, d1 = proj_E1(Ct[:, 0] / r3, Dt[:, 0] / r3)
        C1 = np.empty_like(Ct)
        D1 = np.empty_like(Dt)
        C1[:, 0] = Ct[:, 0] - r3 * c1
        D1[:, 0] = Dt[:, 0] - r3 * d1
        R2, d2 = proj_E2(Ct[:, 1:4] / r3, Dt[:, 1] / r3)
        C1[:, 1:4] = Ct[:, 1:4] - r3 * R2
        D1[:, 1] = Dt[:, 1] - r3 * d2
    elif use_cone:
        Ct = st.C + r3 * X
        C1 = Ct - r3 * proj_polarization_cone(Ct / r3)
    return State(S1, Z1, A1, B1, C1, D1)


def run_alg1(st: State, pb: Problem, gammaW: np.ndarray, iters: int, mode: str = "polsara",
             callback=None) -> State:
    for k in range(iters):
        st = alg1_iteration(st, pb, gammaW, mode)
        if callback is not None:
            callback(k, st)
    return st


def stop_criteria(pb: Problem, S_new: np.ndarray, S_old: np.ndarray, theta: float, rel_var: float,
                  np_max: float):
    """The stopping test of the paper's simulation settings (Sec. 4.6 and the settings that
    follow it): the residual ||phi(S) - Y|| is within (1 + theta) epsilon, the relative variation
    ||S_i^(k+1) - S_i^(k)|| / ||S_i^(k)|| of every Stokes map i is at most rel_var, and, for the
    constrained problem (np_max >= 0), N_p (percent, Sec. 4.2) is at most np_max.  Readings: all
    four maps enter the relative variation; a map that is zero in both iterates varies by 0.
    Returns (met, residual, largest relative variation, N_p)."""
    res = metrics.residual_norm(pb, S_new, pb.Y)
    num = np.linalg.norm(S_new - S_old, axis=0)
    den = np.linalg.norm(S_old, axis=0)
    rv = max(float(a / b) if b > 0 else (math.inf if a > 0 else 0.0) for a, b in zip(num, den))
    n_p = metrics.polarization_error(pb, S_new, pb.Y)[2] if np_max >= 0 else 0.0
    met = res <= (1.0 + theta) * pb.eps and rv <= rel_var and (np_max < 0 or n_p <= np_max)
    return met, res, rv, n_p


def run_alg1_adaptive(st: State, pb: Problem, gammaW: np.ndarray, mode: str, max_iters: int, check_every: int,
                      theta: float, rel_var: float, np_max: float):
    """Algorithm 1 tested against `stop_criteria` after every block of check_every iterations
    (the last block may be shorter), stopping at the first block after which the test holds or
    after max_iters iterations.  Returns (state, iterations run)."""
    done = 0
    while done < max_iters:
        k = min(check_every, max_iters - done)
        prev = st.S
        for _ in range(k):
            prev = st.S
            st = alg1_iteration(st, pb, gammaW, mode)
        done += k
        if stop_criteria(pb, st.S, prev, theta, rel_var, np_max)[0]:
            break
    return st, done


def reweight(pb: Problem, S: np.ndarray, delta: float) -> np.ndarray:
    """Weights of eq. weights: W = delta / (delta + |Psi^dagger S|)."""
    return delta / (delta + np.abs(pb.psi_adj(S)))


def split_iterations(total: int, stages: int):
    """Even split of a total iteration budget over `stages` stages; remainder to the last."""
    base = total // stages
    out = [base] * stages
    out[-1] += total - base * stages
    return out


def alg2(pb: Problem, gamma: float, iters, cycles: int, mode: str = "polsara",
         delta_decay: float = 10.0, callback=None):
    """Algorithm 2: initialisation stage, then `cycles` reweighted solves (warm-started).

    iters: list of per-stage iteration counts (init stage first), length cycles + 1.
    delta^(1) = std of the entries of Psi^dagger S after the initialisation stage,
    then divided by ``delta_decay`` each cycle (the paper only requires
    delta -> 0; this schedule is a reading).  Returns (state, gammaW, deltas).
    """
    S0 = pb.psi_adj(np.zeros((_n_pixels(pb), 4)))
    J = S0.shape[0]
    st = State.zeros(_n_pixels(pb), J, pb.Y.shape[0])
    ones = np.ones((J, 4))
    st = run_alg1(st, pb, gamma * ones, iters[0], "init")
    if callback is not None:
        callback(0, st)
    delta = float(np.std(pb.psi_adj(st.S)))
    deltas = []
    gW = gamma * ones
    for l in range(1, cycles + 1):
        W = reweight(pb, st.S, delta)
        gW = gamma * W
        deltas.append(delta)
        st = run_alg1(st, pb, gW, iters[l], mode)
        if callback is not None:
            callback(l, st)
        delta /= delta_decay
    return st, gW, deltas


def alg2_adaptive(pb: Problem, gamma: float, cycles: int, max_iters: int, check_every: int, theta: float,
                  rel_var: float, np_max: float, mode: str = "polsara", delta_decay: float = 10.0):
    """Algorithm 2 whose stages end by `stop_criteria` (run_alg1_adaptive, at most max_iters
    iterations each); the initialisation stage leaves N_p out of the test (the constraint is not
    part of its problem).  Returns (state, gammaW, iterations per stage)."""
    S0 = pb.psi_adj(np.zeros((_n_pixels(pb), 4)))
    J = S0.shape[0]
    st = State.zeros(_n_pixels(pb), J, pb.Y.shape[0])
    ones = np.ones((J, 4))
    st, it = run_alg1_adaptive(st, pb, gamma * ones, "init", max_iters, check_every, theta, rel_var, -1.0)
    its = [it]
    delta = float(np.std(pb.psi_adj(st.S)))
    gW = gamma * ones
    for _ in range(cycles):
        gW = gamma * reweight(pb, st.S, delta)
        st, it = run_alg1_adaptive(st, pb, gW, mode, max_iters, check_every, theta, rel_var, np_max)
        its.append(it)
        delta /= delta_decay
    return st, gW, its


def _n_pixels(pb: Problem) -> int:
    return pb.phi_adj(np.zeros_like(pb.Y)).shape[0]


def power_iteration(op, x0: np.ndarray, max_iter: int = 1000, rtol: float = 1e-12):
    """Largest eigenvalue of the symmetric PSD map `op` (power method, FP64)."""
    x = x0 / np.linalg.norm(x0)
    lam = 0.0
    for it in range(max_iter):
        y = op(x)
        lam_new = float(np.vdot(x, y).real)
        x = y / np.linalg.norm(y)
        if it > 0 and abs(lam_new - lam) <= rtol * abs(lam_new):
            lam = lam_new
            break
        lam = lam_new
    return lam, it + 1


def phi_norm_sq(mop, N: int, seed: int = 12345, max_iter: int = 1000, rtol: float = 1e-12):
    """||phi||^2 of the real-restricted map X -> Re phi^dagger phi X on N x 4 (power method)."""
    x0 = np.random.default_rng(seed).standard_normal((N, 4))
    return power_iteration(lambda x: np.real(mop.phi_adj(mop.phi(x))), x0, max_iter, rtol)
