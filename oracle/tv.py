"""Algorithm 3 (Sec. 4.3, the TV-based problems) for the independent-Stokes data fidelity of
eq. Akiyama and its constrained generalisation eq. Akiyama_2.  TEST INFRASTRUCTURE ONLY.

FP64 restatement:
  * phi~(S) = Phi(S), the operator without the brightness mixing L, on the data
    Y~ = Y L^{-1}; the data term 1/2 ||Y~ - phi~(S)||^2 enters the primal step through its
    gradient Re phi~^dagger (phi~(S) - Y~) (step 3 of the algorithm);
  * TV: Psi = grad, the concatenation of the forward differences along the two image axes,
    g(Psi^dagger S) = sum_i mu_i ||grad S_i||_{2,1} (eq. TV, isotropic); l1 + TV:
    Psi = [1, grad] with the l1 norm on the Dirac block, weights upsilon_1 and upsilon_2;
  * the dual step A = A~ - rho1 T(A~ / rho1) with T the proximity operator of the weighted
    norm at threshold Lambda / rho1: on a gradient pair the l2,1 norm's (group soft
    thresholding), on the Dirac block the soft threshold; the primal-dual split applies grad
    through its dual variable, so no inner iterations are needed;
  * the primal step P_U (constrained, with C; Z, C, D as in Algorithm 1) or P_U' (eq. Akiyama:
    no constraint, only steps 3, 5 and 6).
Readings: forward differences with a zero difference at the last row / column (the discrete
TV of Chambolle 2004; the paper does not fix the boundary); pixel p = n1 * n + n2 with n1 the
first image index; step sizes rho1 = 1 / ||Psi||^2 (8 for grad, 9 for [1, grad]), rho3 = 1 and
tau = 0.99 / (beta / 2 + rho1 ||Psi||^2 + rho3) with beta = ||phi~||^2 the Lipschitz constant of
the data term's gradient (the primal-dual condition with a smooth term, Condat 2013 and Vu
2013; the paper states the condition only for Algorithm 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .nufft import L_MIX
from .pd import State
from .prox import proj_E1, proj_E2, proj_U, proj_U_prime, proj_V, soft_threshold

PSI_NORM_SQ = {"tv": 8.0, "l1tv": 9.0}
L_INV = np.linalg.inv(L_MIX)


def d1(U: np.ndarray, n: int) -> np.ndarray:
    """Forward difference along the first image index (rows), zero on the last row; U is
    (n*n, k) with pixel p = n1 * n + n2."""
    V = U.reshape(n, n, -1)
    out = np.zeros_like(V)
    out[:-1] = V[1:] - V[:-1]
    return out.reshape(n * n, -1)


def d2(U: np.ndarray, n: int) -> np.ndarray:
    """Forward difference along the second image index (columns), zero on the last column."""
    V = U.reshape(n, n, -1)
    out = np.zeros_like(V)
    out[:, :-1] = V[:, 1:] - V[:, :-1]
    return out.reshape(n * n, -1)


def d1_adj(G: np.ndarray, n: int) -> np.ndarray:
    """The adjoint of d1 (minus the backward-difference divergence)."""
    V = G.reshape(n, n, -1)
    out = np.zeros_like(V)
    out[1:] += V[:-1]
    out[:-1] -= V[:-1]
    return out.reshape(n * n, -1)


def d2_adj(G: np.ndarray, n: int) -> np.ndarray:
    V = G.reshape(n, n, -1)
    out = np.zeros_like(V)
    out[:, 1:] += V[:, :-1]
    out[:, :-1] -= V[:, :-1]
    return out.reshape(n * n, -1)


def psi_adj(S: np.ndarray, n: int, kind: str) -> np.ndarray:
    """Psi^dagger S: [d1 S; d2 S] (TV) or [S; d1 S; d2 S] (l1 + TV)."""
    blocks = [d1(S, n), d2(S, n)]
    if kind == "l1tv":
        blocks = [S] + blocks
    return np.concatenate(blocks, axis=0)


def psi(A: np.ndarray, n: int, kind: str) -> np.ndarray:
    N = n * n
    off = N if kind == "l1tv" else 0
    out = d1_adj(A[off:off + N], n) + d2_adj(A[off + N:off + 2 * N], n)
    if kind == "l1tv":
        out = out + A[:N]
    return out


def group_soft_threshold(V1: np.ndarray, V2: np.ndarray, t: np.ndarray):
    """Proximity operator of t ||.||_{2,1} on pixel pairs (V1, V2): each pair shrinks towards 0
    by t in Euclidean norm (to 0 when its norm is at most t)."""
    nrm = np.sqrt(V1 ** 2 + V2 ** 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(nrm > t, 1.0 - t / np.where(nrm > 0, nrm, 1.0), 0.0)
    return f * V1, f * V2


@dataclass
class TVProblem:
    """Operators and constants of one TV-based solve (phi~ acts on real N x 4 Stokes matrices)."""
    phit: object          # S -> Phi S (M x 4 complex)
    phit_adj: object      # R -> Phi^dagger R (N x 4 complex)
    Yt: np.ndarray        # Y L^{-1}
    n: int
    kind: str             # "tv" or "l1tv"
    tv_weight: np.ndarray   # mu_i (or upsilon_2,i), length 4
    l1_weight: np.ndarray   # upsilon_1,i (l1 + TV), length 4
    tau: float
    rho1: float
    rho3: float


def step_sizes(beta: float, kind: str, margin: float = 0.99):
    psi2 = PSI_NORM_SQ[kind]
    rho1, rho3 = 1.0 / psi2, 1.0
    return margin / (beta / 2.0 + rho1 * psi2 + rho3), rho1, rho3


def build(nufft, Y: np.ndarray, n: int, kind: str, tv_weight, l1_weight, beta: float) -> TVProblem:
    tau, rho1, rho3 = step_sizes(beta, kind)
    return TVProblem(lambda S: nufft.forward(np.asarray(S, dtype=np.complex128)), nufft.adjoint,
                     np.asarray(Y) @ L_INV, n, kind, np.asarray(tv_weight, dtype=float),
                     np.asarray(l1_weight if l1_weight is not None else np.zeros(4), dtype=float),
                     tau, rho1, rho3)


def data_gradient(pb: TVProblem, S: np.ndarray) -> np.ndarray:
    return np.real(pb.phit_adj(pb.phit(S) - pb.Yt))


def alg3_iteration(st: State, pb: TVProblem, constrained: bool) -> State:
    """One iteration of Algorithm 3 (the state's B is not used).  A holds the dual of Psi^dagger:
    [Dirac block (l1 + TV)], d1 block, d2 block, each N x 4."""
    n, N = pb.n, pb.n * pb.n
    tau, r1, r3 = pb.tau, pb.rho1, pb.rho3
    # -- primal updates
    g = data_gradient(pb, st.S) + psi(st.A, n, pb.kind)
    if constrained:
        g = g + st.C
    arg = st.S - tau * g
    S1 = proj_U(arg) if constrained else proj_U_prime(arg)
    Z1 = proj_V(st.Z - tau * st.D) if constrained else st.Z
    X = 2.0 * S1 - st.S
    # -- dual updates: sparsity, A = A~ - rho1 T(A~ / rho1)
    At = st.A + r1 * psi_adj(X, n, pb.kind)
    A1 = np.empty_like(At)
    off = 0
    if pb.kind == "l1tv":
        A1[:N] = At[:N] - r1 * soft_threshold(At[:N] / r1, pb.l1_weight[None, :] / r1)
        off = N
    G1, G2 = At[off:off + N], At[off + N:off + 2 * N]
    T1, T2 = group_soft_threshold(G1 / r1, G2 / r1, pb.tv_weight[None, :] / r1)
    A1[off:off + N] = G1 - r1 * T1
    A1[off + N:off + 2 * N] = G2 - r1 * T2
    # -- dual updates: epigraphical projections (as Algorithm 1)
    C1, D1 = st.C, st.D
    if constrained:
        Ct = st.C + r3 * X
        Dt = st.D + r3 * (2.0 * Z1 - st.Z)
        c1, e1 = proj_E1(Ct[:, 0] / r3, Dt[:, 0] / r3)
        C1 = np.empty_like(Ct)
        D1 = np.empty_like(Dt)
        C1[:, 0] = Ct[:, 0] - r3 * c1
        D1[:, 0] = Dt[:, 0] - r3 * e1
        R2, e2 = proj_E2(Ct[:, 1:4] / r3, Dt[:, 1] / r3)
        C1[:, 1:4] = Ct[:, 1:4] - r3 * R2
        D1[:, 1] = Dt[:, 1] - r3 * e2
    return State(S1, Z1, A1, st.B, C1, D1)


def run_alg3(st: State, pb: TVProblem, iters: int, constrained: bool) -> State:
    for _ in range(iters):
        st = alg3_iteration(st, pb, constrained)
    return st


def objective(pb: TVProblem, S: np.ndarray) -> float:
    """1/2 ||Y~ - phi~(S)||^2 + sum_i mu_i ||grad S_i||_{2,1} (+ sum_i upsilon_1,i ||S_i||_1)."""
    n = pb.n
    tv = np.sqrt(d1(S, n) ** 2 + d2(S, n) ** 2)
    val = 0.5 * float(np.sum(np.abs(pb.Yt - pb.phit(S)) ** 2)) + float(np.sum(tv * pb.tv_weight[None, :]))
    if pb.kind == "l1tv":
        val += float(np.sum(np.abs(S) * pb.l1_weight[None, :]))
    return val


def zeros(n: int, M: int, kind: str) -> State:
    N = n * n
    J = (3 if kind == "l1tv" else 2) * N
    return State(np.zeros((N, 4)), np.zeros((N, 2)), np.zeros((J, 4)),
                 np.zeros((M, 4), dtype=np.complex128), np.zeros((N, 4)), np.zeros((N, 2)))
