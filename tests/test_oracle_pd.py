"""Pins of the oracle's Algorithm 1 / Algorithm 2 (Sec. 3.3)."""
import dataclasses
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq, minimize

from oracle import pd, metrics, problem
from oracle.nufft import NUFFT, MeasurementOp
from oracle.prox import soft_threshold
from oracle.sara import SARA
from paper_1801_02417_amd import workloads as wk

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _with_steps(pb, phi_norm, rho1, rho2_scale, rho3):
    rho2 = rho2_scale / phi_norm
    tau = 0.99 / (rho1 + rho2 * phi_norm + rho3)
    return dataclasses.replace(pb, tau=tau, rho1=rho1, rho2=rho2, rho3=rho3)


def _high_pol_tiny():
    wl = wk.tiny(seed=11)
    rng = np.random.default_rng(5)
    I = wl.truth[..., 0]
    chi = math.pi * rng.uniform(size=I.shape)
    wl.truth = np.stack([I, 0.95 * I * np.cos(2 * chi), 0.95 * I * np.sin(2 * chi), 0 * I], -1)
    return wl


@pytest.fixture(scope="module")
def tiny_built():
    return problem.build(wk.tiny())


def test_step_size_condition():
    tau, r1, r2, r3 = pd.step_sizes(1234.5)
    assert 1 / tau - r1 * 1.0 - r2 * 1234.5 - r3 >= 0


def test_convergence_same_objective_for_steps_and_gamma(tiny_built):
    """Four runs (two step-size sets x two gamma) reach the same objective and an active data
    constraint; gamma only changes the speed (Sec. 3.3.1)."""
    b = tiny_built
    J = b.sara.J
    W = np.ones((J, 4))
    objs, ress, viol = [], [], []
    for steps in ((1.0, 1.0, 1.0), (2.0, 0.3, 0.5)):
        pb = _with_steps(b.pb, b.phi_norm_sq, *steps)
        for gamma in (b.gamma, 5 * b.gamma):
            st = pd.run_alg1(pd.State.zeros(256, J, b.pb.Y.shape[0]), pb, gamma * W, 4000, "polsara")
            objs.append(metrics.weighted_l1(b.sara.adjoint, st.S, W))
            ress.append(metrics.residual_norm(b.mop, st.S, b.pb.Y))
            viol.append(metrics.cone_violation(st.S))
    objs = np.array(objs)
    assert np.max(np.abs(objs - objs.mean())) <= 1e-6 * objs.mean()
    assert np.linalg.norm(b.pb.Y) > b.pb.eps
    for r in ress:
        assert abs(r / b.pb.eps - 1.0) <= 1e-6
    assert max(viol) <= 1e-8 * b.truth[:, 0].max()


def test_epigraph_split_matches_direct_cone_projection_when_active():
    """Polarisation cone active: the epigraphical split and a direct Lorentz-cone dual reach the same
    objective, above the unconstrained one, with the constraint met."""
    b = problem.build(_high_pol_tiny())
    J = b.sara.J
    W = np.ones((J, 4))
    out = {}
    for mode, its in (("polsara", 6000), ("cone", 6000), ("nocons", 4000)):
        st = pd.run_alg1(pd.State.zeros(256, J, b.pb.Y.shape[0]), b.pb, b.gamma * W, its, mode)
        out[mode] = (metrics.weighted_l1(b.sara.adjoint, st.S, W), metrics.cone_violation(st.S), st)
    o_pol, o_cone, o_nc = out["polsara"][0], out["cone"][0], out["nocons"][0]
    # measured agreement 6.4e-7 relative after 6000 iterations
    assert abs(o_pol - o_cone) <= 2e-6 * o_pol
    assert o_nc < o_pol * (1 - 1e-3)                     # the constraint costs objective
    assert out["nocons"][1] > 1e-2                        # ... because the unconstrained solution violates it
    assert out["polsara"][1] <= 1e-6 * b.truth[:, 0].max()
    assert out["cone"][1] <= 1e-6 * b.truth[:, 0].max()


def test_matches_brute_force_on_4x4():
    """Dirac prior, 4x4 Stokes images, M = 20: SLSQP on the explicit l1 / l2-ball / cone problem."""
    rng = np.random.default_rng(3)
    n, N, M = 4, 16, 20
    uv = np.clip(rng.normal(0, 1.0, size=(M, 2)), -math.pi, math.pi - 1e-9)
    mop = MeasurementOp(NUFFT(uv, n, 2, 6))
    I = rng.uniform(0.2, 1, size=N)
    chi = rng.uniform(0, np.pi, N)
    S = np.stack([I, 0.9 * I * np.cos(2 * chi), 0.9 * I * np.sin(2 * chi), 0.05 * I], 1)
    y0 = mop.phi(S)
    sigma = 0.05 * np.linalg.norm(y0) / math.sqrt(4 * M)
    Y = y0 + sigma * (rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4))) / math.sqrt(2)
    eps = problem.chi2_epsilon(M, sigma)

    A = np.zeros((128, 128))
    A[:64, :64], A[:64, 64:], A[64:, :64], A[64:, 64:] = np.eye(64), np.eye(64), -np.eye(64), np.eye(64)

    def data(z):
        return eps ** 2 - np.sum(np.abs(mop.phi(z[:64].reshape(N, 4)) - Y) ** 2)

    def data_j(z):
        g = np.zeros(128)
        g[:64] = -2 * np.real(mop.phi_adj(mop.phi(z[:64].reshape(N, 4)) - Y)).ravel()
        return g

    def cone(z):
        X = z[:64].reshape(N, 4)
        return np.concatenate([X[:, 0] ** 2 - np.sum(X[:, 1:] ** 2, 1), X[:, 0]])

    def cone_j(z):
        X = z[:64].reshape(N, 4)
        Jm = np.zeros((2 * N, 128))
        for i in range(N):
            Jm[i, 4 * i] = 2 * X[i, 0]
            Jm[i, 4 * i + 1:4 * i + 4] = -2 * X[i, 1:]
            Jm[N + i, 4 * i] = 1
        return Jm

    cons = [{"type": "ineq", "fun": lambda z: A @ z, "jac": lambda z: A},
            {"type": "ineq", "fun": data, "jac": data_j},
            {"type": "ineq", "fun": cone, "jac": cone_j}]
    z0 = np.concatenate([S.ravel(), np.abs(S.ravel()) + 0.01])
    r = minimize(lambda z: z[64:].sum(), z0, jac=lambda z: np.r_[np.zeros(64), np.ones(64)],
                 constraints=cons, method="SLSQP", options={"maxiter": 2000, "ftol": 1e-12})
    brute = float(np.abs(r.x[:64]).sum())

    pn, _ = pd.phi_norm_sq(mop, N)
    tau, r1, r2, r3 = pd.step_sizes(pn)
    sara = SARA(n, 0, ("dirac",))
    pb = pd.Problem(mop.phi, mop.phi_adj, sara.forward, sara.adjoint, Y, eps, tau, r1, r2, r3)
    st = pd.run_alg1(pd.State.zeros(N, N, M), pb, 0.1 * np.ones((N, 4)), 4000, "polsara")
    got = float(np.abs(st.S).sum())
    assert abs(got - brute) <= 1e-7 * brute
    assert abs(metrics.residual_norm(mop, st.S, Y) / eps - 1) < 1e-9


def test_zero_solution_when_data_inside_ball(tiny_built):
    b = tiny_built
    pb = dataclasses.replace(b.pb, Y=b.pb.Y * 1e-3, eps=1.01 * np.linalg.norm(b.pb.Y * 1e-3))
    rng = np.random.default_rng(0)
    st = pd.State.zeros(256, b.sara.J, pb.Y.shape[0])
    st.S = rng.standard_normal((256, 4)) * 0.1
    st = pd.run_alg1(st, pb, b.gamma * np.ones((b.sara.J, 4)), 3000, "polsara")
    assert np.max(np.abs(st.S)) < 1e-7


def test_denoising_closed_form():
    """Phi = I, Psi = Dirac, W = 1, no cone: the solution is soft(Y, lambda*) with
    ||soft(Y, lambda*) - Y|| = epsilon (l1 ball-constrained denoising)."""
    rng = np.random.default_rng(17)
    N = 64
    Y = rng.standard_normal((N, 4)) * np.array([3.0, 1.0, 1.0, 0.3])
    eps = 0.2 * np.linalg.norm(Y)
    lam = brentq(lambda t: np.linalg.norm(soft_threshold(Y, t) - Y) - eps, 0.0, np.max(np.abs(Y)))
    ref = soft_threshold(Y, lam)
    ident = lambda X: np.asarray(X, dtype=np.complex128)
    tau, r1, r2, r3 = pd.step_sizes(1.0)
    pb = pd.Problem(ident, lambda B: np.asarray(B), lambda A: np.real(A), lambda S: np.real(S),
                    Y.astype(np.complex128), eps, tau, r1, r2, r3)
    st = pd.run_alg1(pd.State.zeros(N, N, N), pb, 0.5 * np.ones((N, 4)), 3000, "plain")
    assert np.max(np.abs(st.S - ref)) < 1e-9 * np.max(np.abs(Y))


def test_iteration_invariants(tiny_built):
    """I1 |A| <= gW; I2 C1 = D1 <= 0; I3 ||C_{2:4}|| <= -D2; I4 Z1 + Z2 <= 0;
    I5 B' = c (B~ - rho2 Y), c in [0, 1)  -- after every iteration."""
    b = tiny_built
    pb = b.pb
    J = b.sara.J
    gW = b.gamma * np.random.default_rng(2).uniform(0.1, 1.0, size=(J, 4))
    st = pd.State.zeros(256, J, pb.Y.shape[0])
    for k in range(60):
        nxt = pd.alg1_iteration(st, pb, gW, "polsara")
        At = st.A + pb.rho1 * pb.psi_adj(2 * nxt.S - st.S)
        # A~ - rho1 T(A~/rho1) cancels: allow a few ulps of |A~|
        assert np.all(np.abs(nxt.A) <= gW + 4 * np.finfo(float).eps * np.abs(At))
        Ct1 = st.C[:, 0] + pb.rho3 * (2 * nxt.S[:, 0] - st.S[:, 0])
        Dt1 = st.D[:, 0] + pb.rho3 * (2 * nxt.Z[:, 0] - st.Z[:, 0])
        ulp = 4 * np.finfo(float).eps * (np.abs(Ct1) + np.abs(Dt1))
        assert np.all(np.abs(nxt.C[:, 0] - nxt.D[:, 0]) <= ulp) and np.all(nxt.C[:, 0] <= 0)
        Ct = st.C[:, 1:] + pb.rho3 * (2 * nxt.S[:, 1:] - st.S[:, 1:])
        Dt2 = st.D[:, 1] + pb.rho3 * (2 * nxt.Z[:, 1] - st.Z[:, 1])
        ulp2 = 8 * np.finfo(float).eps * (np.linalg.norm(Ct, axis=1) + np.abs(Dt2))
        assert np.all(np.linalg.norm(nxt.C[:, 1:], axis=1) <= -nxt.D[:, 1] + ulp2)
        assert np.all(nxt.Z[:, 0] + nxt.Z[:, 1] <= 1e-15)
        X = 2 * nxt.S - st.S
        base = st.B + pb.rho2 * pb.phi(X) - pb.rho2 * pb.Y
        c = np.vdot(base, nxt.B).real / np.vdot(base, base).real
        assert 0 <= c < 1
        assert np.max(np.abs(nxt.B - c * base)) <= 1e-13 * np.max(np.abs(base))
        st = nxt


def test_init_stage_updates_only_S_and_B(tiny_built):
    b = tiny_built
    J = b.sara.J
    st = pd.run_alg1(pd.State.zeros(256, J, b.pb.Y.shape[0]), b.pb, np.ones((J, 4)), 20, "init")
    for v in (st.Z, st.A, st.C, st.D):
        assert not np.any(v)
    assert np.all(st.S[:, 0] >= 0) and np.any(st.S) and np.any(st.B)


def test_reweighting_formula(tiny_built):
    b = tiny_built
    S = np.random.default_rng(1).standard_normal((256, 4))
    W = pd.reweight(b.pb, S, 0.25)
    c = b.sara.adjoint(S)
    assert np.allclose(W * (0.25 + np.abs(c)), 0.25, rtol=1e-15, atol=0)
    assert np.all((W > 0) & (W <= 1))


def test_alg2_on_blobs32_meets_constraints():
    wl = wk.blobs32()
    b = problem.build(wl)
    st, gW, deltas = pd.alg2(b.pb, b.gamma, pd.split_iterations(wl.iters, wl.cycles + 1), wl.cycles)
    assert len(deltas) == 2 and deltas[1] == deltas[0] / 10
    res = metrics.residual_norm(b.mop, st.S, b.pb.Y)
    assert res <= 1.001 * b.pb.eps
    assert metrics.cone_violation(st.S) <= 1e-3 * b.truth[:, 0].max()
    assert metrics.snr_db(st.S[:, 0], b.truth[:, 0]) > 30.0


def test_split_iterations():
    assert pd.split_iterations(300, 3) == [100, 100, 100]
    assert pd.split_iterations(2000, 6) == [333, 333, 333, 333, 333, 335]


def test_table1_snr_uses_natural_log():
    """Sec. 4.7 defines SNR with log10, but every printed Table 1 pair satisfies SNR ~ -20 ln(NRMSE)."""
    with open(os.path.join(GOLDEN, "table1_snr_nrmse.json")) as f:
        pairs = json.load(f)["pairs"]
    dev = [abs(snr - (-20 * math.log(e))) for snr, e in pairs]
    # 22 of the 24 cells agree to 0.03 dB, the other two to 0.25 dB (means over 5 runs)
    assert max(dev) <= 0.3 and sorted(dev)[len(dev) // 2] <= 0.01
    for snr, e in pairs:      # the log10 value would be snr / ln(10)
        assert abs(snr - (-20 * math.log10(e))) >= 0.5 * snr


def test_metrics():
    t = np.array([3.0, 4.0])
    e = np.array([3.0, 4.5])
    assert abs(metrics.nrmse(e, t) - 0.1) < 1e-15
    assert abs(metrics.snr_db(e, t) - 20.0) < 1e-12
    rv = metrics.relative_variation(np.array([[1.0, 0.0]]), np.array([[2.0, 0.0]]))
    assert rv[0] == 0.5 and np.isinf(rv[1])
    assert metrics.cone_violation(np.array([[1.0, 3.0, 4.0, 0.0], [5.0, 3.0, 4.0, 0.0]])) == 4.0


def test_chi2_epsilon():
    # eps^2 = (8M + 2 sqrt(2 * 8M)) sigma^2 / 2 with M = 2, sigma = 1: (16 + 2*sqrt(32))/2
    assert abs(problem.chi2_epsilon(2, 1.0) ** 2 - (16 + 2 * math.sqrt(32)) / 2) < 1e-13


def test_stop_criteria_closed_forms():
    """The stopping test on states whose quantities are known exactly: noise-free data
    Y = phi(S_true), so the residual at S_true is 0 and the residual image (hence zeta) is 0;
    N_p then counts the pixels with ||S_2:4|| > S_1 by construction; the relative variation
    is the column-norm ratio, with 0/0 read as 0 and x/0 as infinite."""
    wl = wk.tiny(n=16, M=150, taps=6, levels=2, seed=7)
    b = problem.build(wl)
    S = wl.truth.reshape(-1, 4).copy()
    pb = dataclasses.replace(b.pb, Y=b.pb.phi(S), eps=1e-3)
    # residual 0 <= (1 + theta) eps; unchanged iterate: relative variation 0; truth in the cone
    met, res, rv, n_p = pd.stop_criteria(pb, S, S, 0.0, 0.0, 0.0)
    assert met and res < 1e-12 and rv == 0.0 and n_p == 0.0
    # a known relative variation per map: scale map 2 by 1.1 -> 0.1 / 1
    S2 = S.copy()
    S2[:, 2] *= 1.1
    _, _, rv, _ = pd.stop_criteria(pb, S2, S, 1e9, 1.0, -1.0)
    assert abs(rv - 0.1) < 1e-12
    assert not pd.stop_criteria(pb, S2, S, 1e9, 0.0999, -1.0)[0]
    assert pd.stop_criteria(pb, S2, S, 1e9, 0.1001, -1.0)[0]
    # 0/0 -> 0 and x/0 -> inf for a map that is zero in the old iterate
    Sz = S.copy()
    Sz[:, 3] = 0.0
    assert pd.stop_criteria(pb, Sz, Sz, 1e9, 0.0, -1.0)[2] == 0.0
    Sn = Sz.copy()
    Sn[0, 3] = 1e-3
    assert pd.stop_criteria(pb, Sn, Sz, 1e9, 1e9, -1.0)[2] == math.inf
    # N_p: push k pixels out of the cone (zeta = 0 with noise-free data at S)
    k = 13
    Sp = S.copy()
    Sp[:k, 1] = Sp[:k, 0] + 1.0
    pbp = dataclasses.replace(pb, Y=pb.phi(Sp))
    _, _, _, n_p = pd.stop_criteria(pbp, Sp, Sp, 0.0, 0.0, 0.0)
    assert abs(n_p - 100.0 * k / S.shape[0]) < 1e-12
    assert not pd.stop_criteria(pbp, Sp, Sp, 0.0, 0.0, 100.0 * k / S.shape[0] - 1e-9)[0]
    assert pd.stop_criteria(pbp, Sp, Sp, 0.0, 0.0, 100.0 * k / S.shape[0])[0]
    # the residual bound: (1 + theta) eps with eps at the residual of S = 0
    r0 = float(np.linalg.norm(pb.Y))
    pbr = dataclasses.replace(pb, eps=r0)
    Z = np.zeros_like(S)
    assert pd.stop_criteria(pbr, Z, Z, 0.0, 0.0, -1.0)[0]
    assert not pd.stop_criteria(dataclasses.replace(pbr, eps=r0 * (1 - 1e-6)), Z, Z, 0.0, 0.0, -1.0)[0]


def test_run_alg1_adaptive_stops_at_first_passing_check(tiny_built):
    """run_alg1_adaptive returns the state of run_alg1 after the iterations it reports, the test
    fails after every earlier block and holds after the last one; with an unreachable test it
    runs exactly max_iters (a last partial block included)."""
    b = tiny_built
    J = b.sara.J
    gW = b.gamma * np.ones((J, 4))
    N = b.pb.psi(np.zeros((J, 4))).shape[0]
    st0 = pd.run_alg1(pd.State.zeros(N, J, b.pb.Y.shape[0]), b.pb, gW, 10, "init")
    crit = (0.05, 2e-3, 5.0)
    st, it = pd.run_alg1_adaptive(st0.copy(), b.pb, gW, "polsara", 400, 10, *crit)
    assert 0 < it < 400 and it % 10 == 0
    ref = st0.copy()
    for k in range(it):
        prev = ref.S
        ref = pd.alg1_iteration(ref, b.pb, gW, "polsara")
        if (k + 1) % 10 == 0:
            met = pd.stop_criteria(b.pb, ref.S, prev, *crit)[0]
            assert met == (k + 1 == it), k
    assert np.array_equal(ref.S, st.S)
    _, it2 = pd.run_alg1_adaptive(st0.copy(), b.pb, gW, "polsara", 25, 10, 0.0, 0.0, 0.0)
    assert it2 == 25


def test_reweighting_is_the_log_penalty_majorizer(tiny_built):
    """The weights of eq. weights are those of the reweighting scheme the paper takes from
    Candes, Wakin & Boyd (2008): each weighted l1 problem minimises the linear majorizer of the
    log-sum penalty delta * sum log(delta + |x|) at the previous estimate, whose slope in |x| is
    delta / (delta + |x|).  Checked against a central difference of that penalty."""
    b = tiny_built
    S = np.random.default_rng(2).standard_normal((256, 4))
    c = np.abs(b.sara.adjoint(S))
    for delta in (0.05, 0.25, 2.0):
        W = pd.reweight(b.pb, S, delta)
        h = 1e-6 * (delta + c)
        slope = delta * (np.log(delta + c + h) - np.log(delta + c - h)) / (2 * h)
        assert np.max(np.abs(W - slope)) <= 1e-8
