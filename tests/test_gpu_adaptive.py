"""Adaptive stopping evaluated on the device: the stopping test of the paper's simulation
settings (residual within (1 + theta) epsilon, relative variation of every Stokes map, N_p)
run inside the captured graph after every check_every iterations, against the oracle's
run_alg1_adaptive / alg2_adaptive on the same inputs; batched members stop on their own."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_common import P, say, solver_for
from oracle import pd, problem
from paper_1801_02417_amd import workloads as wk

pytestmark = pytest.mark.gpu

CRIT = (5e-3, 1e-4, 0.5)        # the paper's theta and N_p bound, a looser relative variation
CHECK = 10


def _setup(prec, n=32, M=600, seed=3, levels=3):
    wl = wk.tiny(n=n, M=M, taps=8, levels=levels, seed=seed)
    b = problem.build(wl)
    s = solver_for(wl, n, 8, prec, levels=levels, gamma=b.gamma)
    s.set_data(b.pb.Y, b.pb.eps)
    s.opnorm(200, 1e-8)
    s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
    return wl, b, s


def _rel(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adaptive_stage_matches_oracle(prec):
    wl, b, s = _setup(prec)
    try:
        J = b.sara.J
        gW = b.gamma * np.ones((J, 4))
        s.solve(P.PSARA_NNLS_INIT, 30, report=False)
        st = pd.run_alg1(pd.State.zeros(wl.n * wl.n, J, wl.M), b.pb, gW, 30, "init")
        it, rep = s.solve_adaptive(P.PSARA_CONSTRAINED, 600, CHECK, CRIT)
        ref, it_ref = pd.run_alg1_adaptive(st, b.pb, gW, "polsara", 600, CHECK, *CRIT)
        say(f"[adaptive] {prec}: device stopped after {it}, oracle after {it_ref}; "
            f"residual/eps {rep['residual'] / rep['epsilon']:.6f}, N_p {rep['n_p']:.3f}")
        assert 0 < it < 600 and it % CHECK == 0
        assert rep["iterations"] == 30 + it
        assert rep["residual"] <= (1 + CRIT[0]) * rep["epsilon"] * (1 + 1e-9) and rep["n_p"] <= CRIT[2]
        if prec == "fp64":
            assert it == it_ref
            assert _rel(s.image(), ref.S) <= 1e-9
        else:
            # FP32 rounding may move the decision by one check; compare at the device's count
            assert abs(it - it_ref) <= CHECK
            if it != it_ref:
                ref = pd.run_alg1(st, b.pb, gW, it, "polsara")
            assert _rel(s.image(), ref.S) <= 1e-4
    finally:
        s.close()


def test_adaptive_cap_and_halt_cleared():
    """With a test that cannot pass, exactly max_iters iterations run (a short last block
    included), and the same state as a plain solve; afterwards plain solves iterate again."""
    wl, b, s = _setup("fp64", n=16, M=150, seed=7, levels=2)
    try:
        it, _ = s.solve_adaptive(P.PSARA_NNLS_INIT, 25, CHECK, (0.0, 0.0, -1.0))
        assert it == 25
        adaptive = s.image()
        s.reset()
        s.solve(P.PSARA_NNLS_INIT, 25, report=False)
        assert np.array_equal(adaptive, s.image())
        # a test that passes at once halts after the first block; the next plain solve moves
        it, _ = s.solve_adaptive(P.PSARA_NNLS_INIT, 100, CHECK, (1e9, 1e9, -1.0))
        assert it == CHECK
        before = s.image()
        s.solve(P.PSARA_NNLS_INIT, 3, report=False)
        assert not np.array_equal(before, s.image())
    finally:
        s.close()


def test_batch_adaptive_members_stop_alone():
    """Members of different sizes stop after different counts; each ends bitwise where its
    solo adaptive run ends, with the same count."""
    cases = [(16, 150, 7, 2), (32, 600, 3, 3), (64, 2500, 9, 4)]
    solo_it, solo_img = [], []
    for n, M, seed, L in cases:
        wl, b, s = _setup("fp32", n=n, M=M, seed=seed, levels=L)
        s.solve(P.PSARA_NNLS_INIT, 20, report=False)
        it, _ = s.solve_adaptive(P.PSARA_CONSTRAINED, 400, CHECK, CRIT)
        solo_it.append(it)
        solo_img.append(s.image())
        s.close()
    members = []
    for n, M, seed, L in cases:
        members.append(_setup("fp32", n=n, M=M, seed=seed, levels=L)[2])
    try:
        P.batch_solve(members, P.PSARA_NNLS_INIT, 20, report=False)
        its, reps = P.batch_solve_adaptive(members, P.PSARA_CONSTRAINED, 400, CHECK, CRIT)
        say(f"[adaptive] batch iterations {its}, solo {solo_it}")
        assert its == solo_it
        for s, img in zip(members, solo_img):
            assert np.array_equal(s.image(), img)
    finally:
        for s in members:
            s.close()


def test_reweighted_adaptive_matches_oracle():
    wl, b, s = _setup("fp64")
    try:
        crit = (5e-3, 5e-4, 0.5)          # every stage stops before the cap on this problem
        its, rep = s.reweighted_solve_adaptive(P.PSARA_CONSTRAINED, 2, 300, CHECK, crit)
        ref, _, its_ref = pd.alg2_adaptive(b.pb, b.gamma, 2, 300, CHECK, *crit)
        say(f"[adaptive] Algorithm 2 stages: device {its}, oracle {its_ref}")
        assert its == its_ref
        assert rep["iterations"] == sum(its)
        assert _rel(s.image(), ref.S) <= 1e-9
    finally:
        s.close()
