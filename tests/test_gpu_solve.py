"""GPU parity of whole solves (Algorithm 2: initialisation, reweighting, warm starts) and of
the stopping quantities against the oracle, on the synthetic workloads."""
import math

import numpy as np
import pytest

from oracle import metrics, pd, problem
from paper_1801_02417_amd import workloads as wk
from tests.gpu_common import P, say, rel_err, solver_for

pytestmark = pytest.mark.gpu


def _gpu_alg2(wl, b, prec, stages, phi_norm=None, mode=P.PSARA_CONSTRAINED):
    s = solver_for(wl, wl.n, wl.taps, prec, levels=wl.levels, gamma=b.gamma)
    s.set_data(b.pb.Y, b.pb.eps)
    s.opnorm(300, 1e-9)
    s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
    rep = s.reweighted_solve(mode, stages, 10.0)
    return s, rep


def _oracle_alg2(b, stages):
    return pd.alg2(b.pb, b.gamma, stages, len(stages) - 1)


def _per_stokes(S, R):
    return [float(np.linalg.norm(S[:, i] - R[:, i]) / np.linalg.norm(R[:, i])) for i in range(4)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_blobs32_full_solve(prec, tol):
    """Blob workload: 32x32, 600 uv, KB 6, 3 levels, 300 iterations = init + 2 reweighting cycles."""
    wl = wk.blobs32()
    b = problem.build(wl)
    stages = pd.split_iterations(wl.iters, wl.cycles + 1)
    say(f"[solve] blobs32 {prec} stages={stages}")
    st, gW, deltas = _oracle_alg2(b, stages)
    s, rep = _gpu_alg2(wl, b, prec, stages)
    try:
        S = s.image()
        errs = _per_stokes(S, st.S)
        snr_g = [metrics.snr_db(S[:, i], b.truth[:, i]) for i in range(4)]
        snr_o = [metrics.snr_db(st.S[:, i], b.truth[:, i]) for i in range(4)]
        say(f"   per-Stokes rel err {['%.2e' % e for e in errs]}")
        say(f"   SNR gpu {['%.3f' % v for v in snr_g]} oracle {['%.3f' % v for v in snr_o]}")
        assert max(errs) <= tol
        assert max(abs(x - y) for x, y in zip(snr_g, snr_o)) <= (1e-6 if prec == "fp64" else 1e-2)
        # stopping quantities
        res = metrics.residual_norm(b.mop, st.S, b.pb.Y)
        assert abs(rep["residual"] - res) <= (1e-9 if prec == "fp64" else 1e-4) * res
        assert rep["iterations"] == wl.iters
        obj = metrics.weighted_l1(b.sara.adjoint, st.S, gW / b.gamma)
        assert abs(rep["objective"] - obj) <= (1e-9 if prec == "fp64" else 1e-4) * obj
    finally:
        s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_blobs32_unconstrained_solve_and_np(prec, tol):
    """Polarized SARA without the polarization constraint (Sec. 4.2: U', no epigraph terms)
    on the 32x32 blob workload against the oracle's "nocons" run, and the polarization-error share N_p of
    both estimates: the constrained solve's N_p is no larger than the unconstrained one's."""
    wl = wk.blobs32()
    b = problem.build(wl)
    stages = pd.split_iterations(wl.iters, wl.cycles + 1)
    st, _, _ = pd.alg2(b.pb, b.gamma, stages, len(stages) - 1, mode="nocons")
    st_c, _, _ = _oracle_alg2(b, stages)
    s, rep = _gpu_alg2(wl, b, prec, stages, mode=P.PSARA_UNCONSTRAINED)
    try:
        errs = _per_stokes(s.image(), st.S)
        _, _, np_u = metrics.polarization_error(b.mop, st.S, b.pb.Y)
        _, _, np_c = metrics.polarization_error(b.mop, st_c.S, b.pb.Y)
        say(f"[solve] blobs32 unconstrained {prec}: per-Stokes rel err {['%.2e' % e for e in errs]}; "
            f"N_p gpu {rep['n_p']:.3f}% oracle {np_u:.3f}% (constrained oracle {np_c:.3f}%)")
        assert max(errs) <= tol
        if prec == "fp64":
            assert abs(rep["n_p"] - np_u) <= 1e-9
        assert np_c <= np_u
    finally:
        s.close()


def test_report_matches_oracle_metrics():
    """Every reported stopping quantity against the oracle's on its own final state: residual,
    zeta, N_p, epsilon, and the relative variation of the last iteration per Stokes map."""
    wl = wk.blobs32()
    b = problem.build(wl)
    stages = [60, 60]
    # the oracle's run one iteration short, then that iteration: the last two iterates
    st, gW, _ = _oracle_alg2(b, [60, 59])
    prev = st.S.copy()
    st = pd.alg1_iteration(st, b.pb, gW, "polsara")
    s, rep = _gpu_alg2(wl, b, "fp64", stages)
    try:
        res = metrics.residual_norm(b.mop, st.S, b.pb.Y)
        p, zeta, n_p = metrics.polarization_error(b.mop, st.S, b.pb.Y)
        rv = metrics.relative_variation(st.S, prev)
        say(f"[report] gpu {rep}")
        say(f"         oracle residual {res} zeta {zeta} n_p {n_p} rel_var {list(rv)}")
        assert abs(rep["residual"] - res) <= 1e-9 * res
        assert abs(rep["zeta"] - zeta) <= 1e-9 * zeta
        assert abs(rep["n_p"] - n_p) <= 1e-9
        assert abs(rep["epsilon"] - b.pb.eps) <= 1e-15 * b.pb.eps
        # a difference of nearly equal iterates: the images' 1e-12 agreement over the step size
        for a, o in zip(rep["rel_var"], rv):
            assert abs(a - o) <= 1e-6 * o + 1e-11, (a, o)
    finally:
        s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_near_cone_unconstrained_np_matches_oracle(prec):
    """A workload whose unconstrained estimate leaves the polarization cone (fraction 0.97, sparse
    arcs; the oracle's N_p is about a third of the pixels): the GPU's unconstrained solve and its
    reported N_p and zeta against the oracle's "nocons" run, and the constrained solve's N_p = 0."""
    wl = wk.near_cone()
    b = problem.build(wl)
    stages = pd.split_iterations(wl.iters, wl.cycles + 1)
    st, _, _ = pd.alg2(b.pb, b.gamma, stages, len(stages) - 1, mode="nocons")
    _, zeta, n_p = metrics.polarization_error(b.mop, st.S, b.pb.Y)
    assert n_p > 10.0
    s, rep = _gpu_alg2(wl, b, prec, stages, mode=P.PSARA_UNCONSTRAINED)
    try:
        errs = _per_stokes(s.image(), st.S)
        say(f"[solve] near_cone32 unconstrained {prec}: per-Stokes rel err {['%.2e' % e for e in errs]}; "
            f"N_p gpu {rep['n_p']:.4f}% oracle {n_p:.4f}%; zeta gpu {rep['zeta']:.6e} oracle {zeta:.6e}")
        assert max(errs) <= (1e-9 if prec == "fp64" else 1e-4)
        if prec == "fp64":
            assert rep["n_p"] == n_p
            assert abs(rep["zeta"] - zeta) <= 1e-9 * zeta
        else:
            # pixels within the FP32 image error of zeta may fall either side
            assert abs(rep["n_p"] - n_p) <= 1.0
            assert abs(rep["zeta"] - zeta) <= 1e-4 * zeta
    finally:
        s.close()
    s, rep = _gpu_alg2(wl, b, prec, stages, mode=P.PSARA_CONSTRAINED)
    try:
        say(f"   constrained: N_p gpu {rep['n_p']:.4f}%")
        assert rep["n_p"] <= 0.5
    finally:
        s.close()


def test_ring128_reduced_schedule_fp32():
    """Ring workload (128x128 ring+jet, 8-station arcs, KB 8, 4 levels) with a 6-stage schedule of 40
    iterations each (the stated 2000-iteration budget is split the same way in the bench)."""
    wl = wk.ring128()
    b = problem.build(wl)
    stages = [40] * 6
    say(f"[solve] ring128 fp32 stages={stages}")
    st, gW, _ = pd.alg2(b.pb, b.gamma, stages, 5)
    s, rep = _gpu_alg2(wl, b, "fp32", stages)
    try:
        errs = _per_stokes(s.image(), st.S)
        say(f"   per-Stokes rel err {['%.2e' % e for e in errs]}")
        assert max(errs) <= 1e-4
    finally:
        s.close()


def test_ring256_full_size_fp32():
    """Ring workload at 256x256 (2e5 uv, KB 8, 4 levels): the launch configuration the benchmark times,
    with a short 3-stage schedule the oracle finishes in about half a minute."""
    wl = wk.ring256()
    # a loose power iteration suffices for the step sizes (tau keeps a 1% margin)
    b = problem.build(wl, norm_rtol=1e-5, norm_max_iter=60)
    stages = [10, 10, 10]
    say(f"[solve] ring256 fp32 stages={stages}")
    st, gW, _ = pd.alg2(b.pb, b.gamma, stages, 2)
    s, rep = _gpu_alg2(wl, b, "fp32", stages)
    try:
        errs = _per_stokes(s.image(), st.S)
        say(f"   per-Stokes rel err {['%.2e' % e for e in errs]}")
        assert max(errs) <= 1e-4
    finally:
        s.close()
