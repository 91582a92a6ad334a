"""GPU parity on the stated full schedules against stored FP64 oracle solves (written by
tests/golden/make_oracle_solves.py, which calls only the oracle; the oracle takes minutes on
these sizes):

* the 128x128 ring + jet workload on its full schedule, 2000 iterations = initialisation and 5
  reweighting cycles (333 x 5 + 335), in FP64 and in FP32 with FP64 reductions;
* the 256x256, 2e5-row workload the benchmark times, 300 iterations = 100 x (initialisation +
  2 cycles), FP32 with FP64 reductions;

each with the per-Stokes relative image error, the SNR difference (log10, Sec. 4.7), and the
reported stopping quantities (residual, relative variation of the last iteration per Stokes map,
zeta, N_p, objective) compared element by element with the oracle's."""
import os
import sys

import numpy as np
import pytest

from oracle import metrics, problem
from paper_1801_02417_amd import workloads as wk
from tests.gpu_common import P, say, solver_for

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
sys.path.insert(0, GOLDEN)
import make_oracle_solves as mk  # noqa: E402


def _golden(name, wl):
    g = np.load(mk.golden_path(name), allow_pickle=False)
    assert str(g["oracle_hash"]) == mk.oracle_hash(), "stored oracle solve is stale: rerun make_oracle_solves.py"
    assert str(g["input_hash"]) == mk.input_hash(wl), "the workload generator changed: rerun make_oracle_solves.py"
    return g


def _gpu_solve(wl, g, prec):
    b = problem.build(wl, phi_norm=float(g["phi_norm_sq"]), gamma=float(g["gamma"]))
    assert abs(b.pb.eps - float(g["eps"])) <= 1e-12 * b.pb.eps      # the same data as the oracle's run
    s = solver_for(wl, wl.n, wl.taps, prec, levels=wl.levels, gamma=float(g["gamma"]))
    s.set_data(b.pb.Y, b.pb.eps)
    s.opnorm(300, 1e-9)
    s.set_steps(*[float(v) for v in g["steps"]])
    rep = s.reweighted_solve(P.PSARA_CONSTRAINED, [int(v) for v in g["stages"]], 10.0)
    return s, rep, b


def _compare(name, wl, g, s, rep, b, prec, tol):
    S, R = s.image(), g["S"]
    errs = [float(np.linalg.norm(S[:, i] - R[:, i]) / np.linalg.norm(R[:, i])) for i in range(4)]
    snr_g = [metrics.snr_db(S[:, i], b.truth[:, i]) for i in range(4)]
    snr_o = [float(v) for v in g["snr_db"]]
    dsnr = [a - o for a, o in zip(snr_g, snr_o)]
    say(f"[{name} {prec}] per-Stokes rel err {['%.2e' % e for e in errs]}; SNR gpu {['%.3f' % v for v in snr_g]} "
        f"oracle {['%.3f' % v for v in snr_o]} (diff {['%.1e' % v for v in dsnr]} dB)")
    say(f"   report {rep}")
    say(f"   oracle residual {float(g['residual'])} rel_var {list(g['rel_var'])} zeta {float(g['zeta'])} "
        f"n_p {float(g['n_p'])} objective {float(g['objective'])}")
    assert max(errs) <= tol
    assert rep["iterations"] == int(np.sum(g["stages"]))
    q = 1e-9 if prec == "fp64" else 1e-4
    assert abs(rep["residual"] - float(g["residual"])) <= q * float(g["residual"])
    assert abs(rep["objective"] - float(g["objective"])) <= q * float(g["objective"])
    assert abs(rep["zeta"] - float(g["zeta"])) <= q * float(g["zeta"])
    if prec == "fp64":
        assert rep["n_p"] == float(g["n_p"])
        # the relative variation of the last iteration, ||S^k - S^(k-1)|| / ||S^(k-1)|| per map:
        # a difference of nearly equal iterates, so it carries the images' absolute error divided
        # by the step size
        for a, o in zip(rep["rel_var"], g["rel_var"]):
            assert abs(a - float(o)) <= 1e-6 * float(o) + 1e-11, (a, float(o))
    else:
        for a, o in zip(rep["rel_var"], g["rel_var"]):
            assert abs(a - float(o)) <= 0.5 * float(o) + 1e-6, (a, float(o))
    return max(abs(v) for v in dsnr)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_ring128_full_schedule(prec, tol):
    wl = wk.ring128()
    g = _golden("ring128", wl)
    say(f"[full] ring128 {prec} stages {list(g['stages'])}")
    s, rep, b = _gpu_solve(wl, g, prec)
    try:
        d = _compare("ring128", wl, g, s, rep, b, prec, tol)
        assert d <= (1e-6 if prec == "fp64" else 1e-2)
    finally:
        s.close()


def test_ring256_300_iterations_fp32():
    wl = wk.ring256()
    g = _golden("ring256", wl)
    say(f"[full] ring256 fp32 stages {list(g['stages'])}")
    s, rep, b = _gpu_solve(wl, g, "fp32")
    try:
        d = _compare("ring256", wl, g, s, rep, b, "fp32", 1e-4)
        assert d <= 1e-2
    finally:
        s.close()
