"""Batched solves: several independent problems advanced by one launch per pass.

* Batch invariance: every member of a batch of mixed sizes (image sides 16 to 512, different
  visibility counts and SARA depths, so the batch's FFT cells per workgroup, de-grid window
  and coarse-level split differ from the members' own) ends bit for bit where the same solve
  run alone ends, in FP32 and FP64, over the whole of Algorithm 2 (initialisation, two
  reweighted stages).
* A batched member against the FP64 oracle's Algorithm 2 on the same inputs.
* Argument checking of the batch entry points.
"""
from __future__ import annotations

import numpy as np
import pytest

from gpu_common import PREC, say
from oracle import pd, problem
from paper_1801_02417_amd import psara as P
from paper_1801_02417_amd import workloads as wk

pytestmark = pytest.mark.gpu

STAGES = [6, 4, 4]


def mixed_workloads():
    return [wk.tiny(n=16, M=150, taps=8, levels=2, seed=7),
            wk.tiny(n=32, M=700, taps=8, levels=3, seed=8),
            wk.tiny(n=64, M=3000, taps=8, levels=4, seed=9),
            wk.tiny(n=512, M=4000, taps=8, levels=4, seed=10)]


_BUILT = {}


def built(wl):
    if wl.name not in _BUILT:
        _BUILT[wl.name] = problem.build(wl, norm_rtol=1e-6, norm_max_iter=40)
    return _BUILT[wl.name]


def make_solver(wl, prec):
    b = built(wl)
    s = P.Solver(wl.n, wl.uv, taps=wl.taps, precision=PREC[prec])
    s.set_prior(wl.levels, b.gamma)
    s.set_data(b.pb.Y, b.pb.eps)
    s.opnorm(60, 1e-6)            # the library checks the step-size condition against its own norm
    s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
    return s


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_equals_alone_bitwise(prec):
    wls = mixed_workloads()
    alone, reps_alone = [], []
    for wl in wls:
        say(f"alone {wl.name} n={wl.n} M={wl.M} {prec}")
        s = make_solver(wl, prec)
        reps_alone.append(s.reweighted_solve(P.PSARA_CONSTRAINED, STAGES))
        alone.append(s.image())
        s.close()
    say(f"batch of {len(wls)} {prec}")
    members = [make_solver(wl, prec) for wl in wls]
    reps = P.batch_reweighted_solve(members, P.PSARA_CONSTRAINED, STAGES)
    for wl, s, a, ra, rb in zip(wls, members, alone, reps_alone, reps):
        img = s.image()
        diff = float(np.max(np.abs(img - a)))
        say(f"  {wl.name}: max |batch - alone| = {diff:.3e}, residual {rb['residual']:.6e} vs {ra['residual']:.6e}")
        assert np.array_equal(img, a), f"{wl.name}: batch result differs from the solo run ({diff})"
        assert rb["iterations"] == ra["iterations"] == sum(STAGES)
        assert rb["residual"] == ra["residual"]
        s.close()


def test_batch_member_matches_oracle():
    wl = wk.blobs32()
    b = problem.build(wl)
    stages = [20, 10, 10]
    ref, _, _ = pd.alg2(b.pb, b.gamma, stages, 2)
    other = wk.tiny(n=32, M=500, taps=6, levels=2, seed=3)
    members = [make_solver(other, "fp64")]
    s = P.Solver(wl.n, wl.uv, taps=wl.taps, precision=P.PSARA_FP64)
    s.set_prior(wl.levels, b.gamma)
    s.set_data(b.pb.Y, b.pb.eps)
    s.opnorm(300, 1e-9)
    s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
    members.insert(0, s)
    P.batch_reweighted_solve(members, P.PSARA_CONSTRAINED, stages)
    S = s.image()
    err = max(float(np.linalg.norm(S[:, i] - ref.S[:, i]) / np.linalg.norm(ref.S[:, i])) for i in range(4))
    say(f"batched member vs oracle: max per-Stokes rel err {err:.3e}")
    assert err <= 1e-9
    for m in members:
        m.close()


def test_batch_argument_checks():
    wl = wk.tiny(n=16, M=150, taps=8, levels=2, seed=7)
    a = make_solver(wl, "fp32")
    b = make_solver(wl, "fp64")
    with pytest.raises(P.PsaraError) as e:
        P.batch_solve([a, b], P.PSARA_CONSTRAINED, 2)
    assert e.value.status == P.PSARA_EINVAL
    with pytest.raises(P.PsaraError) as e:
        P.batch_solve([a, a], P.PSARA_CONSTRAINED, 2)
    assert e.value.status == P.PSARA_EINVAL
    c = P.Solver(wl.n, wl.uv, taps=6, precision=P.PSARA_FP32_MIXED)
    bb = built(wl)
    c.set_prior(wl.levels, bb.gamma)
    c.set_data(bb.pb.Y, bb.pb.eps)
    c.opnorm(60, 1e-6)
    c.set_steps(bb.pb.tau, bb.pb.rho1, bb.pb.rho2, bb.pb.rho3)
    with pytest.raises(P.PsaraError) as e:
        P.batch_solve([a, c], P.PSARA_CONSTRAINED, 2)
    assert e.value.status == P.PSARA_EINVAL
    d = P.Solver(wl.n, wl.uv, taps=8, precision=P.PSARA_FP32_MIXED)
    with pytest.raises(P.PsaraError) as e:
        P.batch_solve([a, d], P.PSARA_CONSTRAINED, 2)
    assert e.value.status == P.PSARA_ESTATE
    # a plain batched stage leaves both members advanced by the same count
    reps = P.batch_solve([a, make_solver(wk.tiny(n=32, M=300, taps=8, levels=2, seed=4), "fp32")],
                         P.PSARA_NNLS_INIT, 3)
    assert [r["iterations"] for r in reps] == [3, 3]
    for s in (a, b, c, d):
        s.close()


def test_batch_profile_passes_times_and_advances_like_alone():
    """psara_batch_profile_passes times every pass of a mixed batch (positive times, the fused
    row pass included) and advances each member by 2 * iters iterations, bitwise as the same
    number of iterations run alone."""
    wls = mixed_workloads()[:3]
    alone = []
    for wl in wls:
        s = make_solver(wl, "fp32")
        s.solve(P.PSARA_CONSTRAINED, 6, report=False)
        alone.append(s.state())
        s.close()
    members = [make_solver(wl, "fp32") for wl in wls]
    try:
        ms = P.psara_batch_profile_passes([s.ctx for s in members], P.PSARA_CONSTRAINED, 3)
        say(f"batch pass ms: {np.round(ms, 4)}")
        assert all(ms[i] > 0 for i in (0, 1, 4, 5, 6, 7, 8, 9)), ms
        assert ms[2] == 0 and ms[3] == 0
        for wl, s, a in zip(wls, members, alone):
            st = s.state()
            for name in ("S", "Z", "A", "B", "C", "D"):
                assert np.array_equal(st[name], a[name]), (wl.name, name)
    finally:
        for s in members:
            s.close()


def test_batch_member_with_mueller_matrices_equals_alone():
    """A member whose phi carries per-row Mueller matrices and one with the plain L, batched:
    each ends bit for bit where it ends alone."""
    wls = mixed_workloads()[1:3]
    Ds = [wk.station_mueller(np.random.default_rng(61), wls[0].M, leakage=0.2), None]

    def make(wl, D):
        b = built(wl)
        s = P.Solver(wl.n, wl.uv, taps=wl.taps, precision=PREC["fp32"])
        s.set_prior(wl.levels, b.gamma)
        if D is not None:
            s.set_mueller(D)
        s.set_data(b.pb.Y, b.pb.eps)
        s.opnorm(60, 1e-6)
        s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
        return s

    alone = []
    for wl, D in zip(wls, Ds):
        s = make(wl, D)
        s.reweighted_solve(P.PSARA_CONSTRAINED, STAGES)
        alone.append(s.image())
        s.close()
    members = [make(wl, D) for wl, D in zip(wls, Ds)]
    try:
        P.batch_reweighted_solve(members, P.PSARA_CONSTRAINED, STAGES)
        for s, a in zip(members, alone):
            assert np.array_equal(s.image(), a)
    finally:
        for s in members:
            s.close()
