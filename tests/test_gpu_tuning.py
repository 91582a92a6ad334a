"""Launch shapes and the autotuner: every tuning the autotuner may choose gives iterations that
match the oracle (from a random state, in FP64 and FP32, to the bars of the iteration tests);
changing the tuning keeps the state; the autotuner's choice on the 256x256 / 2e5-row workload
then runs the stored 300-iteration oracle solve's schedule to the same bar; a tuned batch is
bitwise equal to its members run alone with the same shapes; the per-class store."""
import os
import sys

import numpy as np
import pytest

from oracle import problem
from paper_1801_02417_amd import workloads as wk
from tests.gpu_common import P, say, solver_for
from tests.test_gpu_iteration import _compare, _oracle_steps, _random_state

pytestmark = pytest.mark.gpu

TUNINGS = [
    {"grid_chunk": 256},
    {"grid_chunk": 512, "degrid_item": 64},
    {"degrid_item": 1024},
    {"degrid_item": 128, "fft_cells": 2048},
    {"fft_cells": 1024, "analysis_wide": 0},
    {"analysis_wide": 2},
    {"analysis_wide": 3, "fft_cells": 1024},
]


def _dense(prec, n=64, M=6000, seed=21):
    """A 64x64 problem with a concentrated uv distribution, so the central gridding tiles hold
    more rows than the smallest chunk and the de-grid tiles more than the smallest item."""
    rng = np.random.default_rng(seed)
    wl = wk.tiny(n=n, M=M, taps=8, levels=3, seed=seed)
    wl.uv = np.clip(rng.normal(0.0, 0.25, size=(M, 2)), -np.pi, np.pi - 1e-9)
    b = problem.build(wl, norm_rtol=1e-7, norm_max_iter=200)
    W = rng.uniform(0.2, 1.0, size=(b.sara.J, 4))
    s = solver_for(wl, n, 8, prec, levels=3, gamma=b.gamma, weights=W)
    s.set_data(b.pb.Y, b.pb.eps)
    s.opnorm(100, 1e-8)
    s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
    return wl, b, s, b.gamma * W


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: "-".join(f"{k}{v}" for k, v in t.items()))
def test_iterations_under_tuning(tuning, prec, tol):
    wl, b, s, gW = _dense(prec)
    try:
        s.set_tuning(tuning)
        got = s.tuning()
        assert all(got[k] == v for k, v in tuning.items()), got
        rng = np.random.default_rng(5)
        st = _random_state(rng, wl.n * wl.n, b.sara.J, wl.M, gW)
        s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
        ref, scale = st.copy(), {}
        for k in (1, 4):
            s.solve(P.PSARA_CONSTRAINED, k, report=False)
            ref = _oracle_steps(ref, b.pb, gW, "polsara", k, scale)
            w = _compare(s.state(), ref, tol, f"{tuning} +{k}", scale if prec == "fp32" else None)
            say(f"[tuning] {tuning} {prec} +{k}: worst rel err {w:.2e}")
    finally:
        s.close()


@pytest.mark.parametrize("prec,n,per_basis", [("fp64", 64, 0), ("fp32", 64, 0), ("fp32", 256, 1)])
def test_all_bases_analysis_bitwise_equals_per_basis(prec, n, per_basis):
    """The all-bases bit (analysis_wide 2, 3) runs every basis of a level-1 tile in one workgroup
    over one staged image region; the tiles and every coefficient's arithmetic are those of the
    per-basis items of the same width (0: 8-wide; 1: 16-wide, which FP32 takes for the level-1
    bands of a 256-pixel image), so the iterations end bitwise equal."""
    out = {}
    for aw in (per_basis, per_basis | 2):
        wl, b, s, gW = _dense(prec, n=n)
        try:
            s.set_tuning({"analysis_wide": aw})
            rng = np.random.default_rng(8)
            st = _random_state(rng, wl.n * wl.n, b.sara.J, wl.M, gW)
            s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
            s.solve(P.PSARA_CONSTRAINED, 6, report=False)
            out[aw] = s.state()
        finally:
            s.close()
    a, c = out[per_basis], out[per_basis | 2]
    for k in a:
        assert np.array_equal(a[k], c[k]), k
    say(f"[tuning] analysis_wide {per_basis | 2} vs {per_basis} ({prec}, n={n}): bitwise equal after 6 iterations")


def test_batch_all_bases_analysis_equals_alone():
    stages = [12, 10, 10]
    shapes = {"analysis_wide": 2}
    members = [_batch_member(i, "fp32") for i in range(4)]
    try:
        for s in members:
            s.set_tuning(shapes)
        P.batch_reweighted_solve(members, P.PSARA_CONSTRAINED, stages)
        batched = [s.image() for s in members]
    finally:
        for s in members:
            s.close()
    for i, img in enumerate(batched):
        s = _batch_member(i, "fp32")
        try:
            s.set_tuning(shapes)
            s.reweighted_solve(P.PSARA_CONSTRAINED, stages)
            assert np.array_equal(s.image(), img), i
        finally:
            s.close()


def test_set_tuning_keeps_state_and_checks_ranges():
    wl, b, s, gW = _dense("fp32")
    try:
        s.solve(P.PSARA_NNLS_INIT, 5, report=False)
        before = s.state()
        s.set_tuning({"grid_chunk": 256, "degrid_item": 64, "fft_cells": 2048})
        after = s.state()
        for k in before:
            assert np.array_equal(before[k], after[k]), k
        for bad in ({"grid_chunk": 300}, {"degrid_item": 32}, {"degrid_item": 96}, {"analysis_wide": 4},
                    {"fft_cells": 4096}, {"fft_cells": 100}):
            with pytest.raises(P.PsaraError) as e:
                s.set_tuning(bad)
            assert e.value.status == P.PSARA_EINVAL
        s.set_tuning(None)
        assert s.tuning() == P.DEFAULT_TUNING
    finally:
        s.close()


def test_autotune_ring256_then_full_schedule_parity():
    """The autotuner on the benchmark's workload (FP32), then the 300-iteration schedule with the
    chosen shapes against the stored FP64 oracle solve."""
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_oracle_solves as mk
    wl = wk.ring256()
    g = np.load(mk.golden_path("ring256"), allow_pickle=False)
    assert str(g["oracle_hash"]) == mk.oracle_hash() and str(g["input_hash"]) == mk.input_hash(wl)
    b = problem.build(wl, phi_norm=float(g["phi_norm_sq"]), gamma=float(g["gamma"]))
    s = solver_for(wl, wl.n, wl.taps, "fp32", levels=wl.levels, gamma=float(g["gamma"]))
    try:
        s.set_data(b.pb.Y, b.pb.eps)
        s.opnorm(100, 1e-6)
        s.set_steps(*[float(v) for v in g["steps"]])
        chosen, ms = s.autotune(P.PSARA_CONSTRAINED)
        say(f"[autotune] ring256: chosen {chosen}; ms/iteration default {ms[0]:.4f}, chosen {ms[1]:.4f}")
        assert s.tuning() == chosen and ms[1] <= ms[0] and ms[1] > 0
        assert not np.any(s.image())            # the trials leave the (zero) state as it was
        rep = s.reweighted_solve(P.PSARA_CONSTRAINED, [int(v) for v in g["stages"]], 10.0)
        S, R = s.image(), g["S"]
        errs = [float(np.linalg.norm(S[:, i] - R[:, i]) / np.linalg.norm(R[:, i])) for i in range(4)]
        say(f"   tuned solve: per-Stokes rel err {['%.2e' % e for e in errs]}")
        assert max(errs) <= 1e-4
        assert rep["iterations"] == 300
    finally:
        s.close()


def _batch_member(i, prec):
    wl = wk.batch_request(i, sides=(64, 128), m_range=(3.0, 3.6))
    b = problem.build(wl, norm_rtol=1e-6, norm_max_iter=60)
    s = solver_for(wl, wl.n, wl.taps, prec, levels=wl.levels, gamma=b.gamma)
    s.set_data(b.pb.Y, b.pb.eps)
    s.opnorm(60, 1e-6)
    s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
    return s


def test_batch_autotune_then_batch_equals_alone():
    stages = [12, 10, 10]
    members = [_batch_member(i, "fp32") for i in range(4)]
    try:
        chosen, ms = P.batch_autotune(members, P.PSARA_CONSTRAINED)
        say(f"[autotune] batch of 4: chosen {chosen}; ms/iteration default {ms[0]:.4f}, chosen {ms[1]:.4f}")
        for s in members:
            assert s.tuning() == chosen
        P.batch_reweighted_solve(members, P.PSARA_CONSTRAINED, stages)
        batched = [s.image() for s in members]
    finally:
        for s in members:
            s.close()
    for i, img in enumerate(batched):
        s = _batch_member(i, "fp32")
        try:
            s.set_tuning(chosen)
            s.reweighted_solve(P.PSARA_CONSTRAINED, stages)
            assert np.array_equal(s.image(), img), i
        finally:
            s.close()


def test_tuning_store_and_cache():
    wl, b, s, gW = _dense("fp64", seed=33)
    wl2, b2, s2, _ = _dense("fp64", seed=34)      # the same shape class
    try:
        assert P.psara_tuning_lookup(wl.n, wl.M, 8, 3, P.ALL_BASES, P.PSARA_FP64) is None
        chosen, ms = s.autotune(P.PSARA_CONSTRAINED, P.PSARA_TUNE_STORE)
        assert ms[1] > 0
        assert P.psara_tuning_lookup(wl.n, wl.M, 8, 3, P.ALL_BASES, P.PSARA_FP64) == chosen
        got, ms2 = s2.autotune(P.PSARA_CONSTRAINED, P.PSARA_TUNE_USE_CACHE)
        assert got == chosen and ms2 == [0.0, 0.0] and s2.tuning() == chosen
    finally:
        s.close()
        s2.close()
