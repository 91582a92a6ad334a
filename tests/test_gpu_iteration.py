"""GPU parity of Algorithm 1 iterations: from the same random state (S, Z, A, B, C, D) the HIP
iteration and the oracle's alg1_iteration give the same next state, in every mode."""
import math

import numpy as np
import pytest

from oracle import pd, problem
from oracle.nufft import NUFFT, MeasurementOp
from oracle.sara import SARA, BASES
from paper_1801_02417_amd import workloads as wk
from tests.gpu_common import P, say, rel_err, solver_for, mask_of

pytestmark = pytest.mark.gpu

MODES = {"polsara": P.PSARA_CONSTRAINED, "init": P.PSARA_NNLS_INIT, "nocons": P.PSARA_UNCONSTRAINED}


def _random_state(rng, N, J, M, gW):
    S = rng.standard_normal((N, 4)) * 0.1
    Z = rng.standard_normal((N, 2)) * 0.1
    A = np.clip(rng.standard_normal((J, 4)) * 0.5, -gW, gW)
    B = (rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4))) * 0.01
    C = rng.standard_normal((N, 4)) * 0.1
    D = rng.standard_normal((N, 2)) * 0.1
    return pd.State(S, Z, A, B, C, D)


def _setup(n, M, T, L, prec, seed, bases=BASES):
    wl = wk.tiny(n=n, M=M, taps=T, levels=L, seed=seed)
    b = problem.build(wl, bases=bases)
    rng = np.random.default_rng(seed + 1)
    W = rng.uniform(0.2, 1.0, size=(b.sara.J, 4))
    s = solver_for(wl, n, T, prec, levels=L, bases=bases, gamma=b.gamma, weights=W)
    s.set_data(b.pb.Y, b.pb.eps)
    s.opnorm(200, 1e-8)
    s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
    return wl, b, s, b.gamma * W


def _oracle_steps(ref, pb, gW, mode, k, scale):
    """k oracle iterations; `scale` collects, per variable, the largest magnitude of its value
    before the projection / clipping (A~, B~, C~, D~, S - tau grad), which bounds the absolute
    rounding error an FP32 evaluation can make."""
    for _ in range(k):
        new = pd.alg1_iteration(ref, pb, gW, mode)
        X = 2 * new.S - ref.S
        pre = {"S": np.max(np.abs(ref.S)) + np.max(np.abs(new.S - ref.S)),
               "Z": np.max(np.abs(ref.Z)) + pb.tau * np.max(np.abs(ref.D)),
               "A": np.max(np.abs(ref.A + pb.rho1 * pb.psi_adj(X))),
               "B": np.max(np.abs(ref.B + pb.rho2 * pb.phi(X))),
               "C": np.max(np.abs(ref.C + pb.rho3 * X)),
               "D": np.max(np.abs(ref.D)) + 2 * pb.rho3 * np.max(np.abs(new.Z - ref.Z)) + np.max(np.abs(new.Z))}
        for name, v in pre.items():
            scale[name] = max(scale.get(name, 0.0), float(v), float(np.max(np.abs(getattr(new, name)))))
        ref = new
    return ref


def _compare(st_gpu, st_ref, tol, label, scale=None):
    """Max error of every variable relative to its largest magnitude (FP64) or to its
    pre-projection scale (FP32)."""
    worst = 0.0
    for name in ("S", "Z", "A", "B", "C", "D"):
        ref = getattr(st_ref, name)
        den = scale[name] if scale is not None else np.max(np.abs(ref))
        if den == 0:
            assert np.max(np.abs(st_gpu[name])) <= tol, (label, name)
            continue
        e = float(np.max(np.abs(st_gpu[name] - ref)) / den)
        worst = max(worst, e)
        assert e <= tol, (label, name, e)
    return worst


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
@pytest.mark.parametrize("case", [(16, 150, 6, 2), (32, 600, 8, 3)], ids=lambda c: "n%d" % c[0])
def test_iterations_from_random_state(case, mode, prec, tol):
    n, M, T, L = case
    say(f"[iter] n={n} mode={mode} prec={prec}")
    wl, b, s, gW = _setup(n, M, T, L, prec, seed=3 + n)
    try:
        rng = np.random.default_rng(77 + n)
        st = _random_state(rng, n * n, b.sara.J, M, gW)
        if mode == "init":
            st.Z[:] = 0; st.A[:] = 0; st.C[:] = 0; st.D[:] = 0
        if mode == "nocons":
            st.Z[:] = 0; st.C[:] = 0; st.D[:] = 0
        s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
        ref = st.copy()
        scale = {}
        for k in (1, 4):
            s.solve(MODES[mode], k, report=False)
            ref = _oracle_steps(ref, b.pb, gW, mode, k, scale)
            w = _compare(s.state(), ref, tol, f"{mode} after +{k}", scale if prec == "fp32" else None)
            say(f"   +{k} iterations: worst rel err {w:.2e}")
    finally:
        s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
def test_iterations_dirac_only_and_wavelets_only(prec, tol):
    for bases in (("dirac",), ("db2", "db5", "db8")):
        wl, b, s, gW = _setup(16, 120, 6, 2, prec, seed=11, bases=bases)
        try:
            rng = np.random.default_rng(5)
            st = _random_state(rng, 256, b.sara.J, wl.M, gW)
            s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
            s.solve(P.PSARA_CONSTRAINED, 3, report=False)
            scale = {}
            ref = _oracle_steps(st, b.pb, gW, "polsara", 3, scale)
            _compare(s.state(), ref, tol, str(bases), scale if prec == "fp32" else None)
        finally:
            s.close()


def _run_and_compare(s, b, gW, wl, rng, tol, prec, label):
    st = _random_state(rng, wl.n * wl.n, b.sara.J, wl.M, gW)
    s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
    s.solve(P.PSARA_CONSTRAINED, 3, report=False)
    scale = {}
    ref = _oracle_steps(st, b.pb, gW, "polsara", 3, scale)
    return _compare(s.state(), ref, tol, label, scale if prec == "fp32" else None)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
def test_iterations_one_wavelet_and_prior_change(prec, tol):
    """A single wavelet basis, with and without the Dirac basis (each tile's last-level synthesis
    is one work item and the second partial image of Psi A stays zero); then, on one solver, a
    prior of all nine bases (whose iterations fill both partial images) replaced by a single
    basis: the new state's upload has to clear the second image."""
    for bases in (("db3",), ("dirac", "db7")):
        wl, b, s, gW = _setup(16, 120, 6, 2, prec, seed=12, bases=bases)
        try:
            _run_and_compare(s, b, gW, wl, np.random.default_rng(6), tol, prec, str(bases))
        finally:
            s.close()
    wl, b, s, gW = _setup(16, 120, 6, 2, prec, seed=13)
    try:
        rng = np.random.default_rng(9)
        _run_and_compare(s, b, gW, wl, rng, tol, prec, "all bases")
        b2 = problem.build(wl, bases=("db3",))
        W2 = rng.uniform(0.2, 1.0, size=(b2.sara.J, 4))
        s.set_prior(2, b2.gamma, mask_of(("db3",)), W2)
        s.set_data(b2.pb.Y, b2.pb.eps)
        s.set_steps(b2.pb.tau, b2.pb.rho1, b2.pb.rho2, b2.pb.rho3)
        w = _run_and_compare(s, b2, b2.gamma * W2, wl, rng, tol, prec, "after the prior change")
        say(f"[iter] prior of nine bases replaced by db3, {prec}: worst rel err {w:.2e}")
    finally:
        s.close()


def test_state_roundtrip_and_reset():
    wl, b, s, gW = _setup(16, 100, 6, 2, "fp64", seed=21)
    try:
        rng = np.random.default_rng(1)
        st = _random_state(rng, 256, b.sara.J, wl.M, gW)
        s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
        got = s.state()
        for name in ("S", "Z", "A", "B", "C", "D"):
            assert np.array_equal(got[name], getattr(st, name)), name
        s.reset()
        got = s.state()
        for name in ("S", "Z", "A", "B", "C", "D"):
            assert not np.any(got[name]), name
    finally:
        s.close()


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
def test_fused_row_pass_chain(mode, prec, tol):
    """Nine iterations in one call run as a captured chain of eight (the inverse row FFT of each
    iteration fused with the next primal step and row FFT, seven fused launches) plus one; the
    state is bitwise the one of nine one-iteration calls (separate passes), and matches the
    oracle's nine iterations."""
    n, M, T, L = 32, 600, 8, 3
    say(f"[fused] n={n} mode={mode} prec={prec}")
    wl, b, s, gW = _setup(n, M, T, L, prec, seed=41)
    try:
        rng = np.random.default_rng(43)
        st = _random_state(rng, n * n, b.sara.J, M, gW)
        if mode == "init":
            st.Z[:] = 0; st.A[:] = 0; st.C[:] = 0; st.D[:] = 0
        if mode == "nocons":
            st.Z[:] = 0; st.C[:] = 0; st.D[:] = 0
        s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
        s.solve(MODES[mode], 9, report=False)
        chained = s.state()
        s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
        for _ in range(9):
            s.solve(MODES[mode], 1, report=False)
        single = s.state()
        for name in ("S", "Z", "A", "B", "C", "D"):
            assert np.array_equal(chained[name], single[name]), name
        scale = {}
        ref = _oracle_steps(st.copy(), b.pb, gW, mode, 9, scale)
        w = _compare(chained, ref, tol * 4, f"{mode} fused chain", scale if prec == "fp32" else None)
        say(f"   9 iterations: worst rel err {w:.2e}")
    finally:
        s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
def test_iterations_with_mueller_matrices(prec, tol):
    """Algorithm 1 with known direction-independent Mueller matrices in phi (every row mixed by
    its own L D_m^T): nine iterations from a random state (one captured chain plus one) against
    the oracle run with the same matrices."""
    n, M, T, L = 32, 600, 8, 3
    wl = wk.tiny(n=n, M=M, taps=T, levels=L, seed=52)
    D = wk.station_mueller(np.random.default_rng(53), M, leakage=0.2)
    b = problem.build(wl, mueller=D)
    rng = np.random.default_rng(54)
    W = rng.uniform(0.2, 1.0, size=(b.sara.J, 4))
    s = solver_for(wl, n, T, prec, levels=L, gamma=b.gamma, weights=W)
    try:
        s.set_mueller(D)
        s.set_data(b.pb.Y, b.pb.eps)
        s.opnorm(200, 1e-8)
        s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
        gW = b.gamma * W
        st = _random_state(rng, n * n, b.sara.J, M, gW)
        s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
        s.solve(P.PSARA_CONSTRAINED, 9, report=False)
        scale = {}
        ref = _oracle_steps(st.copy(), b.pb, gW, "polsara", 9, scale)
        w = _compare(s.state(), ref, tol * 4, "mueller", scale if prec == "fp32" else None)
        say(f"[mueller] {prec} 9 iterations: worst rel err {w:.2e}")
    finally:
        s.close()


def test_max_image_side():
    """The largest image side the boundary accepts (1024: a 2048^2 grid, 2048-point FFT lines,
    every wavelet level on the tiled kernels): one constrained iteration from a random state against
    the oracle, in FP64 and FP32.  Three bases and two levels keep the oracle's share to well under
    a minute; its step sizes come from its own five-step power iteration, inflated by 1.5 so that
    they bound ||phi||^2 from above (the device checks the step condition with its own norm)."""
    n, M, T, L = 1024, 20000, 8, 2
    bases = ("dirac", "db1", "db4")
    say(f"[iter] n={n} M={M}: oracle set-up")
    wl = wk.tiny(n=n, M=M, taps=T, levels=L, seed=91)
    est, _ = pd.phi_norm_sq(MeasurementOp(NUFFT(wl.uv, n, 2, T)), n * n, max_iter=5, rtol=0.0)
    b = problem.build(wl, bases=bases, phi_norm=1.5 * est)
    rng = np.random.default_rng(92)
    W = rng.uniform(0.2, 1.0, size=(b.sara.J, 4))
    gW = b.gamma * W
    st = _random_state(rng, n * n, b.sara.J, M, gW)
    scale = {}
    ref = _oracle_steps(st.copy(), b.pb, gW, "polsara", 1, scale)
    for prec, tol in (("fp64", 1e-9), ("fp32", 5e-6)):
        say(f"[iter] n={n} {prec}")
        s = solver_for(wl, n, T, prec, levels=L, bases=bases, gamma=b.gamma, weights=W)
        try:
            s.set_data(b.pb.Y, b.pb.eps)
            s.opnorm(100, 1e-6)
            s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
            s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
            s.solve(P.PSARA_CONSTRAINED, 1, report=False)
            w = _compare(s.state(), ref, tol, f"n={n} {prec}", scale if prec == "fp32" else None)
            say(f"   n={n} {prec}: worst rel err {w:.2e}")
        finally:
            s.close()


def test_served_large_request_one_iteration():
    """The served mix's large request at its full size (512^2 per Stokes map, 1e6 visibility rows,
    8x8 taps, all nine bases at four levels, the launch shapes the large-solve benchmark runs):
    one constrained iteration from a random state against the oracle, in FP64 and FP32.  The
    oracle's step sizes come from its own five-step power iteration, inflated by 1.5 so that
    they bound ||phi||^2 from above; its share is about 40 s."""
    wl = wk.batch_request(0, sides=(512,))
    n, M, T, L = wl.n, wl.M, wl.taps, wl.levels
    assert (n, M, T, L) == (512, 1_000_000, 8, 4)
    say(f"[iter] n={n} M={M}: oracle set-up")
    est, _ = pd.phi_norm_sq(MeasurementOp(NUFFT(wl.uv, n, 2, T)), n * n, max_iter=5, rtol=0.0)
    b = problem.build(wl, phi_norm=1.5 * est)
    rng = np.random.default_rng(93)
    W = rng.uniform(0.2, 1.0, size=(b.sara.J, 4))
    gW = b.gamma * W
    st = _random_state(rng, n * n, b.sara.J, M, gW)
    scale = {}
    ref = _oracle_steps(st.copy(), b.pb, gW, "polsara", 1, scale)
    for prec, tol in (("fp64", 1e-9), ("fp32", 5e-6)):
        say(f"[iter] n={n} M={M} {prec}")
        s = solver_for(wl, n, T, prec, levels=L, gamma=b.gamma, weights=W)
        try:
            s.set_data(b.pb.Y, b.pb.eps)
            s.opnorm(100, 1e-6)
            s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
            s.set_state(st.S, st.Z, st.A, st.B, st.C, st.D)
            s.solve(P.PSARA_CONSTRAINED, 1, report=False)
            w = _compare(s.state(), ref, tol, f"n={n} M={M} {prec}", scale if prec == "fp32" else None)
            say(f"   n={n} M={M} {prec}: worst rel err {w:.2e}")
        finally:
            s.close()
