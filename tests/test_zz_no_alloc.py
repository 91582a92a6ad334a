"""psara_solve_noalloc (the allocation-free variant of psara_solve, scratch in the library's
static device array) against psara_solve on the same problems: bit for bit the same state, on
two calls in a row of which the second has a smaller input, in both precisions; and a problem
whose scratch exceeds the array is rejected with PSARA_EINVAL."""
import numpy as np
import pytest

from oracle import problem
from paper_1801_02417_amd import workloads as wk
from tests.gpu_common import P, PREC, say, solver_for

pytestmark = pytest.mark.gpu


def _ready(wl, b, prec):
    s = solver_for(wl, wl.n, wl.taps, prec, levels=wl.levels, gamma=b.gamma)
    s.set_data(b.pb.Y, b.pb.eps)
    s.opnorm(100, 1e-8)
    s.set_steps()
    return s


def _run(s, noalloc):
    # the initialisation stage, a reweighting, then constrained iterations (every pass runs)
    solve = (lambda m, k: P.psara_solve_noalloc(s.ctx, m, k)) if noalloc else (lambda m, k: s.solve(m, k, report=False))
    solve(P.PSARA_NNLS_INIT, 20)
    P.psara_reweight(s.ctx, P.psara_coef_std(s.ctx))
    solve(P.PSARA_CONSTRAINED, 37)
    s.synchronize()
    return s.image(), s.state()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_solve_equals_solve(prec):
    for wl in (wk.ring128(), wk.blobs32()):        # the second call has the smaller input
        b = problem.build(wl, norm_rtol=1e-6, norm_max_iter=100)
        say(f"[noalloc] {wl.name} {prec}: n={wl.n} M={wl.M}")
        ref, na = _ready(wl, b, prec), _ready(wl, b, prec)
        try:
            img_r, st_r = _run(ref, False)
            img_n, st_n = _run(na, True)
            assert np.array_equal(img_r, img_n), np.max(np.abs(img_r - img_n))
            for k in st_r:
                assert np.array_equal(st_r[k], st_n[k]), k
            rep_r, rep_n = ref.report(), na.report()
            assert rep_r["iterations"] == rep_n["iterations"] == 57
            assert rep_r["residual"] == rep_n["residual"]
            # the context's own buffers are back in use: a graph-replayed solve after the call
            # continues identically on both
            ref.solve(P.PSARA_CONSTRAINED, 5, report=False)
            na.solve(P.PSARA_CONSTRAINED, 5, report=False)
            assert np.array_equal(ref.image(), na.image())
        finally:
            ref.close()
            na.close()


def test_noalloc_rejects_oversized_scratch():
    rng = np.random.default_rng(3)
    n, M = 512, 200000
    uv = wk.gaussian_uv(rng, M, sigma=1.2)
    s = solver_for(uv, n, 8, "fp64", levels=2, gamma=1.0)
    try:
        Y = (rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4)))
        s.set_data(Y, 1.0)
        s.opnorm(3, 1e-2)
        s.set_steps()
        with pytest.raises(P.PsaraError) as e:
            P.psara_solve_noalloc(s.ctx, P.PSARA_NNLS_INIT, 1)
        assert e.value.status == P.PSARA_EINVAL and "scratch" in str(e.value)
        say(f"[noalloc] rejected: {e.value}")
    finally:
        s.close()
