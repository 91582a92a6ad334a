"""Pins of the oracle's SARA dictionary (Sec. 3.1): filters, DWT, tight frame."""
import json
import math
import os

import numpy as np
import pytest

from oracle.sara import SARA, daubechies_lowpass, highpass, dwt2, idwt2, analysis_1d, filterbank_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _eval(expr):
    return eval(expr, {"sqrt": math.sqrt})


def test_closed_form_filters():
    with open(os.path.join(GOLDEN, "daubechies_closed_forms.json")) as f:
        ref = json.load(f)
    for name in ("db1", "db2", "db3"):
        h = daubechies_lowpass(int(name[2:]))
        want = np.array([_eval(e) for e in ref[name]])
        assert np.max(np.abs(h - want)) < 1e-14, name


@pytest.mark.parametrize("p", range(1, 9))
def test_filter_identities(p):
    h = daubechies_lowpass(p)
    F = len(h)
    assert F == 2 * p
    assert abs(h.sum() - math.sqrt(2)) < 1e-14
    assert abs((h * h).sum() - 1) < 1e-14
    for m in range(1, p):
        assert abs(np.dot(h[:F - 2 * m], h[2 * m:])) < 1e-14
    # p vanishing moments of the high-pass filter (scaled by j^q growth)
    g = highpass(h)
    j = np.arange(F, dtype=float)
    for q in range(p):
        assert abs(np.sum(g * j ** q)) < 1e-13 * max(1.0, (F - 1) ** q)
    # quadrature-mirror orthogonality between low and high pass at even shifts
    for m in range(-p + 1, p):
        s = sum(h[i] * g[i + 2 * m] for i in range(F) if 0 <= i + 2 * m < F)
        assert abs(s) < 1e-14


@pytest.mark.parametrize("m,p", [(16, 2), (8, 8), (4, 8), (2, 5)])
def test_filterbank_matrix_orthogonal_even_when_filter_wraps(m, p):
    W = filterbank_matrix(m, tuple(daubechies_lowpass(p)))
    assert np.max(np.abs(W @ W.T - np.eye(m))) < 1e-14


def test_filterbank_matrix_matches_definition():
    """a_k = sum_j h[j] x[(2k+j) mod m] written as a loop."""
    rng = np.random.default_rng(0)
    h = daubechies_lowpass(4)
    g = highpass(h)
    for m in (4, 16):
        x = rng.standard_normal(m)
        a, d = analysis_1d(x, h, 0)
        for k in range(m // 2):
            assert abs(a[k] - sum(h[j] * x[(2 * k + j) % m] for j in range(8))) < 1e-14
            assert abs(d[k] - sum(g[j] * x[(2 * k + j) % m] for j in range(8))) < 1e-14


def test_haar_dwt_by_hand():
    x = np.array([[1.0, 3.0], [5.0, 9.0]])
    c = dwt2(x, daubechies_lowpass(1), 1)
    s = 1 / math.sqrt(2)
    rows = np.array([[(1 + 3) * s, (1 - 3) * s], [(5 + 9) * s, (5 - 9) * s]])
    want = np.array([[(rows[0, 0] + rows[1, 0]) * s, (rows[0, 1] + rows[1, 1]) * s],
                     [(rows[0, 0] - rows[1, 0]) * s, (rows[0, 1] - rows[1, 1]) * s]])
    assert np.max(np.abs(c - want)) < 1e-14


@pytest.mark.parametrize("n,levels", [(16, 2), (32, 3), (8, 3)])
def test_tight_frame_and_orthonormal_bases(n, levels):
    """Psi Psi^dagger = I and W_b^dagger W_b = I."""
    rng = np.random.default_rng(n)
    sara = SARA(n, levels)
    X = rng.standard_normal((n * n, 4))
    assert np.max(np.abs(sara.forward(sara.adjoint(X)) - X)) < 1e-13
    for b, h in sara.filters.items():
        c = dwt2(X.reshape(n, n, 4), h, levels)
        assert abs(np.linalg.norm(c) - np.linalg.norm(X)) < 1e-12 * np.linalg.norm(X)
        assert np.max(np.abs(idwt2(c, h, levels) - X.reshape(n, n, 4))) < 1e-13
    # ||Psi^dagger x|| = ||x|| (Parseval of a tight frame with bound 1)
    assert abs(np.linalg.norm(sara.adjoint(X)) - np.linalg.norm(X)) < 1e-12 * np.linalg.norm(X)


def test_adjoint_pair():
    rng = np.random.default_rng(5)
    sara = SARA(16, 2)
    X = rng.standard_normal((256, 4))
    A = rng.standard_normal((sara.J, 4))
    assert abs(np.sum(sara.adjoint(X) * A) - np.sum(X * sara.forward(A))) < 1e-12 * np.sum(np.abs(A))


def test_explicit_matrix_spectral_norm_is_one():
    sara = SARA(8, 3)
    N = 64
    Mat = np.array([sara.adjoint(np.eye(N)[:, j]) for j in range(N)]).T   # J x N
    assert abs(np.linalg.norm(Mat, 2) - 1.0) < 1e-13
    assert np.max(np.abs(Mat.T @ Mat - np.eye(N))) < 1e-13


@pytest.mark.parametrize("p", [1, 4, 8])
def test_constant_image_has_no_details(p):
    n, L = 16, 3
    c = dwt2(np.full((n, n), 2.5), daubechies_lowpass(p), L)
    m = n >> L
    assert np.max(np.abs(c[:m, :m] - 2.5 * 2 ** L)) < 1e-12
    mask = np.ones((n, n), bool)
    mask[:m, :m] = False
    assert np.max(np.abs(c[mask])) < 1e-12


@pytest.mark.parametrize("p", range(2, 9))
def test_filters_are_minimum_phase(p):
    """Daubechies' choice among the spectral factors (Sec. 3.1 names the Daubechies bases; the
    filters are the minimum-phase ones): h(z) = (1 + z)^p q(z), and every zero of q lies inside
    the unit circle.  Checked on the output filter with library polynomial division and root
    finding, independently of how the filter was built; the identities above hold for every
    spectral factor, so they cannot tell the phases apart."""
    h = daubechies_lowpass(p)
    binom = np.array([math.comb(p, k) for k in range(p + 1)], dtype=np.float64)
    q, rem = np.polydiv(h, binom)
    assert np.max(np.abs(rem)) < 1e-12
    assert len(q) == p
    zeros = np.roots(q)
    assert np.all(np.abs(zeros) < 1.0 - 1e-6), np.abs(zeros)
    # the p-fold zero at -1 is all of the unit-circle zeros: q has none there
    assert abs(np.polyval(q, -1.0)) > 1e-3
