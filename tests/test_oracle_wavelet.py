"""Pins of the oracle's wavelet transform (Sec. 5.1: Daubechies n = 3,
orthonormal) against published values, closed forms and invariants."""
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_db3():
    vals = [float(l) for l in open(os.path.join(GOLD, "db3_filter.txt"))
            if l.strip() and not l.startswith("#")]
    return np.array(vals)


def test_db3_matches_published_table():
    h = O.db3_lowpass()
    assert np.max(np.abs(h - _golden_db3())) < 1e-11


def test_db3_filter_identities():
    h = O.db3_lowpass()
    g = O.highpass(h)
    assert abs(h.sum() - math.sqrt(2.0)) < 1e-15
    assert abs((h * h).sum() - 1.0) < 1e-15
    # double-shift orthogonality
    for m in (1, 2):
        assert abs(np.dot(h[:-2 * m], h[2 * m:])) < 1e-15
    # three vanishing moments of the wavelet filter, and the fourth is not zero
    n = np.arange(6.0)
    for p in range(3):
        assert abs(np.sum(g * n ** p)) < 1e-13
    assert abs(np.sum(g * n ** 3)) > 1.0


def test_phase_convention_on_unit_impulse():
    # a_k = sum_n h_n x[(2k+n) mod M] for x = e_0 on M = 8:
    # k=0 takes n=0, k=2 takes n=4 (2*2+4=8), k=3 takes n=2 (6+2=8).
    h = O.db3_lowpass()
    g = O.highpass(h)
    x = np.zeros(8)
    x[0] = 1.0
    a, d = O.analysis_1d(x, h)
    np.testing.assert_allclose(a, [h[0], 0.0, h[4], h[2]], atol=0, rtol=0)
    np.testing.assert_allclose(d, [g[0], 0.0, g[4], g[2]], atol=0, rtol=0)


def test_haar_closed_form():
    h = O.haar_lowpass()
    x = np.array([3.0, 1.0, -2.0, 5.0])
    a, d = O.analysis_1d(x, h)
    np.testing.assert_allclose(a, [(3 + 1) / math.sqrt(2), (-2 + 5) / math.sqrt(2)], rtol=1e-15)
    np.testing.assert_allclose(d, [(3 - 1) / math.sqrt(2), (-2 - 5) / math.sqrt(2)], rtol=1e-15)
    # 2-D one level on a 2x2 block: LL = sum/2, and the three details
    blk = np.array([[1.0, 2.0], [3.0, 4.0]])
    c = O.fdwt2(blk, 1, h)
    # y first: rows -> [(1+2)/r2, (1-2)/r2], [(3+4)/r2, (3-4)/r2]; then x
    np.testing.assert_allclose(c, [[(1 + 2 + 3 + 4) / 2, (1 - 2 + 3 - 4) / 2],
                                   [(1 + 2 - 3 - 4) / 2, (1 - 2 - 3 + 4) / 2]], rtol=1e-15)


def _dense(fn, n):
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(fn(e))
    return np.array(cols).T


@pytest.mark.parametrize("N,levels", [(16, 1), (16, 2), (32, 3), (24, 2)])
def test_2d_transform_is_orthonormal(N, levels):
    W = _dense(lambda v: O.fdwt2(v.reshape(N, N), levels).ravel(), N * N)
    Wi = _dense(lambda v: O.idwt2(v.reshape(N, N), levels).ravel(), N * N)
    assert np.max(np.abs(W @ W.T - np.eye(N * N))) < 1e-12
    assert np.max(np.abs(Wi - W.T)) < 1e-13


def test_2d_transform_against_kronecker_assembly():
    # independent construction: one level is (A1 kron I) (I kron A1) on the
    # row-major [x][y] block, with A1 the 1-D periodic analysis matrix.
    h = O.db3_lowpass()
    g = O.highpass(h)

    def a1(M):
        A = np.zeros((M, M))
        for k in range(M // 2):
            for n in range(6):
                A[k, (2 * k + n) % M] += h[n]
                A[M // 2 + k, (2 * k + n) % M] += g[n]
        return A

    N, levels = 32, 3
    W = np.eye(N * N)
    for lev in range(levels):
        M = N >> lev
        step = np.kron(a1(M), np.eye(M)) @ np.kron(np.eye(M), a1(M))
        E = np.eye(N * N)
        sel = np.array([x * N + y for x in range(M) for y in range(M)])
        E[np.ix_(sel, sel)] = step
        W = E @ W
    x = np.random.default_rng(3).standard_normal((N, N))
    assert np.max(np.abs(O.fdwt2(x, levels).ravel() - W @ x.ravel())) < 1e-12


def test_quadratic_has_zero_interior_details():
    # three vanishing moments: level-1 details of a quadratic vanish away from
    # the periodic wrap.
    N = 64
    xs = np.arange(N, dtype=float)
    f = 0.3 * xs[:, None] ** 2 - 2.0 * xs[:, None] * xs[None, :] + 0.7 * xs[None, :] ** 2 + 5.0
    c = O.fdwt2(f, 1)
    H = N // 2
    interior = slice(0, H - 3)
    scale = np.abs(f).max()
    assert np.max(np.abs(c[:H, H:][interior, interior])) < 1e-12 * scale
    assert np.max(np.abs(c[H:, :H][interior, interior])) < 1e-12 * scale
    assert np.max(np.abs(c[H:, H:][interior, interior])) < 1e-12 * scale


def test_parseval_and_roundtrip():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((128, 128))
    c = O.fdwt2(x, 5)
    assert abs(np.sum(c * c) - np.sum(x * x)) < 1e-10 * np.sum(x * x)
    assert np.max(np.abs(O.idwt2(c, 5) - x)) < 1e-12


def test_1d_multilevel_roundtrip():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(160)
    c = O.fdwt1_multilevel(x, 5)
    assert np.max(np.abs(O.idwt1_multilevel(c, 5) - x)) < 1e-13


def test_coefficient_level_map():
    k = O.coefficient_level(16, 2)
    assert k[0, 0] == 2 and k[3, 3] == 2 and k[4, 0] == 2 and k[7, 7] == 2
    assert k[8, 0] == 1 and k[0, 8] == 1 and k[15, 15] == 1
    assert (k == 1).sum() == 16 * 16 - 8 * 8
