"""ORACLE (test infrastructure only): periodic orthonormal Daubechies wavelet
transforms in plain FP64 NumPy.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library.

The paper represents every layer in a Daubechies-3 orthonormal wavelet basis
(Sec. 5.1; the transform W and its inverse in the operator of Sec. 5.1).  It
does not fix boundary handling, filter phase or band layout; the readings used
here are:

* periodic boundaries (the only standard choice that keeps W exactly
  orthonormal);
* analysis a_k = sum_n h_n x[(2k+n) mod M], d_k = sum_n g_n x[(2k+n) mod M]
  with g_n = (-1)^n h_{L-1-n}; synthesis is the exact transpose;
* one 2-D level filters along y (the fast index) first, then along x; the
  result is stored in Mallat layout (LL top-left, recursed on).
"""
import math

import numpy as np


def db3_lowpass():
    """Daubechies' 6-tap (3 vanishing moments) scaling filter in closed form
    (Daubechies 1988), normalised so that sum h = sqrt(2)."""
    s10 = math.sqrt(10.0)
    q = math.sqrt(5.0 + 2.0 * s10)
    h = np.array([1.0 + s10 + q,
                  5.0 + s10 + 3.0 * q,
                  10.0 - 2.0 * s10 + 2.0 * q,
                  10.0 - 2.0 * s10 - 2.0 * q,
                  5.0 + s10 - 3.0 * q,
                  1.0 + s10 - q])
    return h / (16.0 * math.sqrt(2.0))


def haar_lowpass():
    """Daubechies-1 (Haar) scaling filter."""
    return np.array([1.0, 1.0]) / math.sqrt(2.0)


def highpass(h):
    """Quadrature mirror wavelet filter g_n = (-1)^n h_{L-1-n}."""
    L = len(h)
    return np.array([(-1.0) ** n * h[L - 1 - n] for n in range(L)])


def analysis_1d(x, h, axis=-1):
    """One periodic analysis step along ``axis``: returns (a, d), each half
    the length: a_k = sum_n h_n x[(2k+n) mod M], likewise d with g."""
    g = highpass(h)
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    M = x.shape[-1]
    assert M % 2 == 0
    k = np.arange(M // 2)
    a = np.zeros(x.shape[:-1] + (M // 2,))
    d = np.zeros(x.shape[:-1] + (M // 2,))
    for n in range(len(h)):
        idx = (2 * k + n) % M
        a += h[n] * x[..., idx]
        d += g[n] * x[..., idx]
    return np.moveaxis(a, -1, axis), np.moveaxis(d, -1, axis)


def synthesis_1d(a, d, h, axis=-1):
    """Transpose of ``analysis_1d``: x_i = sum over (k, n) with
    (2k+n) mod M = i of h_n a_k + g_n d_k."""
    g = highpass(h)
    a = np.moveaxis(np.asarray(a, dtype=np.float64), axis, -1)
    d = np.moveaxis(np.asarray(d, dtype=np.float64), axis, -1)
    half = a.shape[-1]
    M = 2 * half
    k = np.arange(half)
    x = np.zeros(a.shape[:-1] + (M,))
    for n in range(len(h)):
        idx = (2 * k + n) % M
        contrib = h[n] * a + g[n] * d
        # indices within one tap are distinct (2k+n covers distinct values mod M)
        x[..., idx] += contrib
    return np.moveaxis(x, -1, axis)


def fdwt2(layer, levels, h=None):
    """Forward 2-D transform W of an N x N layer [x][y] into Mallat layout."""
    h = db3_lowpass() if h is None else h
    c = np.array(layer, dtype=np.float64, copy=True)
    M = c.shape[0]
    assert c.shape == (M, M)
    for _ in range(levels):
        blk = c[:M, :M]
        lo, hi = analysis_1d(blk, h, axis=1)           # along y (fast index)
        tmp = np.concatenate([lo, hi], axis=1)
        lo, hi = analysis_1d(tmp, h, axis=0)           # along x
        c[:M, :M] = np.concatenate([lo, hi], axis=0)
        M //= 2
    return c


def idwt2(coeffs, levels, h=None):
    """Inverse 2-D transform W^-1 (= W^T): Mallat layout -> layer [x][y]."""
    h = db3_lowpass() if h is None else h
    c = np.array(coeffs, dtype=np.float64, copy=True)
    N = c.shape[0]
    for k in range(levels, 0, -1):
        M = N >> (k - 1)
        blk = c[:M, :M]
        tmp = synthesis_1d(blk[:M // 2, :], blk[M // 2:, :], h, axis=0)   # undo x step
        c[:M, :M] = synthesis_1d(tmp[:, :M // 2], tmp[:, M // 2:], h, axis=1)  # undo y step
    return c


def fdwt1_multilevel(x, levels, h=None):
    """1-D multi-level transform (Mallat layout) of a length-N vector."""
    h = db3_lowpass() if h is None else h
    c = np.array(x, dtype=np.float64, copy=True)
    M = len(c)
    for _ in range(levels):
        a, d = analysis_1d(c[:M], h)
        c[:M] = np.concatenate([a, d])
        M //= 2
    return c


def idwt1_multilevel(c, levels, h=None):
    """Inverse of ``fdwt1_multilevel``."""
    h = db3_lowpass() if h is None else h
    x = np.array(c, dtype=np.float64, copy=True)
    N = len(x)
    for k in range(levels, 0, -1):
        M = N >> (k - 1)
        x[:M] = synthesis_1d(x[:M // 2], x[M // 2:M], h)
    return x


def coefficient_level(N, levels):
    """N x N array of the scale index k of each Mallat coefficient: k = 1 for
    the finest details ... k = levels for the coarsest details and the final
    low-pass band."""
    idx = np.arange(N)
    m = np.maximum(idx[:, None], idx[None, :])
    k = np.full((N, N), levels, dtype=np.int64)
    for lev in range(levels, 0, -1):
        k[m >= (N >> lev)] = lev
    return k
