"""Pins for the oracle's blur operator (zero boundary, true convolution).

Each test checks the oracle against something other than itself: a library
routine (scipy.signal), an algebraic identity, or a special case.
"""
import numpy as np
import pytest
import scipy.signal

import synthetic as S
from oracle import operator as O


CASES = [(7, 5), (9, 3), (12, 7), (5, 9), (16, 15), (1, 1)]


@pytest.mark.parametrize("n,k", CASES)
def test_blur_equals_library_convolution(n, k):
    rng = np.random.default_rng(n * 100 + k)
    psf = rng.uniform(0, 1, (k, k))
    x = rng.standard_normal((n, n))
    ref = scipy.signal.convolve2d(x, psf, mode="same", boundary="fill")
    assert np.allclose(O.blur(psf, x), ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n,k", CASES)
def test_blur_t_equals_library_correlation(n, k):
    rng = np.random.default_rng(n * 77 + k)
    psf = rng.uniform(0, 1, (k, k))
    y = rng.standard_normal((n, n))
    ref = scipy.signal.correlate2d(y, psf, mode="same", boundary="fill")
    assert np.allclose(O.blur_t(psf, y), ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n,k", CASES)
def test_adjoint_identity(n, k):
    rng = np.random.default_rng(3 + n + k)
    psf = rng.standard_normal((k, k))
    x, y = rng.standard_normal((2, n, n))
    lhs = np.sum(O.blur(psf, x) * y)
    rhs = np.sum(x * O.blur_t(psf, y))
    assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))


def test_delta_psf_is_identity():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((11, 11))
    for k in (1, 3, 9):
        d = np.zeros((k, k))
        d[k // 2, k // 2] = 1.0
        assert np.array_equal(O.blur(d, x), x)
        assert np.array_equal(O.blur_t(d, x), x)


def test_off_centre_tap_is_a_shift():
    # P[h+1, h] = 1 moves the image one row down: (AX)[i,j] = X[i-1, j]
    x = np.arange(36, dtype=float).reshape(6, 6)
    p = np.zeros((3, 3))
    p[2, 1] = 1.0
    y = O.blur(p, x)
    assert np.array_equal(y[1:], x[:-1]) and np.all(y[0] == 0)


@pytest.mark.parametrize("n,k", [(16, 5), (33, 15), (64, 31), (40, 63)])
def test_fft_form_equals_direct(n, k):
    rng = np.random.default_rng(n + k)
    psf = rng.uniform(0, 1, (k, k))
    psf /= psf.sum()
    x = rng.standard_normal((n, n))
    f = O.FFTBlur(psf, n)
    d, dt = O.blur(psf, x), O.blur_t(psf, x)
    assert np.linalg.norm(f.blur(x) - d) <= 1e-13 * np.linalg.norm(d)
    assert np.linalg.norm(f.blur_t(x) - dt) <= 1e-13 * np.linalg.norm(dt)


def _shift(n, d):
    return np.eye(n, k=-d)   # Z_d[i, i'] = [i - i' = d]


@pytest.mark.parametrize("n,k", [(6, 3), (7, 5), (5, 7)])
def test_dense_matrix_is_kronecker_sum_of_shifts(n, k):
    """Column-major vec: A = sum_{u,v} P[h+u, h+v] Z_v (x) Z_u (Section 3's
    vec/Kronecker rules), an independent construction of the BTTB matrix."""
    rng = np.random.default_rng(n + 10 * k)
    psf = rng.standard_normal((k, k))
    h = k // 2
    ref = np.zeros((n * n, n * n))
    for u in range(-h, h + 1):
        for v in range(-h, h + 1):
            ref += psf[h + u, h + v] * np.kron(_shift(n, v), _shift(n, u))
    assert np.allclose(O.dense_matrix(psf, n), ref, atol=1e-14)


def test_kronecker_vec_identity():
    """(C (x) D) vec(Y) = vec(D Y C^T) (Section 3, fourth Kronecker rule)."""
    rng = np.random.default_rng(5)
    c, d, y = rng.standard_normal((3, 6, 6))
    assert np.allclose(np.kron(c, d) @ O.vec(y), O.vec(d @ y @ c.T), atol=1e-13)


def test_generator_data_uses_same_operator():
    """The generator's data b_true (scipy fftconvolve) equals the oracle's A x."""
    p = S.small_gaussian(3)
    ax = O.blur(p.psf, p.x_true)
    resid = p.b.astype(np.float64) - ax
    # what is left is the noise, of the requested level
    lvl = np.linalg.norm(resid) / np.linalg.norm(ax)
    assert abs(lvl - 0.01) < 1e-4
