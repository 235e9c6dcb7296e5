"""The blurring operator A (a BTTB matrix) and its transpose, in FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper applies A and A^T through IR Tools' structured matvecs (Section 5,
and the work-unit discussion in Section 5.2).  It does not state the boundary
condition, the PSF centre, or convolution vs correlation; the reading taken
here is: zero boundary, centre (h, h), A = true convolution,
A^T = correlation:

    (A X)[i, j]   = sum_{u,v=-h..h} P[h+u, h+v] X[i-u, j-v]
    (A^T Y)[i, j] = sum_{u,v=-h..h} P[h+u, h+v] Y[i+u, j+v]

with X, Y = 0 outside [0, n)^2.

Pins (tests/test_oracle_operator.py): the direct form equals
scipy.signal.convolve2d ('same', zero fill); the dense matrix equals the
Kronecker-sum expansion sum_{k,l} P[k,l] Z_{l-h} (x) Z_{k-h}; adjointness
<Ax, y> = <x, A^T y>; PSF = delta gives the identity; the FFT form equals the
direct form.
"""
from __future__ import annotations

import numpy as np
import scipy.fft


def _check(psf: np.ndarray, x: np.ndarray):
    k = psf.shape[0]
    if psf.shape != (k, k) or k % 2 != 1:
        raise ValueError("PSF must be K x K with K odd")
    if x.ndim != 2 or x.shape[0] != x.shape[1]:
        raise ValueError("image must be square")
    return k, (k - 1) // 2, x.shape[0]


def blur(psf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A X by the definition: one shifted, weighted copy of X per PSF tap."""
    k, h, n = _check(psf, x)
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros((n, n), dtype=np.float64)
    for u in range(-h, h + 1):
        # rows i with 0 <= i-u < n
        i0, i1 = max(0, u), min(n, n + u)
        if i0 >= i1:
            continue
        for v in range(-h, h + 1):
            j0, j1 = max(0, v), min(n, n + v)
            if j0 >= j1:
                continue
            y[i0:i1, j0:j1] += psf[h + u, h + v] * x[i0 - u:i1 - u, j0 - v:j1 - v]
    return y


def blur_t(psf: np.ndarray, y: np.ndarray) -> np.ndarray:
    """A^T Y by the definition (correlation with the PSF)."""
    k, h, n = _check(psf, y)
    y = np.asarray(y, dtype=np.float64)
    x = np.zeros((n, n), dtype=np.float64)
    for u in range(-h, h + 1):
        i0, i1 = max(0, -u), min(n, n - u)
        if i0 >= i1:
            continue
        for v in range(-h, h + 1):
            j0, j1 = max(0, -v), min(n, n - v)
            if j0 >= j1:
                continue
            x[i0:i1, j0:j1] += psf[h + u, h + v] * y[i0 + u:i1 + u, j0 + v:j1 + v]
    return x


class FFTBlur:
    """A and A^T through a zero-padded linear convolution by real FFTs.

    The full linear convolution of an n x n image with a K x K PSF has size
    (n+K-1)^2; padding both to L >= n+K-1 makes the circular convolution of
    the padded arrays equal to it, and A X is its central n x n block
    starting at (h, h).  A^T is the same with the PSF rotated by 180 degrees.
    """

    def __init__(self, psf: np.ndarray, n: int, workers: int | None = None):
        k = psf.shape[0]
        if psf.shape != (k, k) or k % 2 != 1:
            raise ValueError("PSF must be K x K with K odd")
        self.n, self.k, self.h = n, k, (k - 1) // 2
        self.L = scipy.fft.next_fast_len(n + k - 1, real=True)
        self.workers = workers
        p = np.zeros((self.L, self.L))
        p[:k, :k] = psf
        self._f = scipy.fft.rfft2(p, workers=workers)
        pf = np.zeros((self.L, self.L))
        pf[:k, :k] = psf[::-1, ::-1]
        self._ft = scipy.fft.rfft2(pf, workers=workers)

    def _conv(self, f, x):
        n, h, L = self.n, self.h, self.L
        xp = np.zeros((L, L))
        xp[:n, :n] = x
        full = scipy.fft.irfft2(scipy.fft.rfft2(xp, workers=self.workers) * f,
                                s=(L, L), workers=self.workers)
        return full[h:h + n, h:h + n]

    def blur(self, x):
        return self._conv(self._f, x)

    def blur_t(self, y):
        return self._conv(self._ft, y)


def dense_matrix(psf: np.ndarray, n: int) -> np.ndarray:
    """The N x N matrix of A (N = n^2) in the paper's column-major vec
    ordering (Section 3, vec stacks columns): column q of the result is
    vec(A E_q) where vec(E_q) is the q-th unit vector."""
    N = n * n
    a = np.zeros((N, N))
    for q in range(N):
        e = np.zeros(N)
        e[q] = 1.0
        a[:, q] = blur(psf, e.reshape((n, n), order="F")).reshape(N, order="F")
    return a


def vec(x: np.ndarray) -> np.ndarray:
    """Column-major stacking of an image (Section 3)."""
    return np.asarray(x).reshape(-1, order="F")


def unvec(v: np.ndarray, n: int) -> np.ndarray:
    return np.asarray(v).reshape((n, n), order="F")


def normal_op(psf: np.ndarray, lam: float, x: np.ndarray, fft: FFTBlur | None = None):
    """H_lambda x = A^T A x + lambda^2 x (eq. (tik:normal2))."""
    if fft is not None:
        return fft.blur_t(fft.blur(x)) + lam * lam * x
    return blur_t(psf, blur(psf, x)) + lam * lam * x
