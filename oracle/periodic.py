"""Periodic boundary condition: the blurring matrix as a block-circulant
(BCCB) matrix, its one-term Kronecker approximation with circulant factors,
and the exact Tikhonov minimiser through the 2-D DFT.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper does not state a boundary condition; it applies A through IR
Tools' structured operators, which also offer periodic and reflexive
boundaries.  The reading for the periodic case keeps the zero-boundary
conventions (centre (h, h), A = true convolution, A^T = correlation) and
extends the image periodically:

    (A X)[i, j]   = sum_{u,v=-h..h} P[h+u, h+v] X[(i-u) mod n, (j-v) mod n]
    (A^T Y)[i, j] = sum_{u,v=-h..h} P[h+u, h+v] Y[(i+u) mod n, (j+v) mod n]

for K <= n (a larger PSF would wrap onto itself).  Then

    A = sum_{u,v} P[h+u, h+v] C_v (x) C_u,   C_d[i, i'] = [i - i' = d mod n],

the cyclic-shift analogue of the zero-boundary expansion.  The C_v (x) C_u
have disjoint supports and ||C_d||_F^2 = n for every d, so for circulant
factors C(a) (x) C(c) with C(f) = sum_d f[h+d] C_d,

    ||A - C(a) (x) C(c)||_F^2 = n^2 sum_{u,v} (P[u, v] - c_u a_v)^2,

and the Frobenius-optimal term (Section 5, eq. (KronSumDecomp)) comes from
the leading singular triple of P itself: c = sqrt(s1) u1, a = sqrt(s1) v1,
i.e. the zero-boundary weighted-PSF construction with every weight equal to
n.  ||A - A_hat||_F / ||A||_F = sqrt(sum_{k>1} s_k^2 / sum_k s_k^2) with the
singular values s_k of P.

The factor SVDs (Section 3, eq. (AKronSVD)) and the preconditioner solve
(eq. (PreconSolve)) are those of kp.py, applied to the circulant factors.

A BCCB matrix is diagonalised by the 2-D DFT.  With P placed cyclically
around (0, 0) (P0[u mod n, v mod n] = P[h+u, h+v]), A X = ifft2(P0^ X^),
A^T Y = ifft2(conj(P0^) Y^), and the Tikhonov minimiser of eq.
(tik:normal2) has the closed form

    x_lambda = ifft2(conj(P0^) B^ / (|P0^|^2 + lambda^2)).

The singular values of a circulant C(f) are the moduli of the DFT of its
first column.

Pins (tests/test_oracle_periodic.py): scipy.signal.convolve2d and
correlate2d with boundary='wrap'; adjointness; the constant image is an
eigenvector with eigenvalue sum(P); the DFT form equals the definition; the
dense matrix equals the cyclic Kronecker-sum expansion; the one-term KP is
exact for separable PSFs, equals the brute-force Van Loan-Pitsianis nearest
Kronecker product on tiny images, and its error matches the singular-value
formula; the circulant factors' singular values are |DFT| of their columns;
the closed-form x_lambda equals a dense Cholesky solve; the oracle's PCG
converges to it; the exact KP-basis diagonal (exact_diag, the circulant
form of kp.exact_diag) equals ||A (v_c,i v_r,j^T)||_F^2 from blurring every
basis image, reduces to s_c^2 s_r^2 for separable PSFs and sums to
||A||_F^2 = n^2 ||P||_F^2.
"""
from __future__ import annotations

import numpy as np

from . import kp as kpmod


def _check(psf: np.ndarray, n: int):
    k = psf.shape[0]
    if psf.shape != (k, k) or k % 2 != 1:
        raise ValueError("PSF must be K x K with K odd")
    if k > n:
        raise ValueError("periodic boundary needs K <= n")
    return k, (k - 1) // 2


def blur(psf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A X by the definition: one cyclically shifted, weighted copy of X per
    PSF tap (np.roll(X, (u, v))[i, j] = X[(i-u) mod n, (j-v) mod n])."""
    x = np.asarray(x, dtype=np.float64)
    k, h = _check(psf, x.shape[0])
    y = np.zeros_like(x)
    for u in range(-h, h + 1):
        for v in range(-h, h + 1):
            y += psf[h + u, h + v] * np.roll(x, (u, v), axis=(0, 1))
    return y


def blur_t(psf: np.ndarray, y: np.ndarray) -> np.ndarray:
    """A^T Y by the definition (cyclic correlation with the PSF)."""
    y = np.asarray(y, dtype=np.float64)
    k, h = _check(psf, y.shape[0])
    x = np.zeros_like(y)
    for u in range(-h, h + 1):
        for v in range(-h, h + 1):
            x += psf[h + u, h + v] * np.roll(y, (-u, -v), axis=(0, 1))
    return x


def psf_spectrum(psf: np.ndarray, n: int) -> np.ndarray:
    """2-D DFT of the PSF placed cyclically around (0, 0): the eigenvalues
    of A."""
    k, h = _check(psf, n)
    p0 = np.zeros((n, n))
    for u in range(-h, h + 1):
        for v in range(-h, h + 1):
            p0[u % n, v % n] += psf[h + u, h + v]
    return np.fft.fft2(p0)


def blur_fft(psf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A X through the DFT diagonalisation."""
    x = np.asarray(x, dtype=np.float64)
    return np.real(np.fft.ifft2(psf_spectrum(psf, x.shape[0]) * np.fft.fft2(x)))


def blur_t_fft(psf: np.ndarray, y: np.ndarray) -> np.ndarray:
    y = np.asarray(y, dtype=np.float64)
    return np.real(np.fft.ifft2(np.conj(psf_spectrum(psf, y.shape[0])) * np.fft.fft2(y)))


def x_lambda(psf: np.ndarray, b: np.ndarray, lam: float) -> np.ndarray:
    """Exact Tikhonov minimiser (eq. (tik:normal2)) by the 2-D DFT."""
    b = np.asarray(b, dtype=np.float64)
    f = psf_spectrum(psf, b.shape[0])
    return np.real(np.fft.ifft2(np.conj(f) * np.fft.fft2(b) / (np.abs(f) ** 2 + lam * lam)))


def shift(d: int, n: int) -> np.ndarray:
    """The cyclic shift C_d[i, i'] = [i - i' = d mod n]."""
    return np.roll(np.eye(n), d, axis=0)


def dense_matrix(psf: np.ndarray, n: int) -> np.ndarray:
    """The N x N matrix of A in the column-major vec ordering (tiny n)."""
    N = n * n
    a = np.zeros((N, N))
    for q in range(N):
        e = np.zeros(N)
        e[q] = 1.0
        a[:, q] = blur(psf, e.reshape((n, n), order="F")).reshape(N, order="F")
    return a


def circulant_band(f: np.ndarray, n: int) -> np.ndarray:
    """C(f)[i, i'] = f[h + d] where d in [-h, h] and d = i - i' mod n."""
    k = f.shape[0]
    h = (k - 1) // 2
    if k > n:
        raise ValueError("periodic boundary needs K <= n")
    return sum(f[h + d] * shift(d, n) for d in range(-h, h + 1))


def kp_profiles(psf: np.ndarray):
    """(c, a, s): the leading singular triple of P as profiles, sum(c) > 0,
    and all singular values of P."""
    u, s, vt = np.linalg.svd(np.asarray(psf, dtype=np.float64))
    c = np.sqrt(s[0]) * u[:, 0]
    a = np.sqrt(s[0]) * vt[0, :]
    if c.sum() < 0:
        c, a = -c, -a
    return c, a, s


def kp_svd(psf: np.ndarray, n: int) -> kpmod.KPSVD:
    """Circulant factors A_c = C(c), A_r = C(a) and their FP64 SVDs (eq.
    (AKronSVD)); A_hat X = A_c X A_r^T as for the zero boundary."""
    _check(psf, n)
    c, a, s = kp_profiles(psf)
    ac = circulant_band(c, n)
    ar = circulant_band(a, n)
    uc, sc, vct = np.linalg.svd(ac)
    ur, sr, vrt = np.linalg.svd(ar)
    return kpmod.KPSVD(n=n, Ac=ac, Ar=ar, Uc=uc, sc=sc, Vc=vct.T, Ur=ur, sr=sr,
                       Vr=vrt.T, s_psf=s)


def kp_all_terms(psf: np.ndarray, rel: float = 1e-12):
    """All terms of the exact expansion A = sum_k C(a_k) (x) C(c_k) from the
    plain SVD of P (c_k = sqrt(s_k) u_k, a_k = sqrt(s_k) v_k, s_k > rel s_1)."""
    u, s, vt = np.linalg.svd(np.asarray(psf, dtype=np.float64))
    t = kpmod.kp_terms(s, rel)
    return ([np.sqrt(s[i]) * u[:, i] for i in range(t)],
            [np.sqrt(s[i]) * vt[i, :] for i in range(t)])


def exact_diag(kp: kpmod.KPSVD, psf: np.ndarray, rel: float = 1e-12) -> np.ndarray:
    """D0[i, j] = ||A (v_c,i v_r,j^T)||_F^2 for the periodic A, through its
    Kronecker sum as in kp.exact_diag with circulant factors."""
    n = kp.n
    cs, as_ = kp_all_terms(psf, rel)
    B = [circulant_band(c, n) @ kp.Vc for c in cs]
    C = [circulant_band(a, n) @ kp.Vr for a in as_]
    d0 = np.zeros((n, n))
    for k in range(len(cs)):
        for l in range(len(cs)):
            d0 += np.outer(np.sum(B[k] * B[l], axis=0), np.sum(C[k] * C[l], axis=0))
    return d0


class NormalOperator:
    """H_lambda = A^T A + lambda^2 I for the periodic boundary, with the same
    interface as solvers.NormalOperator (A, At, H); the DFT form above 64."""

    def __init__(self, psf: np.ndarray, n: int, lam: float, use_fft: bool | None = None):
        _check(psf, n)
        self.psf, self.n, self.lam = psf, n, float(lam)
        self.use_fft = n > 64 if use_fft is None else use_fft
        self._f = psf_spectrum(psf, n) if self.use_fft else None

    def A(self, x):
        if self._f is None:
            return blur(self.psf, x)
        return np.real(np.fft.ifft2(self._f * np.fft.fft2(x)))

    def At(self, y):
        if self._f is None:
            return blur_t(self.psf, y)
        return np.real(np.fft.ifft2(np.conj(self._f) * np.fft.fft2(y)))

    def H(self, x):
        return self.At(self.A(x)) + self.lam * self.lam * x
