"""Reflexive boundary condition for PSFs symmetric in both axes: the
blurring matrix with the image extended by half-sample reflection, its
one-term Kronecker approximation with reflexive (Toeplitz-plus-Hankel)
factors, and the exact Tikhonov minimiser through the 2-D DCT.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper states no boundary condition (IR Tools' operators offer zero,
periodic and reflexive ones).  The reading for the reflexive case keeps the
zero-boundary conventions (centre (h, h), A = true convolution) and extends
the image by half-sample reflection, refl(j) = -j - 1 for j < 0 and
2n - 1 - j for j >= n:

    (A X)[i, j] = sum_{u,v=-h..h} P[h+u, h+v] X[refl(i-u), refl(j-v)],

for K <= n (one reflection covers every index).  Then A = sum_{u,v}
P[h+u, h+v] R_v (x) R_u with R_d[i, i'] = [refl(i - d) = i'].  This module
is restricted to PSFs symmetric in both axes (P[h+u, h+v] = P[h-u, h+v] =
P[h+u, h-v]): their SVD has even profiles, each R(f) = sum_d f[h+d] R_d with
even f is a symmetric Toeplitz-plus-Hankel matrix, so A is symmetric,
A^T = A, and A is diagonalised by the orthonormal 2-D DCT-II:

    A X = idct2(L .* dct2(X)),   L = dct2(A E_00) ./ dct2(E_00),

with E_00 the unit image at (0, 0); the Tikhonov minimiser of eq.
(tik:normal2) is x_lambda = idct2(L .* dct2(B) ./ (L.^2 + lambda^2)).

One-term Kronecker approximation (Section 5, eq. (KronSumDecomp)): the
reflected shifts R_d overlap near the borders, so the weighted-PSF
construction is no longer exactly Frobenius-optimal.  The reading: the
leading term of the exact expansion A = sum_k R(a_k) (x) R(c_k) from the
plain SVD of P (c_k = sqrt(s_k) u_k, a_k = sqrt(s_k) v_k), the same
construction as the periodic boundary; it is exact for separable PSFs.  The
factor SVDs (eq. (AKronSVD)), the preconditioner solve (eq. (PreconSolve))
and the exact KP-basis diagonal follow kp.py with reflexive factors.

PSFs not symmetric in both axes (the `*_general` functions below): A is the
same convolution of the reflected image, but no longer symmetric.  A^T
follows from the definition by scattering: A X gathers X[refl(i-u),
refl(j-v)] with weight P[h+u, h+v] into (i, j), so A^T Y adds
P[h+u, h+v] Y[i, j] into (refl(i-u), refl(j-v)) -- the correlation of Y
(zero outside the image) evaluated on the positions [-h, n+h) and folded
back onto the image by the reflection.  The DCT no longer diagonalises A;
x_lambda comes from a dense solve (tiny n) or FP64 PCG run to a true
relative residual of 1e-13 with the one-term reflexive KP preconditioner
(the leading term of the same plain-SVD expansion, which holds for any PSF
because the reflection acts on rows and columns separately).

Pins (tests/test_oracle_reflexive.py): scipy.ndimage.convolve with
mode='reflect'; A is symmetric for symmetric PSFs and preserves constant
images; the dense matrix equals the reflexive Kronecker-sum expansion; the
DCT form (with the closed-form corner response A E_00, itself pinned against
the definition) equals the definition; x_lambda equals a dense solve; the one-term
KP is exact for separable symmetric PSFs; the exact diagonal equals
||A (v_c,i v_r,j^T)||_F^2 by brute force; the oracle's PCG converges to
x_lambda.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from . import kp as kpmod


def is_symmetric_psf(psf: np.ndarray, rel: float = 1e-12) -> bool:
    p = np.asarray(psf, dtype=np.float64)
    tol = rel * np.abs(p).max()
    return (np.abs(p - p[::-1, :]).max() <= tol) and (np.abs(p - p[:, ::-1]).max() <= tol)


def _check(psf: np.ndarray, n: int, symmetric: bool = True):
    k = psf.shape[0]
    if psf.shape != (k, k) or k % 2 != 1:
        raise ValueError("PSF must be K x K with K odd")
    if k > n:
        raise ValueError("reflexive boundary needs K <= n")
    if symmetric and not is_symmetric_psf(psf):
        raise ValueError("reflexive boundary needs a PSF symmetric in both axes")
    return k, (k - 1) // 2


def refl(j: np.ndarray, n: int) -> np.ndarray:
    j = np.asarray(j)
    return np.where(j < 0, -j - 1, np.where(j >= n, 2 * n - 1 - j, j))


def blur(psf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A X by the definition (A^T = A for the PSFs accepted here)."""
    _check(psf, np.asarray(x).shape[0])
    return blur_general(psf, x)


def blur_general(psf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A X by the definition for any K x K PSF with K <= n:
    (A X)[i, j] = sum_{u,v} P[h+u, h+v] X[refl(i-u), refl(j-v)]."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    k, h = _check(psf, n, symmetric=False)
    idx = np.arange(n)
    y = np.zeros_like(x)
    for u in range(-h, h + 1):
        ri = refl(idx - u, n)
        for v in range(-h, h + 1):
            y += psf[h + u, h + v] * x[np.ix_(ri, refl(idx - v, n))]
    return y


def blur_t_general(psf: np.ndarray, y: np.ndarray) -> np.ndarray:
    """A^T Y by the definition: every term of blur_general scattered back,
    (A^T Y)[refl(i-u), refl(j-v)] += P[h+u, h+v] Y[i, j]."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    k, h = _check(psf, n, symmetric=False)
    idx = np.arange(n)
    out = np.zeros_like(y)
    for u in range(-h, h + 1):
        ri = refl(idx - u, n)
        for v in range(-h, h + 1):
            np.add.at(out, (ri[:, None], refl(idx - v, n)[None, :]), psf[h + u, h + v] * y)
    return out


def blur_fft_general(psf: np.ndarray, x: np.ndarray, workers: int | None = None) -> np.ndarray:
    """A X through the image extended by half-sample reflection (numpy's
    'symmetric' padding by h) and the 'valid' part of the linear convolution
    by zero-padded FFTs (the same operator as blur_general)."""
    import scipy.signal
    x = np.asarray(x, dtype=np.float64)
    k, h = _check(psf, x.shape[0], symmetric=False)
    return scipy.signal.fftconvolve(np.pad(x, h, mode="symmetric"), psf, mode="valid")


def fold(z: np.ndarray, h: int) -> np.ndarray:
    """The (n + 2h)^2 array z on the positions [-h, n+h)^2 folded onto the
    n x n image: entry (q1, q2) is added into (refl(q1), refl(q2))."""
    m = z.shape[0]
    n = m - 2 * h
    q = refl(np.arange(-h, n + h), n)
    out = np.zeros((n, n))
    np.add.at(out, (q[:, None], q[None, :]), z)
    return out


def blur_t_fft_general(psf: np.ndarray, y: np.ndarray,
                       workers: int | None = None) -> np.ndarray:
    """A^T Y as the correlation of Y (zero outside the image) on the
    positions [-h, n+h) -- the 'full' convolution with the flipped PSF, by
    zero-padded FFTs -- folded back by fold (the same operator as
    blur_t_general)."""
    import scipy.signal
    y = np.asarray(y, dtype=np.float64)
    k, h = _check(psf, y.shape[0], symmetric=False)
    z = scipy.signal.fftconvolve(y, psf[::-1, ::-1], mode="full")
    return fold(z, h)


def shift(d: int, n: int) -> np.ndarray:
    """R_d[i, i'] = [refl(i - d) = i']."""
    r = np.zeros((n, n))
    r[np.arange(n), refl(np.arange(n) - d, n)] = 1.0
    return r


def dense_matrix(psf: np.ndarray, n: int) -> np.ndarray:
    """The N x N matrix of A in the column-major vec ordering (tiny n); any
    PSF with K <= n."""
    N = n * n
    a = np.zeros((N, N))
    for q in range(N):
        e = np.zeros(N)
        e[q] = 1.0
        a[:, q] = blur_general(psf, e.reshape((n, n), order="F")).reshape(N, order="F")
    return a


def corner_response(psf: np.ndarray, n: int) -> np.ndarray:
    """A E_00 (E_00 the unit image at (0, 0)) in closed form: refl(i - u) = 0
    for u in {i, i + 1} only, so (A E_00)[i, j] is the sum of P[h+u, h+v]
    over u in {i, i+1}, v in {j, j+1} with |u|, |v| <= h."""
    k, h = _check(psf, n)
    r = np.zeros((n, n))
    for i in range(min(n, h + 1)):
        for j in range(min(n, h + 1)):
            for u in (i, i + 1):
                for v in (j, j + 1):
                    if u <= h and v <= h:
                        r[i, j] += psf[h + u, h + v]
    return r


def eigenvalues(psf: np.ndarray, n: int) -> np.ndarray:
    """L with A X = idct2(L .* dct2(X)) (orthonormal DCT-II)."""
    e = np.zeros((n, n))
    e[0, 0] = 1.0
    return (scipy.fft.dctn(corner_response(psf, n), type=2, norm="ortho")
            / scipy.fft.dctn(e, type=2, norm="ortho"))


def blur_dct(psf: np.ndarray, x: np.ndarray) -> np.ndarray:
    lam = eigenvalues(psf, x.shape[0])
    return scipy.fft.idctn(lam * scipy.fft.dctn(np.asarray(x, dtype=np.float64), type=2,
                                                norm="ortho"), type=2, norm="ortho")


def x_lambda(psf: np.ndarray, b: np.ndarray, lam: float) -> np.ndarray:
    """Exact Tikhonov minimiser (eq. (tik:normal2)) through the 2-D DCT."""
    b = np.asarray(b, dtype=np.float64)
    ev = eigenvalues(psf, b.shape[0])
    bh = scipy.fft.dctn(b, type=2, norm="ortho")
    return scipy.fft.idctn(ev * bh / (ev * ev + lam * lam), type=2, norm="ortho")


def reflexive_band(f: np.ndarray, n: int) -> np.ndarray:
    """R(f) = sum_d f[h+d] R_d (Toeplitz plus Hankel near the borders)."""
    k = f.shape[0]
    h = (k - 1) // 2
    if k > n:
        raise ValueError("reflexive boundary needs K <= n")
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
    """Reflexive factors A_c = R(c), A_r = R(a) and their FP64 SVDs;
    A_hat X = A_c X A_r^T as for the zero boundary.  Any PSF with K <= n
    (the factors are non-symmetric when the profiles are not even)."""
    _check(psf, n, symmetric=False)
    c, a, s = kp_profiles(psf)
    ac = reflexive_band(c, n)
    ar = reflexive_band(a, n)
    uc, sc, vct = np.linalg.svd(ac)
    ur, sr, vrt = np.linalg.svd(ar)
    return kpmod.KPSVD(n=n, Ac=ac, Ar=ar, Uc=uc, sc=sc, Vc=vct.T, Ur=ur, sr=sr,
                       Vr=vrt.T, s_psf=s)


def exact_diag(kp: kpmod.KPSVD, psf: np.ndarray, rel: float = 1e-12) -> np.ndarray:
    """D0[i, j] = ||A (v_c,i v_r,j^T)||_F^2 through the reflexive Kronecker
    sum (as kp.exact_diag with reflexive factors)."""
    n = kp.n
    u, s, vt = np.linalg.svd(np.asarray(psf, dtype=np.float64))
    t = kpmod.kp_terms(s, rel)
    B = [reflexive_band(np.sqrt(s[i]) * u[:, i], n) @ kp.Vc for i in range(t)]
    C = [reflexive_band(np.sqrt(s[i]) * vt[i, :], n) @ kp.Vr for i in range(t)]
    d0 = np.zeros((n, n))
    for k in range(t):
        for l in range(t):
            d0 += np.outer(np.sum(B[k] * B[l], axis=0), np.sum(C[k] * C[l], axis=0))
    return d0


class NormalOperator:
    """H_lambda = A^T A + lambda^2 I (= A^2 + lambda^2 I) for the reflexive
    boundary, interface of solvers.NormalOperator; the DCT form above 64."""

    def __init__(self, psf: np.ndarray, n: int, lam: float, use_dct: bool | None = None):
        _check(psf, n)
        self.psf, self.n, self.lam = psf, n, float(lam)
        self.use_dct = n > 64 if use_dct is None else use_dct
        self._ev = eigenvalues(psf, n) if self.use_dct else None

    def A(self, x):
        if self._ev is None:
            return blur(self.psf, x)
        return scipy.fft.idctn(self._ev * scipy.fft.dctn(x, type=2, norm="ortho"), type=2,
                               norm="ortho")

    def At(self, y):
        return self.A(y)

    def H(self, x):
        return self.At(self.A(x)) + self.lam * self.lam * x


class NormalOperatorGeneral:
    """H_lambda = A^T A + lambda^2 I for the reflexive boundary and any PSF
    (K <= n), interface of solvers.NormalOperator: the definitions for
    n <= 64, their FFT forms above."""

    def __init__(self, psf: np.ndarray, n: int, lam: float, use_fft: bool | None = None):
        _check(psf, n, symmetric=False)
        self.psf, self.n, self.lam = psf, n, float(lam)
        self.use_fft = n > 64 if use_fft is None else use_fft

    def A(self, x):
        return blur_fft_general(self.psf, x) if self.use_fft else blur_general(self.psf, x)

    def At(self, y):
        return blur_t_fft_general(self.psf, y) if self.use_fft else blur_t_general(self.psf, y)

    def H(self, x):
        return self.At(self.A(x)) + self.lam * self.lam * x


def x_lambda_dense_general(psf: np.ndarray, b: np.ndarray, lam: float) -> np.ndarray:
    """The Tikhonov minimiser by a dense Cholesky solve of eq. (tik:normal2)
    (tiny n)."""
    import scipy.linalg
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    a = dense_matrix(psf, n)
    h = a.T @ a + lam * lam * np.eye(n * n)
    rhs = a.T @ b.reshape(-1, order="F")
    return scipy.linalg.cho_solve(scipy.linalg.cho_factor(h), rhs).reshape((n, n), order="F")


def x_lambda_general(psf: np.ndarray, b: np.ndarray, lam: float, tol: float = 1e-13,
                     maxit: int = 20000, check: bool = True):
    """x_lambda for any PSF under the reflexive boundary: FP64 PCG with the
    one-term reflexive KP preconditioner to a true relative residual of
    `tol`; with `check`, a run at a 100x looser tolerance must agree to
    1e-7 relative (else ValueError).  Returns (x, info dict)."""
    from . import solvers as sv
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    op = NormalOperatorGeneral(psf, n, lam)
    kp = kp_svd(psf, n)

    def pre(r):
        return kpmod.precond_solve(kp, lam, r)
    out = sv.solve(op, b, mode=sv.PCG, tol=tol, maxit=maxit, precond=pre)
    c = op.At(b)
    info = {"iters": out.iters, "status": out.status,
            "true_relres": float(np.linalg.norm(c - op.H(out.x)) / np.linalg.norm(c))}
    if check:
        loose = sv.solve(op, b, mode=sv.PCG, tol=tol * 100, maxit=maxit, precond=pre)
        agree = float(np.linalg.norm(loose.x - out.x) / np.linalg.norm(out.x))
        info["loose_agreement"] = agree
        if agree > 1e-7:
            raise ValueError(f"x_lambda not settled: loose vs tight differ by {agree:.2e}")
    return out.x, info
