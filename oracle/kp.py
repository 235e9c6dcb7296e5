"""One-term Kronecker approximation of the blur and the KP-SVD preconditioner.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed:
  * Section 3, eq. (AKronSVD): A ~ A_r (x) A_c = (U_r (x) U_c)(S_r (x) S_c)
    (V_r (x) V_c)^T with A_r = U_r S_r V_r^T, A_c = U_c S_c V_c^T computed in
    double precision;
  * Section 5, eq. (KronSumDecomp): the term used is the Frobenius-optimal
    A_r (x) A_c = argmin ||A - A_r (x) A_c||_F, and ||A - A_hat||_F / ||A||_F
    measures its quality (Table 1);
  * Section 2.3, eq. (PreconSystem) and Section 3, eq. (PreconSolve):
    M = A_hat^T A_hat + lambda^2 I, solved as
    Z = V_c (S .* (V_c^T R V_r)) V_r^T with vec(S) = diag(D^{-1}),
    S[i, j] = 1 / (s_c[i]^2 s_r[j]^2 + lambda^2).

The paper cites IR Tools for the construction of the optimal term and does
not state it.  The reading used here: A = sum_{u,v} P[h+u,h+v] Z_v (x) Z_u
where Z_d is the n x n shift matrix Z_d[i,i'] = [i - i' = d].  The Z_d (x) Z_e
have disjoint supports with ||Z_d||_F^2 = n - |d|, so for Toeplitz factors
T(a) (x) T(c),

    ||A - T(a) (x) T(c)||_F^2 = sum_{u,v} w_u w_v (P[u,v] - c_u a_v)^2,
    w_k = n - |k - h|,

whose minimiser is the leading singular triple of W^{1/2} P W^{1/2}:
c = sqrt(s1) u1 / sqrt(w), a = sqrt(s1) v1 / sqrt(w).  Pinned against the
brute-force Van Loan-Pitsianis construction (SVD of the rearranged dense A)
on tiny images, and against exactness for separable PSFs.

Column factor A_c = T(c) acts from the left (vertical, row index i), row
factor A_r = T(a) from the right (horizontal), so A_hat X = A_c X A_r^T.

Exact diagonal in the KP basis (an extension of the paper's preconditioner):
the same weighted SVD gives all terms of eq. (KronSumDecomp),
A = sum_k T(a_k) (x) T(c_k) with c_k = sqrt(s_k) u_k / sqrt(w),
a_k = sqrt(s_k) v_k / sqrt(w), exact once every nonzero s_k is kept (the
paper reports 9 and 10 terms for its motion and shake blurs, Section 5, where
the one-term preconditioner helps least).  Keeping V = V_r (x) V_c from the
leading term, the diagonal of V^T A^T A V is, for basis image
E_ij = v_c,i v_r,j^T,

    D0[i, j] = ||A E_ij||_F^2
             = sum_{k,l} (B_k^T B_l)[i, i] (C_k^T C_l)[j, j],
    B_k = T(c_k) V_c,  C_k = T(a_k) V_r,

and S[i, j] = 1 / (D0[i, j] + lambda^2) replaces 1 / (s_c[i]^2 s_r[j]^2 +
lambda^2) in eq. (PreconSolve): the Frobenius-nearest matrix to H_lambda of
the form V diag(.) V^T.  With one term D0 = s_c^2 s_r^2 exactly.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def weights(k: int, n: int) -> np.ndarray:
    h = (k - 1) // 2
    return n - np.abs(np.arange(k) - h).astype(np.float64)


def kp_profiles(psf: np.ndarray, n: int):
    """Return (c, a, s): column profile c (length K), row profile a, and the
    singular values s of the weighted PSF W^{1/2} P W^{1/2}.

    Sign convention: sum(c) > 0 (the split of sign and scale between the two
    factors does not change A_hat)."""
    k = psf.shape[0]
    w = weights(k, n)
    sw = np.sqrt(w)
    pw = sw[:, None] * psf * sw[None, :]
    u, s, vt = np.linalg.svd(pw)
    c = np.sqrt(s[0]) * u[:, 0] / sw
    a = np.sqrt(s[0]) * vt[0, :] / sw
    if c.sum() < 0:
        c, a = -c, -a
    return c, a, s


def toeplitz_band(f: np.ndarray, n: int) -> np.ndarray:
    """T(f)[i, i'] = f[h + i - i'] for |i - i'| <= h, else 0."""
    k = f.shape[0]
    h = (k - 1) // 2
    t = np.zeros((n, n))
    for d in range(-h, h + 1):
        idx = np.arange(max(0, d), min(n, n + d))
        t[idx, idx - d] = f[h + d]
    return t


def kp_error(s: np.ndarray) -> float:
    """||A - A_hat||_F / ||A||_F from the weighted-PSF singular values
    (Table 1's quality measure), without cancellation."""
    s = np.asarray(s, dtype=np.float64)
    return float(np.sqrt(np.sum(s[1:] ** 2) / np.sum(s ** 2)))


def kp_terms(s: np.ndarray, rel: float = 1e-12) -> int:
    """Number of Kronecker terms in the exact decomposition (Table 1's k):
    the numerical rank of the weighted PSF."""
    s = np.asarray(s)
    return int(np.sum(s > rel * s[0]))


@dataclasses.dataclass
class KPSVD:
    n: int
    Ac: np.ndarray
    Ar: np.ndarray
    Uc: np.ndarray
    sc: np.ndarray
    Vc: np.ndarray
    Ur: np.ndarray
    sr: np.ndarray
    Vr: np.ndarray
    s_psf: np.ndarray

    def sigma(self) -> np.ndarray:
        """sigma[i, j] = s_c[i] s_r[j], the singular values of A_hat laid out
        like an image."""
        return np.outer(self.sc, self.sr)


def kp_svd(psf: np.ndarray, n: int) -> KPSVD:
    """Factors and their FP64 SVDs (eq. (AKronSVD))."""
    c, a, s = kp_profiles(psf, n)
    ac = toeplitz_band(c, n)
    ar = toeplitz_band(a, n)
    uc, sc, vct = np.linalg.svd(ac)
    ur, sr, vrt = np.linalg.svd(ar)
    return KPSVD(n=n, Ac=ac, Ar=ar, Uc=uc, sc=sc, Vc=vct.T, Ur=ur, sr=sr,
                 Vr=vrt.T, s_psf=s)


def fp16_factor(t: np.ndarray) -> np.ndarray:
    """A factor as the reduced-precision construction sees it: scaled by the
    power of two 2^e that puts its largest |entry| in [2^13, 2^14), rounded
    to FP16 (round to nearest even), scaled back (exactly)."""
    mx = float(np.abs(t).max())
    if mx == 0.0:
        return np.zeros_like(t)
    e = 13 - int(np.floor(np.log2(mx)))
    return np.ldexp(np.ldexp(t, e).astype(np.float16).astype(np.float64), -e)


def kp_svd_fp16_factors(kp: KPSVD) -> KPSVD:
    """The exact (FP64) SVDs of the FP16-rounded factors of `kp`: what a
    half-precision construction of S, V_r and V_c (left to future work in
    Section 3) computes up to the rounding of its own SVD."""
    ac, ar = fp16_factor(kp.Ac), fp16_factor(kp.Ar)
    uc, sc, vct = np.linalg.svd(ac)
    ur, sr, vrt = np.linalg.svd(ar)
    return KPSVD(n=kp.n, Ac=ac, Ar=ar, Uc=uc, sc=sc, Vc=vct.T, Ur=ur, sr=sr,
                 Vr=vrt.T, s_psf=kp.s_psf)


def kp_apply(kp: KPSVD, x: np.ndarray) -> np.ndarray:
    """A_hat X = A_c X A_r^T."""
    return kp.Ac @ x @ kp.Ar.T


def precond_diag(kp: KPSVD, lam: float, d0: np.ndarray | None = None) -> np.ndarray:
    """S[i, j] = 1 / (s_c[i]^2 s_r[j]^2 + lambda^2), vec(S) = diag(D^{-1});
    with d0 (exact_diag) S[i, j] = 1 / (d0[i, j] + lambda^2)."""
    base = np.outer(kp.sc ** 2, kp.sr ** 2) if d0 is None else d0
    return 1.0 / (base + lam * lam)


def precond_solve(kp: KPSVD, lam: float, r: np.ndarray,
                  d0: np.ndarray | None = None) -> np.ndarray:
    """z = M^{-1} r as Z = V_c (S .* (V_c^T R V_r)) V_r^T (eq. (PreconSolve))."""
    t = kp.Vc.T @ r @ kp.Vr
    return kp.Vc @ (precond_diag(kp, lam, d0) * t) @ kp.Vr.T


def kp_all_terms(psf: np.ndarray, n: int, rel: float = 1e-12):
    """All terms of eq. (KronSumDecomp) from the weighted PSF SVD: lists of
    column profiles c_k and row profiles a_k with P = sum_k c_k a_k^T, for the
    singular values s_k > rel * s_1."""
    k = psf.shape[0]
    sw = np.sqrt(weights(k, n))
    u, s, vt = np.linalg.svd(sw[:, None] * psf * sw[None, :])
    t = kp_terms(s, rel)
    cs = [np.sqrt(s[i]) * u[:, i] / sw for i in range(t)]
    as_ = [np.sqrt(s[i]) * vt[i, :] / sw for i in range(t)]
    return cs, as_


def kron_sum_apply(cs, as_, x: np.ndarray) -> np.ndarray:
    """A X = sum_k T(c_k) X T(a_k)^T (eq. (KronSumDecomp) in matrix form)."""
    n = x.shape[0]
    return sum(toeplitz_band(c, n) @ x @ toeplitz_band(a, n).T for c, a in zip(cs, as_))


def exact_diag(kp: KPSVD, psf: np.ndarray, rel: float = 1e-12) -> np.ndarray:
    """D0[i, j] = ||A (v_c,i v_r,j^T)||_F^2 through the Kronecker sum:
    sum over term pairs (k, l) of the column dot products of B_k = T(c_k) V_c
    times those of C_k = T(a_k) V_r."""
    n = kp.n
    cs, as_ = kp_all_terms(psf, n, rel)
    B = [toeplitz_band(c, n) @ kp.Vc for c in cs]
    C = [toeplitz_band(a, n) @ kp.Vr for a in as_]
    d0 = np.zeros((n, n))
    for k in range(len(cs)):
        for l in range(len(cs)):
            d0 += np.outer(np.sum(B[k] * B[l], axis=0), np.sum(C[k] * C[l], axis=0))
    return d0


def van_loan_pitsianis(a_dense: np.ndarray, n: int):
    """Brute-force nearest Kronecker product B (x) C to a dense N x N matrix
    (Van Loan & Pitsianis): SVD of the rearrangement
    R(A)[(k,l) block, entries] = vec(A_{kl})^T.  Returns (B, C) with
    A ~ B (x) C.  Only for tiny n (used to pin kp_profiles)."""
    N = n * n
    blocks = a_dense.reshape(n, n, n, n)           # [k, i, l, j] -> A_{kl}[i,j]
    rmat = np.empty((n * n, n * n))
    for kk in range(n):
        for ll in range(n):
            rmat[ll * n + kk, :] = blocks[kk, :, ll, :].reshape(-1, order="F")
    u, s, vt = np.linalg.svd(rmat)
    bvec = np.sqrt(s[0]) * u[:, 0]
    cvec = np.sqrt(s[0]) * vt[0, :]
    B = bvec.reshape((n, n), order="F")
    C = cvec.reshape((n, n), order="F")
    assert B.size * C.size == N * N
    return B, C
