"""Regularisation-parameter rules in a spectral basis, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed (Section 2.2), with b_hat = U^T b, x_hat = V^T x_true
and singular values s_i of the operator:
  * eq. (OptTikSVD):  O(lambda)   = sum_i (s_i b_hat_i / (s_i^2 + lambda^2) - x_hat_i)^2
  * eq. (GCVTikSVD):  G(lambda)   = N sum_i (b_hat_i / (s_i^2+lambda^2))^2
                                    / (sum_i 1 / (s_i^2 + lambda^2))^2
  * eq. (wGCVTikSVD): G_w(lambda) = N sum_i (lambda^2 b_hat_i / (s_i^2+lambda^2))^2
                                    / (sum_i ((1-w) s_i^2 + lambda^2) / (s_i^2+lambda^2))^2
  * eq. (DSCTikSVD):  D(lambda)   = sum_i (lambda^2 b_hat_i / (s_i^2+lambda^2))^2 - eps^2,
                                    eps = eta ||noise||
  * eq. (GCVTik): the trace form of GCV, used here only to pin the SVD form.

Section 5.1 evaluates them with the Kronecker approximation's SVD in place
of the SVD of A: s_ij = s_c[i] s_r[j], b_hat = U_c^T B U_r,
x_hat = V_c^T X_true V_r.  The "n" in the GCV numerator is read as the number
of data points N (it only scales G).  The paper minimises with fminbnd and
roots D with fzero; here every rule is evaluated on a grid, argmin ties go to
the smallest grid index, and the discrepancy root on a grid is the largest
grid lambda with D <= 0.  Parity: pinned by the trace form and the dense SVD
of A on tiny separable problems, and by D's monotonicity.
"""
from __future__ import annotations

import numpy as np

from . import kp as kpmod
from .operator import dense_matrix, vec


def spectrum(kp: kpmod.KPSVD, b: np.ndarray):
    """(s2, bhat2): s_ij^2 and b_hat_ij^2 in the KP basis, as flat arrays."""
    s = kp.sigma()
    bhat = kp.Uc.T @ np.asarray(b, dtype=np.float64) @ kp.Ur
    return (s * s).ravel(), (bhat * bhat).ravel()


def gcv(s2, bhat2, lams, omega: float = 1.0):
    """G_w on each grid lambda (G for omega = 1), eq. (wGCVTikSVD).

    For omega > 1 the trace term T(lambda) = sum((1 - omega) s^2 + lambda^2)
    / (s^2 + lambda^2) increases with lambda and is negative below some
    lambda_0, where G_w falls back towards 0 as lambda -> 0.  The paper
    minimises G_w on a bracket (Section 2.2) without naming the branch; the
    reading taken: only the branch T > 0, continuous with large lambda, is
    admissible, and G_w is +inf elsewhere (never for omega <= 1)."""
    s2 = np.asarray(s2, dtype=np.float64)
    bhat2 = np.asarray(bhat2, dtype=np.float64)
    N = s2.size
    out = []
    for lam in np.atleast_1d(lams):
        l2 = lam * lam
        den = s2 + l2
        num = N * np.sum(l2 * l2 * bhat2 / (den * den))
        tr = np.sum(((1.0 - omega) * s2 + l2) / den)
        out.append(num / (tr * tr) if tr > 0.0 else np.inf)
    return np.asarray(out)


def gcv_unweighted_form(s2, bhat2, lams):
    """G as printed in eq. (GCVTikSVD) (the lambda^4 factors cancelled)."""
    s2 = np.asarray(s2, dtype=np.float64)
    N = s2.size
    out = []
    for lam in np.atleast_1d(lams):
        den = s2 + lam * lam
        out.append(N * np.sum(bhat2 / (den * den)) / np.sum(1.0 / den) ** 2)
    return np.asarray(out)


def discrepancy(s2, bhat2, lams, eps: float):
    """D on each grid lambda, eq. (DSCTikSVD); eps = eta * ||noise||."""
    s2 = np.asarray(s2, dtype=np.float64)
    out = []
    for lam in np.atleast_1d(lams):
        l2 = lam * lam
        out.append(np.sum(l2 * l2 * bhat2 / (s2 + l2) ** 2) - eps * eps)
    return np.asarray(out)


def optimal_error(kp: kpmod.KPSVD, b: np.ndarray, x_true: np.ndarray, lams):
    """O on each grid lambda, eq. (OptTikSVD), in the KP basis."""
    s = kp.sigma().ravel()
    bhat = (kp.Uc.T @ np.asarray(b, dtype=np.float64) @ kp.Ur).ravel()
    xhat = (kp.Vc.T @ np.asarray(x_true, dtype=np.float64) @ kp.Vr).ravel()
    out = []
    for lam in np.atleast_1d(lams):
        out.append(np.sum((s * bhat / (s * s + lam * lam) - xhat) ** 2))
    return np.asarray(out)


def grid_argmin(scores) -> int:
    """Index of the smallest score; ties go to the smallest index."""
    return int(np.argmin(np.asarray(scores)))


def grid_discrepancy(dvals) -> int:
    """Largest grid index with D <= 0 (D increases with lambda), else 0."""
    d = np.asarray(dvals)
    idx = np.nonzero(d <= 0.0)[0]
    return int(idx[-1]) if idx.size else 0


def discrepancy_root(s2, bhat2, eps: float, lo: float = 1e-8, hi: float = 1e2,
                     iters: int = 200) -> float:
    """Root of D by bisection in log(lambda) (the fzero step of Section 2.2)."""
    f = lambda lam: discrepancy(s2, bhat2, [lam], eps)[0]
    flo, fhi = f(lo), f(hi)
    if flo > 0 or fhi < 0:
        raise ValueError("discrepancy root not bracketed")
    a, b = np.log(lo), np.log(hi)
    for _ in range(iters):
        m = 0.5 * (a + b)
        if f(np.exp(m)) > 0:
            b = m
        else:
            a = m
    return float(np.exp(0.5 * (a + b)))


# --------------------------------------------------------------------------
# dense forms (tiny problems only), used to pin the spectral forms
# --------------------------------------------------------------------------

def gcv_trace_form(psf: np.ndarray, b: np.ndarray, lam: float, omega: float = 1.0) -> float:
    """Eq. (GCVTik)/(wGCVTik) with the dense influence matrix
    A A_lambda^+ = A (A^T A + lambda^2 I)^{-1} A^T; +inf where the trace of
    I - omega A A_lambda^+ is not positive (the branch rule of gcv)."""
    n = b.shape[0]
    N = n * n
    a = dense_matrix(psf, n)
    infl = a @ np.linalg.solve(a.T @ a + lam * lam * np.eye(N), a.T)
    bv = vec(np.asarray(b, dtype=np.float64))
    res = bv - infl @ bv
    tr = np.trace(np.eye(N) - omega * infl)
    return float(N * (res @ res) / tr ** 2) if tr > 0.0 else float("inf")


def dense_spectrum(psf: np.ndarray, b: np.ndarray):
    """(s2, bhat2) from the dense SVD of A."""
    n = b.shape[0]
    a = dense_matrix(psf, n)
    u, s, vt = np.linalg.svd(a)
    bhat = u.T @ vec(np.asarray(b, dtype=np.float64))
    return s * s, bhat * bhat
