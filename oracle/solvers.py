"""CG, PCG and flexible PCG on the Tikhonov normal equations, in FP64, and
the exact Tikhonov minimiser x_lambda.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed:
  * eq. (lsp:Tik) / eq. (eq:Tik): x_lambda minimises ||b - A x||^2 +
    lambda^2 ||x||^2, equivalently solves the normal equations
    (A^T A + lambda^2 I) x = A^T b, eq. (tik:normal1) / (tik:normal2);
  * eq. (eq:TikSV): x = sum_i phi_i (u_i^T b / s_i) v_i with
    phi_i = s_i^2 / (s_i^2 + lambda^2);
  * Section 2.3: PCG with M = A_hat^T A_hat + lambda^2 I (eq. (PreconSystem));
  * Section 3 (last paragraph) and Section 5.2: standard PCG uses the
    Fletcher-Reeves update of the search direction; flexible PCG uses the
    Polak-Ribiere update, at the price of one more inner product and one
    more stored vector (the previous residual).

The paper does not state x_0, the stopping rule or the iteration itself.
Reading used: x_0 = 0, r_0 = A^T b, stop when ||r_k|| <= tol ||r_0|| (a
relative normal-equation residual), and the textbook PCG recurrence.

Exact x_lambda (the parity target) comes from three independent routes:
  * dense Cholesky of H_lambda (tiny images);
  * the SVD filter formula (eq. (eq:TikSV)) with the exact Kronecker SVD
    when the PSF is separable, where A = A_r (x) A_c exactly;
  * otherwise FP64 PCG iterated until the true residual reaches 1e-13 of
    ||A^T b|| or stagnates.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg

from . import kp as kpmod
from .operator import FFTBlur, blur, blur_t, dense_matrix, unvec, vec

CG, PCG, FPCG = "cg", "pcg", "fpcg"


@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    status: str                 # 'converged' | 'maxit' | 'breakdown' | 'zero'
    resnorms: list              # ||r_k|| (recurrence), k = 0..iters
    energies: list              # phi(x_k) = 1/2 x^T H x - x^T c
    errors: list                # ||x_k - x_true|| / ||x_true|| if x_true given
    alphas: list


class NormalOperator:
    """H_lambda = A^T A + lambda^2 I and c = A^T b for one problem."""

    def __init__(self, psf: np.ndarray, n: int, lam: float, use_fft: bool | None = None,
                 workers: int | None = None):
        self.psf, self.n, self.lam = psf, n, float(lam)
        if use_fft is None:
            use_fft = n > 64
        self.fft = FFTBlur(psf, n, workers=workers) if use_fft else None

    def A(self, x):
        return self.fft.blur(x) if self.fft is not None else blur(self.psf, x)

    def At(self, y):
        return self.fft.blur_t(y) if self.fft is not None else blur_t(self.psf, y)

    def H(self, x):
        return self.At(self.A(x)) + self.lam * self.lam * x


def solve(op: NormalOperator, b: np.ndarray, mode: str = PCG, tol: float = 1e-6,
          maxit: int = 1000, precond=None, x_true: np.ndarray | None = None,
          track_energy: bool = False) -> SolveResult:
    """CG / PCG (Fletcher-Reeves) / flexible PCG (Polak-Ribiere) from x_0 = 0.

    `precond(r)` returns z = M^{-1} r; it is ignored for mode 'cg'.  In
    'fpcg' the previous residual is kept and beta = (r_new . z_new -
    r_old . z_new) / (r_old . z_old)."""
    b = np.asarray(b, dtype=np.float64)
    c = op.At(b)
    n = op.n
    x = np.zeros((n, n))
    r = c.copy()
    gamma0 = float(np.linalg.norm(r))
    res = SolveResult(x=x, iters=0, status="zero", resnorms=[gamma0], energies=[],
                      errors=[], alphas=[])
    xt_norm = None if x_true is None else float(np.linalg.norm(x_true))
    if x_true is not None:
        res.errors.append(float(np.linalg.norm(x - x_true) / xt_norm))
    if track_energy:
        res.energies.append(0.0)
    if gamma0 == 0.0:
        return res
    pre = (lambda v: v) if (mode == CG or precond is None) else precond
    z = pre(r)
    rho = float(np.sum(r * z))
    p = z.copy()
    res.status = "maxit"
    for k in range(maxit):
        w = op.H(p)
        delta = float(np.sum(p * w))
        if not (delta > 0.0) or not math.isfinite(delta):
            res.status = "breakdown"
            break
        alpha = rho / delta
        res.alphas.append(alpha)
        x = x + alpha * p
        r_old = r if mode == FPCG else None
        r = r - alpha * w
        rn = float(np.linalg.norm(r))
        res.resnorms.append(rn)
        res.iters = k + 1
        if x_true is not None:
            res.errors.append(float(np.linalg.norm(x - x_true) / xt_norm))
        if track_energy:
            res.energies.append(float(0.5 * np.sum(x * op.H(x)) - np.sum(x * c)))
        if rn <= tol * gamma0:
            res.status = "converged"
            break
        z = pre(r)
        rho_new = float(np.sum(r * z))
        if not (rho_new > 0.0) or not math.isfinite(rho_new):
            res.status = "breakdown"
            break
        if mode == FPCG:
            beta = (rho_new - float(np.sum(r_old * z))) / rho
        else:
            beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
    res.x = x
    return res


def kp_preconditioner(psf: np.ndarray, n: int, lam: float, kp: kpmod.KPSVD | None = None,
                      exact_diag: bool = False):
    """z = M^{-1} r with the exact FP64 KP-SVD factors; exact_diag uses
    S = 1 / (diag(V^T A^T A V) + lambda^2) (kp.exact_diag) instead of the
    one-term singular values."""
    kp = kp if kp is not None else kpmod.kp_svd(psf, n)
    d0 = kpmod.exact_diag(kp, psf) if exact_diag else None
    return lambda r: kpmod.precond_solve(kp, lam, r, d0)


def true_residual(op: NormalOperator, b: np.ndarray, x: np.ndarray) -> float:
    """||A^T b - H x|| / ||A^T b||."""
    c = op.At(np.asarray(b, dtype=np.float64))
    return float(np.linalg.norm(c - op.H(x)) / np.linalg.norm(c))


# --------------------------------------------------------------------------
# exact Tikhonov minimiser
# --------------------------------------------------------------------------

def x_lambda_dense(psf: np.ndarray, b: np.ndarray, lam: float) -> np.ndarray:
    """Dense Cholesky solve of (A^T A + lambda^2 I) x = A^T b (tiny n only)."""
    n = b.shape[0]
    a = dense_matrix(psf, n)
    h = a.T @ a + lam * lam * np.eye(n * n)
    rhs = a.T @ vec(np.asarray(b, dtype=np.float64))
    cf = scipy.linalg.cho_factor(h)
    return unvec(scipy.linalg.cho_solve(cf, rhs), n)


def x_lambda_separable(psf: np.ndarray, b: np.ndarray, lam: float,
                       kp: kpmod.KPSVD | None = None) -> np.ndarray:
    """SVD filter solution (eq. (eq:TikSV)) with A = A_r (x) A_c, exact when
    the PSF is rank one:  X = V_c (F .* (U_c^T B U_r)) V_r^T,
    F[i,j] = s_ij / (s_ij^2 + lambda^2), s_ij = s_c[i] s_r[j]."""
    n = b.shape[0]
    kp = kp if kp is not None else kpmod.kp_svd(psf, n)
    s = kp.sigma()
    bhat = kp.Uc.T @ np.asarray(b, dtype=np.float64) @ kp.Ur
    return kp.Vc @ (s / (s * s + lam * lam) * bhat) @ kp.Vr.T


def x_lambda_iterative(psf: np.ndarray, b: np.ndarray, lam: float, tol: float = 1e-13,
                       maxit: int = 20000, kp: kpmod.KPSVD | None = None,
                       workers: int | None = None, check: bool = True):
    """FP64 KP-preconditioned CG iterated to a true relative residual of
    `tol` or until the recurrence stagnates.  With `check`, a second run at a
    100x looser tolerance must agree to 1e-7 relative, else ValueError.
    Returns (x, info dict)."""
    n = b.shape[0]
    op = NormalOperator(psf, n, lam, workers=workers)
    kp = kp if kp is not None else kpmod.kp_svd(psf, n)
    pre = kp_preconditioner(psf, n, lam, kp)
    out = solve(op, b, mode=PCG, tol=tol, maxit=maxit, precond=pre)
    info = {"iters": out.iters, "status": out.status,
            "true_relres": true_residual(op, b, out.x)}
    if check:
        loose = solve(op, b, mode=PCG, tol=tol * 100, maxit=maxit, precond=pre)
        agree = float(np.linalg.norm(loose.x - out.x) / np.linalg.norm(out.x))
        info["loose_agreement"] = agree
        if agree > 1e-7:
            raise ValueError(f"x_lambda not settled: loose vs tight differ by {agree:.2e}")
    return out.x, info


def x_lambda(psf: np.ndarray, b: np.ndarray, lam: float, workers: int | None = None):
    """Best available exact x_lambda for the problem: dense Cholesky for
    n <= 32, else settled FP64 PCG.  (Float32-rounded PSFs are never exactly
    rank one, so the separable closed form serves as a pin, not a target.)"""
    n = b.shape[0]
    if n <= 32:
        return x_lambda_dense(psf, b, lam)
    return x_lambda_iterative(psf, b, lam, workers=workers)[0]
