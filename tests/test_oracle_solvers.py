"""Pins for the oracle's CG / PCG / FPCG and its exact x_lambda."""
import math

import numpy as np
import pytest
import scipy.signal

import synthetic as S
from oracle import kp as KP
from oracle import operator as O
from oracle import quant as Q
from oracle import solvers as SV


def _library_dense_a(psf, n):
    """Dense A built from scipy.signal.convolve2d on unit images (column-major
    vec), independent of the oracle's operator code."""
    N = n * n
    a = np.zeros((N, N))
    for q in range(N):
        e = np.zeros(N)
        e[q] = 1.0
        img = e.reshape((n, n), order="F")
        a[:, q] = scipy.signal.convolve2d(img, psf, mode="same").reshape(-1, order="F")
    return a


def _small_problem(n, k, seed, sep=False):
    rng = np.random.default_rng(seed)
    if sep:
        g = np.exp(-np.arange(-(k // 2), k // 2 + 1) ** 2 / 3.0)
        f = np.exp(-np.arange(-(k // 2), k // 2 + 1) ** 2 / 5.0)
        psf = np.outer(g, f)
        psf /= psf.sum()
    else:
        psf = S.psf_moffat_motion(k, 2.0, 2.5, 3.0, 0.9)
    x = S.true_image(rng, n)
    b = O.blur(psf, x) + 0.01 * rng.standard_normal((n, n))
    return psf, x, b


@pytest.mark.parametrize("sep", [False, True])
def test_x_lambda_dense_equals_stacked_least_squares(sep):
    """eq. (lsp:Tik): x_lambda minimises || [b; 0] - [A; lambda I] x ||,
    solved here by LAPACK least squares on the stacked dense system."""
    n, k, lam = 8, 5, 0.05
    psf, _, b = _small_problem(n, k, 1, sep)
    a = _library_dense_a(psf, n)
    stacked = np.vstack([a, lam * np.eye(n * n)])
    rhs = np.concatenate([O.vec(b), np.zeros(n * n)])
    ref = np.linalg.lstsq(stacked, rhs, rcond=None)[0]
    x = O.vec(SV.x_lambda_dense(psf, b, lam))
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_separable_closed_form_equals_dense():
    """eq. (eq:TikSV) with the exact Kronecker SVD equals the dense solve."""
    n, k, lam = 9, 5, 0.03
    psf, _, b = _small_problem(n, k, 2, sep=True)
    x1 = SV.x_lambda_separable(psf, b, lam)
    x2 = SV.x_lambda_dense(psf, b, lam)
    assert np.linalg.norm(x1 - x2) <= 1e-11 * np.linalg.norm(x2)


@pytest.mark.parametrize("mode", [SV.CG, SV.PCG, SV.FPCG])
def test_iterative_modes_reach_dense_solution(mode):
    n, k, lam = 16, 5, 0.02
    psf, _, b = _small_problem(n, k, 3)
    ref = SV.x_lambda_dense(psf, b, lam)
    op = SV.NormalOperator(psf, n, lam)
    pre = SV.kp_preconditioner(psf, n, lam)
    out = SV.solve(op, b, mode=mode, tol=1e-12, maxit=2000, precond=pre)
    assert out.status == "converged"
    assert np.linalg.norm(out.x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_x_lambda_iterative_equals_dense():
    n, k, lam = 20, 7, 0.01
    psf, _, b = _small_problem(n, k, 4)
    ref = SV.x_lambda_dense(psf, b, lam)
    x, info = SV.x_lambda_iterative(psf, b, lam)
    assert info["true_relres"] < 1e-12
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_one_iteration_with_exact_preconditioner():
    """Separable PSF + exact FP64 KP preconditioner: M = H_lambda, so PCG
    stops after one iteration with alpha = 1 and x_1 = x_lambda (Section 5.3:
    the Gaussian case, where the only approximation is precision)."""
    n, k, lam = 24, 7, 0.02
    psf, _, b = _small_problem(n, k, 5, sep=True)
    op = SV.NormalOperator(psf, n, lam)
    out = SV.solve(op, b, mode=SV.PCG, tol=1e-10, maxit=10,
                   precond=SV.kp_preconditioner(psf, n, lam))
    assert out.iters == 1 and out.status == "converged"
    assert abs(out.alphas[0] - 1.0) < 1e-12
    ref = SV.x_lambda_separable(psf, b, lam)
    assert np.linalg.norm(out.x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_gaussian_fp16_preconditioner_converges_at_second_iteration():
    """Section 5.3 (Gaussian blur, one Kronecker term): with the
    half-precision KP preconditioner the relative error ||x_k - x_true|| /
    ||x_true|| settles at the second iteration; with the exact FP64
    preconditioner it settles at the first.  Emulated FP16 chain, 128^2."""
    p = S.small_gaussian(0, n=128)
    kp = KP.kp_svd(p.psf, p.n)
    op = SV.NormalOperator(p.psf, p.n, p.lam)
    pre16 = lambda r: Q.precond_fp16(kp.Vc, kp.Vr, kp.sc, kp.sr, p.lam, r)
    out16 = SV.solve(op, p.b, mode=SV.PCG, tol=1e-9, maxit=20, precond=pre16,
                     x_true=p.x_true)
    out64 = SV.solve(op, p.b, mode=SV.PCG, tol=1e-9, maxit=20,
                     precond=SV.kp_preconditioner(p.psf, p.n, p.lam, kp),
                     x_true=p.x_true)
    final = out64.errors[-1]
    assert out64.iters == 1
    assert abs(out16.errors[2] - final) <= 1e-4 * final
    assert abs(out16.errors[1] - final) > 0.1 * final


@pytest.mark.parametrize("mode", [SV.CG, SV.PCG, SV.FPCG])
def test_energy_is_monotone(mode):
    """phi(x_k) = 1/2 x^T H x - x^T c never increases (CG minimises the
    H-norm of the error over a growing Krylov space; both beta formulas
    keep r_{k+1} orthogonal to p_k)."""
    n, k, lam = 24, 7, 0.01
    psf, _, b = _small_problem(n, k, 6)
    op = SV.NormalOperator(psf, n, lam)
    out = SV.solve(op, b, mode=mode, tol=1e-10, maxit=200,
                   precond=SV.kp_preconditioner(psf, n, lam), track_energy=True)
    e = np.asarray(out.energies)
    assert np.all(np.diff(e) <= 1e-12 * np.abs(e).max())
    assert out.iters >= 2


def test_flexible_beta_equals_h_orthogonalisation():
    """Polak-Ribiere beta = (r1.z1 - r0.z1)/(r0.z0) equals -alpha (z1.Hp0)/
    (r0.z0) = -(z1.Hp0)/(p0.Hp0) when r1 = r0 - alpha H p0 (the flexible-CG
    direction update); checked along a run with an inexact preconditioner."""
    n, k, lam = 20, 5, 0.02
    psf, _, b = _small_problem(n, k, 7)
    kp = KP.kp_svd(psf, n)
    op = SV.NormalOperator(psf, n, lam)
    pre = lambda r: Q.precond_fp16(kp.Vc, kp.Vr, kp.sc, kp.sr, lam, r)
    c = op.At(b)
    r = c.copy()
    z = pre(r)
    rho = np.sum(r * z)
    p = z.copy()
    for _ in range(5):
        w = op.H(p)
        delta = np.sum(p * w)
        alpha = rho / delta
        r_new = r - alpha * w
        z_new = pre(r_new)
        pr = (np.sum(r_new * z_new) - np.sum(r * z_new)) / rho
        alt = -np.sum(z_new * w) / delta
        assert abs(pr - alt) <= 1e-9 * (abs(pr) + 1e-300)
        r, z = r_new, z_new
        rho = np.sum(r * z)
        p = z + pr * p


def test_zero_rhs_returns_zero():
    psf = S.psf_gaussian(5, 1.0, 1.0)
    op = SV.NormalOperator(psf, 8, 0.1)
    out = SV.solve(op, np.zeros((8, 8)), mode=SV.PCG)
    assert out.status == "zero" and out.iters == 0 and not out.x.any()


def test_work_unit_break_even_fixture():
    """Section 5.2's break-even ratio follows from its cost model."""
    vals = {}
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "work_unit_break_even.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                key, v = line.split()
                vals[key] = float(v)
    mv, pc = vals["matvecs_per_iteration"], vals["preconditioner_cost_in_matvecs"]
    assert math.isclose(mv / (mv + pc), vals["break_even_ratio"], rel_tol=1e-12)


@pytest.mark.parametrize("mode", [SV.CG, SV.PCG])
def test_residual_history_equals_krylov_galerkin_iterates(mode):
    """The recurrence norms resnorms[k] are ||c - H x_k|| of the k-th
    (P)CG iterate, which for SPD H and M is the Galerkin solution on the
    Krylov space K_k(M^-1 H, M^-1 c): x_k = Q (Q^T H Q)^-1 Q^T c with Q an
    orthonormal basis of that space (textbook characterisation, here formed
    densely with scipy-built H, independent of the solver's recurrences)."""
    n, k, lam = 8, 5, 0.1
    psf, _, b = _small_problem(n, k, 21)
    N = n * n
    a = _library_dense_a(psf, n)
    h = a.T @ a + lam * lam * np.eye(N)
    c = a.T @ b.reshape(-1, order="F")
    op = SV.NormalOperator(psf, n, lam)
    if mode == SV.CG:
        minv = np.eye(N)
        pre = None
    else:
        kp = KP.kp_svd(psf, n)
        pre = SV.kp_preconditioner(psf, n, lam, kp)
        minv = np.column_stack([pre(np.eye(N)[:, q].reshape((n, n), order="F"))
                                .reshape(-1, order="F") for q in range(N)])
    out = SV.solve(op, b, mode=mode, tol=1e-14, maxit=8, precond=pre)
    g = minv @ h
    v = minv @ c
    for it in range(1, min(7, out.iters + 1)):
        kry = np.column_stack([np.linalg.matrix_power(g, j) @ v for j in range(it)])
        q, _ = np.linalg.qr(kry)
        xk = q @ np.linalg.solve(q.T @ h @ q, q.T @ c)
        ref = np.linalg.norm(c - h @ xk)
        assert abs(out.resnorms[it] - ref) <= 1e-7 * out.resnorms[0], (it, out.resnorms[it], ref)
    assert out.resnorms[0] == pytest.approx(np.linalg.norm(c), rel=1e-12)
