"""Pins of the reflexive-boundary oracle (oracle/reflexive.py) against a
library routine, closed forms and brute force."""
import numpy as np
import pytest
import scipy.ndimage

from oracle import kp as KP
from oracle import reflexive as RB
from oracle import solvers as SV


def _sym_psf(rng, k):
    """Non-separable PSF symmetric in both axes, unit sum."""
    p = rng.uniform(0, 1, (k, k))
    p = p + p[::-1, :] + p[:, ::-1] + p[::-1, ::-1]
    return p / p.sum()


@pytest.mark.parametrize("n,k", [(8, 3), (9, 5), (16, 15), (12, 11), (7, 7)])
def test_blur_equals_scipy_reflect(n, k):
    rng = np.random.default_rng(n * 17 + k)
    psf = _sym_psf(rng, k)
    x = rng.standard_normal((n, n))
    ref = scipy.ndimage.convolve(x, psf, mode="reflect")
    assert np.abs(RB.blur(psf, x) - ref).max() < 1e-12


def test_symmetric_and_constant_preserving():
    rng = np.random.default_rng(2)
    n, k = 7, 5
    psf = _sym_psf(rng, k)
    a = RB.dense_matrix(psf, n)
    assert np.abs(a - a.T).max() < 1e-14
    assert np.abs(RB.blur(psf, np.ones((n, n))) - psf.sum()).max() < 1e-13


def test_dense_equals_reflexive_kronecker_sum():
    rng = np.random.default_rng(3)
    n, k, h = 6, 5, 2
    psf = _sym_psf(rng, k)
    ref = sum(psf[h + u, h + v] * np.kron(RB.shift(v, n), RB.shift(u, n))
              for u in range(-h, h + 1) for v in range(-h, h + 1))
    assert np.abs(RB.dense_matrix(psf, n) - ref).max() < 1e-13


def test_dct_form_and_closed_form_solution():
    rng = np.random.default_rng(4)
    n, k, lam = 8, 5, 0.05
    psf = _sym_psf(rng, k)
    x = rng.standard_normal((n, n))
    assert np.abs(RB.blur_dct(psf, x) - RB.blur(psf, x)).max() < 1e-12
    b = rng.standard_normal((n, n))
    a = RB.dense_matrix(psf, n)
    xd = np.linalg.solve(a.T @ a + lam * lam * np.eye(n * n),
                         a.T @ b.reshape(-1, order="F")).reshape((n, n), order="F")
    assert np.abs(RB.x_lambda(psf, b, lam) - xd).max() < 1e-11 * np.abs(xd).max()


def test_kp_exact_for_separable_psf_and_expansion():
    rng = np.random.default_rng(5)
    n, k = 10, 7
    f = rng.uniform(0, 1, k)
    f = f + f[::-1]
    g = rng.uniform(0, 1, k)
    g = g + g[::-1]
    sep = np.outer(f, g)
    kp = RB.kp_svd(sep, n)
    x = rng.standard_normal((n, n))
    assert np.abs(KP.kp_apply(kp, x) - RB.blur(sep, x)).max() < 1e-12
    # every term of the plain PSF SVD reproduces A exactly
    psf = _sym_psf(rng, k)
    u, s, vt = np.linalg.svd(psf)
    full = sum(RB.reflexive_band(np.sqrt(s[i]) * u[:, i], n) @ x
               @ RB.reflexive_band(np.sqrt(s[i]) * vt[i, :], n).T for i in range(k))
    assert np.abs(full - RB.blur(psf, x)).max() < 1e-12


def test_exact_diag_brute_force():
    rng = np.random.default_rng(6)
    n, k = 8, 5
    psf = _sym_psf(rng, k)
    kp = RB.kp_svd(psf, n)
    d0 = RB.exact_diag(kp, psf)
    brute = np.array([[np.sum(RB.blur(psf, np.outer(kp.Vc[:, i], kp.Vr[:, j])) ** 2)
                       for j in range(n)] for i in range(n)])
    assert np.abs(d0 - brute).max() < 1e-13 * brute.max()


def test_oracle_pcg_converges_to_closed_form():
    rng = np.random.default_rng(7)
    n, k, lam = 64, 9, 0.03
    psf = _sym_psf(rng, k)
    b = rng.standard_normal((n, n))
    op = RB.NormalOperator(psf, n, lam)
    kp = RB.kp_svd(psf, n)
    out = SV.solve(op, b, mode=SV.PCG, tol=1e-12, maxit=500,
                   precond=lambda r: KP.precond_solve(kp, lam, r))
    xl = RB.x_lambda(psf, b, lam)
    assert out.status == "converged"
    assert np.linalg.norm(out.x - xl) / np.linalg.norm(xl) < 1e-9


def test_rejects_asymmetric_or_large_psf():
    with pytest.raises(ValueError):
        RB.blur(np.arange(9.0).reshape(3, 3), np.zeros((8, 8)))
    with pytest.raises(ValueError):
        RB.blur(np.ones((9, 9)), np.zeros((8, 8)))


def test_corner_response_closed_form():
    rng = np.random.default_rng(8)
    for n, k in ((8, 5), (16, 15), (9, 9)):
        psf = _sym_psf(rng, k)
        e = np.zeros((n, n))
        e[0, 0] = 1.0
        assert np.abs(RB.corner_response(psf, n) - RB.blur(psf, e)).max() < 1e-15


def test_reflexive_data_generator_matches_oracle_blur():
    """The synthetic reflexive workload's data model (numpy 'symmetric'
    padding, i.e. half-sample reflection, then the 'valid' linear
    convolution) is the oracle's reflexive A, and its PSF is symmetric."""
    import synthetic as S
    from synthetic.problems import _blur_for_data_reflexive
    rng = np.random.default_rng(12)
    for n, k in ((40, 9), (33, 15), (15, 15)):
        psf = _sym_psf(rng, k)
        x = rng.standard_normal((n, n))
        assert np.abs(_blur_for_data_reflexive(psf, x) - RB.blur(psf, x)).max() < 1e-10
    p = S.large_moffat_reflexive(0, n=96, k=15)
    assert RB.is_symmetric_psf(p.psf, rel=0.0)
    noise = p.b.astype(np.float64) - RB.blur(p.psf, p.x_true)
    assert abs(np.linalg.norm(noise) - p.noise_norm) < 1e-9 * p.noise_norm


# ---- PSFs that are not symmetric: A by the definition, A^T by scattering


def _asym_psf(rng, k):
    p = rng.uniform(0, 1, (k, k))
    return p / p.sum()


@pytest.mark.parametrize("n,k", [(8, 3), (9, 5), (16, 15), (12, 11), (7, 7)])
def test_general_blur_equals_scipy_reflect(n, k):
    rng = np.random.default_rng(n * 31 + k)
    psf = _asym_psf(rng, k)
    x = rng.standard_normal((n, n))
    ref = scipy.ndimage.convolve(x, psf, mode="reflect")
    assert np.abs(RB.blur_general(psf, x) - ref).max() < 1e-12


@pytest.mark.parametrize("n,k", [(6, 5), (7, 3), (9, 9), (10, 7)])
def test_general_adjoint_is_dense_transpose(n, k):
    """A^T by scattering equals the transpose of the dense A built column by
    column from the definition, and A is not symmetric for these PSFs."""
    rng = np.random.default_rng(n * 7 + k)
    psf = _asym_psf(rng, k)
    a = RB.dense_matrix(psf, n)
    assert np.abs(a - a.T).max() > 1e-3
    y = rng.standard_normal((n, n))
    want = (a.T @ y.reshape(-1, order="F")).reshape((n, n), order="F")
    assert np.abs(RB.blur_t_general(psf, y) - want).max() < 1e-13
    # and for the symmetric PSFs A^T = A
    sym = _sym_psf(rng, k)
    assert np.abs(RB.blur_t_general(sym, y) - RB.blur(sym, y)).max() < 1e-13


@pytest.mark.parametrize("n,k", [(16, 15), (40, 9), (33, 31), (64, 63)])
def test_general_fft_forms_equal_definitions(n, k):
    rng = np.random.default_rng(n + 3 * k)
    psf = _asym_psf(rng, k)
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((n, n))
    ax = RB.blur_general(psf, x)
    aty = RB.blur_t_general(psf, y)
    assert np.abs(RB.blur_fft_general(psf, x) - ax).max() < 1e-12 * np.abs(ax).max()
    assert np.abs(RB.blur_t_fft_general(psf, y) - aty).max() < 1e-12 * np.abs(aty).max()
    # adjointness at this size
    assert abs(np.sum(ax * y) - np.sum(x * aty)) < 1e-11 * np.abs(ax).sum()


def test_general_kp_expansion_and_separable_exactness():
    """Every term of the plain PSF SVD gives A exactly for an asymmetric
    PSF, and the one-term reflexive KP is exact for a separable one."""
    rng = np.random.default_rng(21)
    n, k = 12, 7
    psf = _asym_psf(rng, k)
    x = rng.standard_normal((n, n))
    u, s, vt = np.linalg.svd(psf)
    full = sum(RB.reflexive_band(np.sqrt(s[i]) * u[:, i], n) @ x
               @ RB.reflexive_band(np.sqrt(s[i]) * vt[i, :], n).T for i in range(k))
    assert np.abs(full - RB.blur_general(psf, x)).max() < 1e-12
    sep = np.outer(rng.uniform(0, 1, k), rng.uniform(0, 1, k))
    kp = RB.kp_svd(sep, n)
    assert np.abs(KP.kp_apply(kp, x) - RB.blur_general(sep, x)).max() < 1e-12


def test_general_x_lambda_equals_dense_solve():
    """The settled FP64 PCG minimiser equals a dense Cholesky solve, and
    the one-term KP preconditioner is exact (one iteration) for a separable
    asymmetric PSF."""
    rng = np.random.default_rng(22)
    n, k, lam = 12, 5, 0.05
    psf = _asym_psf(rng, k)
    b = rng.standard_normal((n, n))
    xd = RB.x_lambda_dense_general(psf, b, lam)
    x, info = RB.x_lambda_general(psf, b, lam)
    assert info["status"] == "converged" and info["true_relres"] < 1e-12
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-11
    sep = np.outer(rng.uniform(0, 1, k), rng.uniform(0, 1, k))
    sep /= sep.sum()
    _, info = RB.x_lambda_general(sep, b, lam, tol=1e-10, check=False)
    assert info["iters"] == 1


def test_general_reflexive_data_generator_matches_oracle_blur():
    import synthetic as S
    from synthetic.problems import _blur_for_data_reflexive
    rng = np.random.default_rng(23)
    for n, k in ((40, 9), (33, 15)):
        psf = _asym_psf(rng, k)
        x = rng.standard_normal((n, n))
        assert np.abs(_blur_for_data_reflexive(psf, x) - RB.blur_general(psf, x)).max() < 1e-10
    p = S.large_moffat_motion_reflexive(0, n=96, k=15)
    assert not RB.is_symmetric_psf(p.psf)
    noise = p.b.astype(np.float64) - RB.blur_general(p.psf, p.x_true)
    assert abs(np.linalg.norm(noise) - p.noise_norm) < 1e-9 * p.noise_norm
