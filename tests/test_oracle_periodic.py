"""Pins of the periodic-boundary oracle (oracle/periodic.py) against library
routines, closed forms and brute force."""
import numpy as np
import pytest
import scipy.signal

from oracle import kp as KP
from oracle import periodic as PB
from oracle import solvers as SV


def _psf(rng, k):
    p = rng.uniform(0, 1, (k, k))
    return p / p.sum()


@pytest.mark.parametrize("n,k", [(8, 3), (9, 5), (16, 15), (12, 11), (7, 7)])
def test_blur_equals_scipy_wrap(n, k):
    """A = convolve2d(mode='same', boundary='wrap'), A^T = correlate2d."""
    rng = np.random.default_rng(n * 31 + k)
    psf = rng.standard_normal((k, k))
    x = rng.standard_normal((n, n))
    ref = scipy.signal.convolve2d(x, psf, mode="same", boundary="wrap")
    assert np.abs(PB.blur(psf, x) - ref).max() < 1e-12
    reft = scipy.signal.correlate2d(x, psf, mode="same", boundary="wrap")
    assert np.abs(PB.blur_t(psf, x) - reft).max() < 1e-12


def test_adjoint_and_constant_eigenvector():
    rng = np.random.default_rng(3)
    n, k = 20, 9
    psf = rng.standard_normal((k, k))
    x, y = rng.standard_normal((2, n, n))
    lhs = np.sum(PB.blur(psf, x) * y)
    rhs = np.sum(x * PB.blur_t(psf, y))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    one = np.ones((n, n))
    assert np.abs(PB.blur(psf, one) - psf.sum()).max() < 1e-12
    assert np.abs(PB.blur_t(psf, one) - psf.sum()).max() < 1e-12


def test_delta_psf_is_identity_and_shift():
    n, k = 10, 5
    d = np.zeros((k, k))
    d[2, 2] = 1.0
    x = np.random.default_rng(1).standard_normal((n, n))
    assert np.array_equal(PB.blur(d, x), x)
    # a tap at offset (u, v) = (1, -2) moves the image cyclically by (1, -2)
    s = np.zeros((k, k))
    s[3, 0] = 1.0
    assert np.array_equal(PB.blur(s, x), np.roll(x, (1, -2), axis=(0, 1)))


def test_dft_form_equals_definition():
    rng = np.random.default_rng(5)
    n, k = 24, 13
    psf = rng.standard_normal((k, k))
    x = rng.standard_normal((n, n))
    assert np.abs(PB.blur_fft(psf, x) - PB.blur(psf, x)).max() < 1e-12
    assert np.abs(PB.blur_t_fft(psf, x) - PB.blur_t(psf, x)).max() < 1e-12


def test_dense_equals_cyclic_kronecker_sum():
    """A = sum_{u,v} P[h+u,h+v] C_v (x) C_u (column-major vec)."""
    rng = np.random.default_rng(6)
    n, k = 6, 5
    h = 2
    psf = rng.standard_normal((k, k))
    ref = sum(psf[h + u, h + v] * np.kron(PB.shift(v, n), PB.shift(u, n))
              for u in range(-h, h + 1) for v in range(-h, h + 1))
    assert np.abs(PB.dense_matrix(psf, n) - ref).max() < 1e-13


def test_kp_exact_for_separable_psf():
    rng = np.random.default_rng(7)
    n, k = 9, 7
    psf = np.outer(rng.uniform(0, 1, k), rng.uniform(0, 1, k))
    kp = PB.kp_svd(psf, n)
    x = rng.standard_normal((n, n))
    assert np.abs(KP.kp_apply(kp, x) - PB.blur(psf, x)).max() < 1e-12
    assert KP.kp_error(kp.s_psf) < 1e-7


@pytest.mark.parametrize("n,k,seed", [(5, 3, 0), (6, 5, 1), (7, 5, 2)])
def test_kp_equals_van_loan_pitsianis(n, k, seed):
    """The rank-1 SVD of P gives the brute-force nearest Kronecker product
    of the dense BCCB matrix, and ||A - A_hat|| / ||A|| = sqrt(sum_{k>1}
    s_k^2 / sum s_k^2)."""
    rng = np.random.default_rng(seed)
    psf = _psf(rng, k)
    a_dense = PB.dense_matrix(psf, n)
    b, c = KP.van_loan_pitsianis(a_dense, n)
    kp = PB.kp_svd(psf, n)
    khat = np.kron(kp.Ar, kp.Ac)
    assert np.abs(np.kron(b, c) - khat).max() < 1e-13
    err = np.linalg.norm(a_dense - khat) / np.linalg.norm(a_dense)
    assert abs(KP.kp_error(kp.s_psf) - err) < 1e-12


def test_circulant_singular_values_are_dft_moduli():
    rng = np.random.default_rng(8)
    n, k = 32, 9
    psf = _psf(rng, k)
    kp = PB.kp_svd(psf, n)
    c, a, _ = PB.kp_profiles(psf)
    for prof, sv in ((c, kp.sc), (a, kp.sr)):
        col = PB.circulant_band(prof, n)[:, 0]
        ref = np.sort(np.abs(np.fft.fft(col)))[::-1]
        assert np.abs(sv - ref).max() < 1e-13


def test_x_lambda_equals_dense_solve():
    rng = np.random.default_rng(9)
    n, k, lam = 8, 5, 0.07
    psf = _psf(rng, k)
    b = rng.standard_normal((n, n))
    a = PB.dense_matrix(psf, n)
    rhs = a.T @ b.reshape(-1, order="F")
    xd = np.linalg.solve(a.T @ a + lam * lam * np.eye(n * n), rhs).reshape((n, n), order="F")
    assert np.abs(PB.x_lambda(psf, b, lam) - xd).max() < 1e-11 * np.abs(xd).max()


def test_oracle_pcg_converges_to_closed_form():
    """The oracle's KP-preconditioned PCG on the periodic operator reaches
    the DFT closed form."""
    rng = np.random.default_rng(10)
    n, k, lam = 64, 9, 0.03
    psf = _psf(rng, k)
    b = rng.standard_normal((n, n))
    op = PB.NormalOperator(psf, n, lam)
    kp = PB.kp_svd(psf, n)
    out = SV.solve(op, b, mode=SV.PCG, tol=1e-12, maxit=500,
                   precond=lambda r: KP.precond_solve(kp, lam, r))
    xl = PB.x_lambda(psf, b, lam)
    assert out.status == "converged"
    assert np.linalg.norm(out.x - xl) / np.linalg.norm(xl) < 1e-9


def test_large_psf_rejected():
    with pytest.raises(ValueError):
        PB.blur(np.ones((9, 9)), np.zeros((8, 8)))


def test_periodic_data_generator_matches_oracle_blur():
    """The synthetic periodic workload's data model (wrap padding + the
    'valid' linear convolution) is the oracle's periodic A."""
    import synthetic as S
    from synthetic.problems import _blur_for_data_periodic
    rng = np.random.default_rng(11)
    for n, k in ((40, 9), (33, 15), (15, 15)):
        psf = rng.standard_normal((k, k))
        x = rng.standard_normal((n, n))
        assert np.abs(_blur_for_data_periodic(psf, x) - PB.blur(psf, x)).max() < 1e-10
    p = S.large_moffat_periodic(0, n=96, k=15)
    noise = p.b.astype(np.float64) - PB.blur(p.psf, p.x_true)
    assert abs(np.linalg.norm(noise) - p.noise_norm) < 1e-9 * p.noise_norm


def test_exact_diag_brute_force_and_closed_forms():
    """D0[i, j] = ||A (v_c,i v_r,j^T)||_F^2 by blurring every basis image;
    D0 = s_c^2 s_r^2 for a separable PSF; sum D0 = ||A||_F^2 = n^2 ||P||_F^2
    (each of the n^2 rows of the BCCB matrix holds every tap once)."""
    rng = np.random.default_rng(12)
    n, k = 8, 5
    psf = _psf(rng, k)
    kp = PB.kp_svd(psf, n)
    d0 = PB.exact_diag(kp, psf)
    brute = np.array([[np.sum(PB.blur(psf, np.outer(kp.Vc[:, i], kp.Vr[:, j])) ** 2)
                       for j in range(n)] for i in range(n)])
    assert np.abs(d0 - brute).max() < 1e-13 * brute.max()
    assert abs(d0.sum() - n * n * np.sum(psf ** 2)) < 1e-12 * d0.sum()
    sep = np.outer(rng.uniform(0, 1, k), rng.uniform(0, 1, k))
    kps = PB.kp_svd(sep, n)
    assert np.allclose(PB.exact_diag(kps, sep), np.outer(kps.sc ** 2, kps.sr ** 2), rtol=1e-12,
                       atol=1e-14)
