"""Pins for the Kronecker approximation and the KP-SVD preconditioner."""
import math

import numpy as np
import pytest

import synthetic as S
from oracle import kp as KP
from oracle import operator as O


def _dense_khat(c, a, n):
    # A_hat = A_r (x) A_c in column-major vec ordering
    return np.kron(KP.toeplitz_band(a, n), KP.toeplitz_band(c, n))


@pytest.mark.parametrize("n,k,seed", [(9, 5, 0), (8, 3, 1), (7, 7, 2), (6, 5, 3)])
def test_weighted_construction_equals_van_loan_pitsianis(n, k, seed):
    """The weighted rank-1 PSF construction gives the same A_hat as the
    brute-force nearest Kronecker product of the dense A (Section 5,
    eq. (KronSumDecomp), argmin ||A - A_r (x) A_c||_F)."""
    rng = np.random.default_rng(seed)
    psf = rng.uniform(0, 1, (k, k))
    psf /= psf.sum()
    a_dense = O.dense_matrix(psf, n)
    b, c = KP.van_loan_pitsianis(a_dense, n)
    cc, aa, s = KP.kp_profiles(psf, n)
    khat = _dense_khat(cc, aa, n)
    assert np.abs(np.kron(b, c) - khat).max() < 1e-13
    err_dense = np.linalg.norm(a_dense - khat) / np.linalg.norm(a_dense)
    assert abs(KP.kp_error(s) - err_dense) < 1e-12


def test_factor_toeplitz_orientation():
    """A_hat X = A_c X A_r^T equals the dense A_hat acting on vec(X)."""
    rng = np.random.default_rng(4)
    n, k = 7, 5
    psf = rng.uniform(0, 1, (k, k))
    kp = KP.kp_svd(psf, n)
    cc, aa, _ = KP.kp_profiles(psf, n)
    x = rng.standard_normal((n, n))
    lhs = O.vec(KP.kp_apply(kp, x))
    rhs = _dense_khat(cc, aa, n) @ O.vec(x)
    assert np.allclose(lhs, rhs, atol=1e-13)


def test_separable_psf_is_exact():
    """A rank-one PSF is exactly one Kronecker term (Section 5, Gaussian)."""
    n = 10
    g = np.exp(-np.arange(-3, 4) ** 2 / 4.0)
    f = np.exp(-np.arange(-3, 4) ** 2 / 9.0)
    psf = np.outer(g, f)
    psf /= psf.sum()
    kp = KP.kp_svd(psf, n)
    assert KP.kp_terms(kp.s_psf) == 1
    assert KP.kp_error(kp.s_psf) < 1e-14
    x = np.random.default_rng(0).standard_normal((n, n))
    assert np.allclose(KP.kp_apply(kp, x), O.blur(psf, x), atol=1e-14)


def test_table1_gauss_row_order_of_magnitude():
    """Table 1 prints ||A - A_hat||_F/||A||_F = 7.9195e-8 for the Gaussian
    blur, where A is one Kronecker term up to rounding.  A float32-stored
    Gaussian PSF reproduces that order (<= 1e-7); the other rows need
    several terms."""
    fixture = {}
    with open(_golden("table1_kp_error.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, terms, err = line.split()
                fixture[name] = (int(terms), float(err))
    gauss_terms, gauss_err = fixture["Gauss"]
    assert gauss_terms == 1
    p = S.psf_gaussian(15, 2.0, 2.0, 0.0)
    kp = KP.kp_svd(p, 128)
    err = KP.kp_error(kp.s_psf)
    assert err < 1e-7 and err > 0
    assert math.floor(math.log10(gauss_err)) >= math.floor(math.log10(err)) - 1
    # the non-separable workloads are not single Kronecker terms
    q = S.psf_gaussian(31, 4.0, 2.0, math.radians(30))
    assert KP.kp_error(KP.kp_svd(q, 64).s_psf) > 0.05
    for name in ("Defocus", "Speckle", "Shake", "Motion"):
        assert fixture[name][0] > 1 and fixture[name][1] > 0.1


def _golden(name):
    import os
    return os.path.join(os.path.dirname(__file__), "golden", name)


@pytest.mark.parametrize("n,k,lam", [(6, 3, 0.05), (8, 5, 0.01), (7, 7, 0.3)])
def test_preconditioner_equals_dense_inverse(n, k, lam):
    """z = M^{-1} r with M = A_hat^T A_hat + lambda^2 I (eq. (PreconSystem))
    through eq. (PreconSolve) equals the dense inverse."""
    rng = np.random.default_rng(n + k)
    psf = rng.uniform(0, 1, (k, k))
    psf /= psf.sum()
    kp = KP.kp_svd(psf, n)
    cc, aa, _ = KP.kp_profiles(psf, n)
    khat = _dense_khat(cc, aa, n)
    m = khat.T @ khat + lam * lam * np.eye(n * n)
    r = rng.standard_normal((n, n))
    z_ref = np.linalg.solve(m, O.vec(r))
    z = O.vec(KP.precond_solve(kp, lam, r))
    assert np.linalg.norm(z - z_ref) <= 1e-10 * np.linalg.norm(z_ref)


def test_preconditioner_sign_and_order_invariance():
    rng = np.random.default_rng(9)
    n, k, lam = 12, 5, 0.02
    psf = S.psf_moffat_motion(k, 3.0, 2.5, 4.0, 0.3)
    kp = KP.kp_svd(psf, n)
    r = rng.standard_normal((n, n))
    z = KP.precond_solve(kp, lam, r)
    sg = rng.choice([-1.0, 1.0], n)
    perm = rng.permutation(n)
    kp.Vc = (kp.Vc * sg)[:, perm]
    kp.sc = kp.sc[perm]
    kp.Vr = kp.Vr[:, ::-1] * -1
    kp.sr = kp.sr[::-1]
    z2 = KP.precond_solve(kp, lam, r)
    assert np.allclose(z, z2, atol=1e-11 * np.abs(z).max())


def test_preconditioner_inverts_h_when_separable():
    """M^{-1} H_lambda = I when A is exactly one Kronecker term."""
    n, lam = 8, 0.03
    g = np.exp(-np.arange(-2, 3) ** 2 / 3.0)
    psf = np.outer(g, g[::-1] * np.linspace(1, 2, 5))
    psf /= psf.sum()
    kp = KP.kp_svd(psf, n)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((n, n))
    hx = O.normal_op(psf, lam, x)
    assert np.allclose(KP.precond_solve(kp, lam, hx), x, atol=1e-10)


# ---------------------------------------------------------------------------
# exact diagonal in the KP basis: D0 = diag(V^T A^T A V) from all terms of
# eq. (KronSumDecomp)
# ---------------------------------------------------------------------------

def _random_psf(rng, k):
    p = rng.random((k, k)) ** 3
    return p / p.sum()


@pytest.mark.parametrize("n,k,seed", [(11, 7, 0), (16, 9, 1), (9, 9, 2)])
def test_kron_sum_reproduces_blur(n, k, seed):
    """All terms of the weighted PSF SVD give A exactly (eq. (KronSumDecomp)):
    sum_k T(c_k) X T(a_k)^T equals the direct zero-boundary convolution, and
    the number of terms is the rank of the PSF."""
    rng = np.random.default_rng(seed)
    psf = _random_psf(rng, k)
    cs, as_ = KP.kp_all_terms(psf, n)
    assert len(cs) == np.linalg.matrix_rank(psf)
    x = rng.standard_normal((n, n))
    assert np.abs(KP.kron_sum_apply(cs, as_, x) - O.blur(psf, x)).max() <= 1e-13


@pytest.mark.parametrize("n,k,seed", [(8, 5, 0), (7, 7, 1), (10, 3, 2)])
def test_exact_diag_equals_definition(n, k, seed):
    """D0[i, j] = ||A (v_c,i v_r,j^T)||_F^2 computed by blurring every basis
    image of the KP basis with the direct operator, against the Kronecker-sum
    Gram formula."""
    rng = np.random.default_rng(seed)
    psf = _random_psf(rng, k)
    kp = KP.kp_svd(psf, n)
    ref = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            ref[i, j] = np.sum(O.blur(psf, np.outer(kp.Vc[:, i], kp.Vr[:, j])) ** 2)
    got = KP.exact_diag(kp, psf)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_exact_diag_is_one_term_spectrum_when_separable():
    """A separable PSF has one Kronecker term, so D0 = s_c^2 s_r^2 and the
    preconditioner is unchanged."""
    g1 = np.exp(-0.5 * ((np.arange(9) - 4) / 1.7) ** 2)
    g2 = np.exp(-0.5 * ((np.arange(9) - 4) / 2.3) ** 2)
    psf = np.outer(g1, g2) / (g1.sum() * g2.sum())
    kp = KP.kp_svd(psf, 20)
    d0 = KP.exact_diag(kp, psf)
    assert len(KP.kp_all_terms(psf, 20)[0]) == 1
    ref = np.outer(kp.sc ** 2, kp.sr ** 2)
    assert np.abs(d0 - ref).max() <= 1e-12 * ref.max()


@pytest.mark.parametrize("n,k", [(40, 15), (64, 31)])
def test_exact_diag_trace_is_frobenius_norm(n, k):
    """The KP basis is orthonormal, so sum_ij D0[i, j] = ||A||_F^2, which the
    disjoint supports of the shift products give in closed form:
    sum_{u,v} P[u, v]^2 (n - |u - h|)(n - |v - h|); and D0 >= 0."""
    psf = S.psf_moffat_motion(k, 3.0, 2.5, 5.0, 0.9)
    kp = KP.kp_svd(psf, n)
    d0 = KP.exact_diag(kp, psf)
    w = KP.weights(k, n)
    fro2 = float(np.sum(psf ** 2 * np.outer(w, w)))
    assert abs(d0.sum() - fro2) <= 1e-12 * fro2
    assert d0.min() >= -1e-15 * d0.max()


def test_exact_diag_preconditioner_same_solution_fewer_iterations():
    """With S = 1 / (D0 + lambda^2) PCG still converges to x_lambda (the
    preconditioner changes only the iteration), and on a non-separable
    Moffat + motion blur it needs fewer iterations than the one-term S."""
    from oracle import solvers as SV
    rng = np.random.default_rng(7)
    n, k, lam = 48, 15, 0.02
    psf = S.psf_moffat_motion(k, 3.5, 2.5, 6.0, 0.6)
    x = S.true_image(rng, n)
    prob = S.make_problem(n, psf, rng, 0.01, lam, 7, "moffat15", x_true=x)
    b = prob.b.astype(np.float64)
    ref = SV.x_lambda(psf, b, lam)
    op = SV.NormalOperator(psf, n, lam)
    kp = KP.kp_svd(psf, n)
    one = SV.solve(op, b, SV.PCG, tol=1e-12, maxit=300,
                   precond=SV.kp_preconditioner(psf, n, lam, kp))
    ex = SV.solve(op, b, SV.PCG, tol=1e-12, maxit=300,
                  precond=SV.kp_preconditioner(psf, n, lam, kp, exact_diag=True))
    assert ex.status == "converged" and one.status == "converged"
    assert np.linalg.norm(ex.x - ref) <= 1e-8 * np.linalg.norm(ref)
    assert ex.iters < one.iters


def test_fp16_factor_construction():
    """The FP16-rounded factors: the power-of-two scale puts the largest
    entry in [2^13, 2^14) and unscales exactly; entries that are FP16 values
    at that scale survive unchanged; every singular value moves by at most
    ||A16 - A||_2 (Weyl), and the rounding is at most 2^-11 relative to the
    largest entry per entry."""
    rng = np.random.default_rng(31)
    n, k = 48, 15
    psf = S.psf_moffat_motion(k, 5.0, 2.5, 6.0, 0.7)
    kp = KP.kp_svd(psf, n)
    lo = KP.kp_svd_fp16_factors(kp)
    for a, a16, s, s16 in ((kp.Ac, lo.Ac, kp.sc, lo.sc), (kp.Ar, lo.Ar, kp.sr, lo.sr)):
        mx = np.abs(a).max()
        e = 13 - int(np.floor(np.log2(mx)))
        assert 2.0 ** 13 <= mx * 2.0 ** e < 2.0 ** 14
        assert np.all(np.abs(a16 - a) <= 2.0 ** -11 * 2.0 ** 14 * 2.0 ** -e)
        assert np.all(np.abs(s16 - s) <= np.linalg.norm(a16 - a, 2) * (1 + 1e-12) + 1e-15)
    q = rng.integers(-2048, 2048, (n, n)) / 2048.0          # FP16 values already
    assert np.array_equal(KP.fp16_factor(q), q)
