"""Pins for the regularisation-parameter rules (Section 2.2)."""
import numpy as np
import pytest

import synthetic as S
from oracle import kp as KP
from oracle import lam as L
from oracle import operator as O
from oracle import solvers as SV


def _separable(n, k, seed):
    rng = np.random.default_rng(seed)
    g = np.exp(-np.arange(-(k // 2), k // 2 + 1) ** 2 / 2.5)
    f = np.exp(-np.arange(-(k // 2), k // 2 + 1) ** 2 / 4.0)
    psf = np.outer(g, f)
    psf /= psf.sum()
    x = S.true_image(rng, n)
    bt = O.blur(psf, x)
    noise = 0.02 * np.linalg.norm(bt) * rng.standard_normal((n, n)) / n
    return psf, x, bt + noise, float(np.linalg.norm(noise))


LAMS = np.logspace(-3, 0, 7)


@pytest.mark.parametrize("omega", [1.0, 3.0, 0.5])
def test_gcv_svd_form_equals_trace_form(omega):
    """eq. (GCVTik)/(wGCVTik) (dense influence matrix) = eq. (GCVTikSVD)/
    (wGCVTikSVD) (dense SVD) = the same in the exact Kronecker basis."""
    n, k = 7, 5
    psf, _, b, _ = _separable(n, k, 0)
    s2, bh2 = L.dense_spectrum(psf, b)
    kp = KP.kp_svd(psf, n)
    ks2, kbh2 = L.spectrum(kp, b)
    inadmissible = 0
    for lam in LAMS:
        tr = L.gcv_trace_form(psf, b, lam, omega)
        sv = L.gcv(s2, bh2, [lam], omega)[0]
        kb = L.gcv(ks2, kbh2, [lam], omega)[0]
        if np.isinf(tr):
            # the dense trace of I - omega A A^+ is not positive: the spectral
            # forms must exclude the same lambda
            inadmissible += 1
            assert np.isinf(sv) and np.isinf(kb)
            continue
        assert abs(sv - tr) <= 1e-8 * tr
        assert abs(kb - tr) <= 1e-8 * tr
    assert inadmissible == 0 or omega > 1.0
    if omega > 1.0:
        assert 0 < inadmissible < len(LAMS)     # both branches are exercised


def test_gcv_printed_form_equals_weighted_form_at_omega_one():
    psf, _, b, _ = _separable(8, 3, 1)
    kp = KP.kp_svd(psf, 8)
    s2, bh2 = L.spectrum(kp, b)
    a = L.gcv(s2, bh2, LAMS, 1.0)
    bb = L.gcv_unweighted_form(s2, bh2, LAMS)
    assert np.allclose(a, bb, rtol=1e-10)


def test_discrepancy_equals_residual_of_solution():
    """eq. (DSCTik): D = ||A x_lambda - b||^2 - eps^2, evaluated with the
    dense solution, equals eq. (DSCTikSVD) in the Kronecker basis."""
    n, k = 8, 5
    psf, _, b, nn = _separable(n, k, 2)
    kp = KP.kp_svd(psf, n)
    s2, bh2 = L.spectrum(kp, b)
    for lam in LAMS:
        x = SV.x_lambda_dense(psf, b, lam)
        d_ref = np.sum((O.blur(psf, x) - b) ** 2) - nn * nn
        d = L.discrepancy(s2, bh2, [lam], nn)[0]
        assert abs(d - d_ref) <= 1e-9 * (abs(d_ref) + nn * nn)


def test_discrepancy_monotone_and_root():
    n, k = 16, 5
    psf, _, b, nn = _separable(n, k, 3)
    kp = KP.kp_svd(psf, n)
    s2, bh2 = L.spectrum(kp, b)
    grid = np.logspace(-5, 1, 61)
    d = L.discrepancy(s2, bh2, grid, nn)
    assert np.all(np.diff(d) >= -1e-15 * np.abs(d).max())
    root = L.discrepancy_root(s2, bh2, nn)
    assert abs(L.discrepancy(s2, bh2, [root], nn)[0]) <= 1e-8 * nn * nn
    i = L.grid_discrepancy(d)
    assert grid[i] <= root <= grid[min(i + 1, grid.size - 1)]


def test_optimal_error_equals_solution_error():
    """eq. (OptTikSVD): O(lambda) = ||x_lambda - x_true||^2 in the exact
    Kronecker basis (V orthogonal)."""
    n, k = 8, 5
    psf, x_true, b, _ = _separable(n, k, 4)
    kp = KP.kp_svd(psf, n)
    o = L.optimal_error(kp, b, x_true, LAMS)
    for lam, ov in zip(LAMS, o):
        x = SV.x_lambda_dense(psf, b, lam)
        ref = np.sum((x - x_true) ** 2)
        assert abs(ov - ref) <= 1e-9 * ref


def test_grid_rules_tie_breaking():
    assert L.grid_argmin([3.0, 1.0, 1.0, 2.0]) == 1
    assert L.grid_discrepancy([-2.0, -1.0, 0.0, 1.0]) == 2
    assert L.grid_discrepancy([1.0, 2.0]) == 0


def test_discrepancy_choice_grows_with_eta():
    """D(lambda) = sum (lambda^2 b_hat / (s^2 + lambda^2))^2 - (eta ||eps||)^2
    increases with lambda, so a larger eta can only move the discrepancy
    choice to a larger (or the same) lambda (eq. (DSCTikSVD) with the modified
    epsilon of Section 5.1); the bisection root grows strictly."""
    psf, x, b, nn = _separable(24, 7, 3)
    kp = KP.kp_svd(psf, 24)
    s2, bh2 = L.spectrum(kp, b)
    grid = np.logspace(-4, 0, 48)
    idx = [L.grid_discrepancy(L.discrepancy(s2, bh2, grid, eta * nn)) for eta in
           (1.0, 2.0, 3.0, 5.0, 10.0, 15.0)]
    assert idx == sorted(idx) and idx[-1] > idx[0]
    roots = [L.discrepancy_root(s2, bh2, eta * nn) for eta in (1.0, 2.0, 3.0)]
    assert roots[0] < roots[1] < roots[2]
