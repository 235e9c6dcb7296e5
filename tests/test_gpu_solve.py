"""End-to-end parity of pcg_solve / gcv_lambda against the FP64 oracle.

Parity measure: ||x - x_lambda|| / ||x_lambda|| with x_lambda the exact
Tikhonov minimiser computed by the oracle (eq. (tik:normal2)).  Bars: 1e-5
for the FP32 preconditioner, 1e-4 for FP16 (and for CG), the solver
tolerance chosen tight enough that the iteration error is below the bar.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import kp as KP
from oracle import lam as L
from oracle import solvers as SV
from tests.gpu_util import rel, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _modes():
    from paper_2311_15393_amd import KP_CG, KP_FPCG, KP_P8, KP_P16, KP_P32, KP_PCG
    return {"cg": KP_CG, "pcg32": KP_PCG | KP_P32, "fpcg32": KP_FPCG | KP_P32,
            "pcg16": KP_PCG | KP_P16, "fpcg16": KP_FPCG | KP_P16, "fpcg8": KP_FPCG | KP_P8}


_XLAM = {}


def _xlam(prob):
    key = (prob.kind, prob.n, prob.seed, prob.lam)
    if key not in _XLAM:
        _XLAM[key] = SV.x_lambda(prob.psf, prob.b.astype(np.float64), prob.lam)
    return _XLAM[key]


@pytest.mark.parametrize("mode,tol,bar,maxit", [
    ("cg", 1e-8, 1e-4, 400), ("pcg32", 1e-9, 1e-5, 50), ("fpcg32", 1e-9, 1e-5, 50),
    ("pcg16", 1e-8, 1e-4, 50), ("fpcg16", 1e-8, 1e-4, 50)])
def test_small_gaussian(mode, tol, bar, maxit):
    """64 x 64, separable Gaussian (K = 15): one Kronecker term, so the FP32
    KP-preconditioned iteration needs only a couple of iterations."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_OK, Plan
    prob = S.small_gaussian(0)
    say(f"small gaussian {mode}")
    ref = _xlam(prob)
    with Plan(prob.psf, prob.n) as plan:
        x, info = plan.solve(to_dev(prob.b), prob.lam, tol=tol, maxit=maxit,
                             mode=_modes()[mode])
        got = to_host(x)
    err = rel(got, ref)
    say(f"  iters={info.iters} status={info.status} relres_true={info.relres_true:.2e} err={err:.2e}")
    assert info.status == KP_OK
    assert info.relres_true <= tol
    assert err <= bar
    if mode in ("pcg32", "fpcg32"):
        assert info.iters <= 3


@pytest.mark.parametrize("mode,tol,bar", [
    ("cg", 1e-8, 1e-4), ("pcg32", 1e-8, 1e-5), ("fpcg32", 1e-8, 1e-5),
    ("pcg16", 1e-7, 1e-4), ("fpcg16", 1e-7, 1e-4), ("fpcg8", 1e-7, 1e-4)])
def test_mid_anisotropic(mode, tol, bar):
    """256 x 256, rotated anisotropic Gaussian (K = 31), lambda = 0.01."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_OK, Plan
    prob = S.mid_anisotropic(0)
    say(f"mid anisotropic {mode}")
    ref = _xlam(prob)
    with Plan(prob.psf, prob.n) as plan:
        x, info = plan.solve(to_dev(prob.b), prob.lam, tol=tol, maxit=3000,
                             mode=_modes()[mode])
        got = to_host(x)
    err = rel(got, ref)
    say(f"  iters={info.iters} repl={info.replacements} relres_true={info.relres_true:.2e} err={err:.2e}")
    assert info.status == KP_OK and info.relres_true <= tol
    assert err <= bar


@pytest.mark.parametrize("n,k", [(37, 9), (100, 15), (130, 31)])
def test_ragged_sizes(n, k):
    """Image sizes that leave partial tiles in every kernel."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_FPCG, KP_OK, KP_P16, KP_P32, KP_PCG, Plan
    rng = np.random.default_rng(n)
    psf = S.psf_moffat_motion(k, 3.0, 2.5, 4.0, 1.0)
    prob = S.make_problem(n, psf, rng, 0.01, 0.02, n, f"ragged{k}")
    say(f"ragged n={n} k={k}")
    ref = _xlam(prob)
    with Plan(psf, n) as plan:
        for mode, bar in ((KP_PCG | KP_P32, 1e-5), (KP_FPCG | KP_P16, 1e-4)):
            x, info = plan.solve(to_dev(prob.b), prob.lam, tol=1e-8, maxit=500, mode=mode)
            err = rel(to_host(x), ref)
            say(f"  mode={mode:#x} iters={info.iters} err={err:.2e}")
            assert info.status == KP_OK and err <= bar


@pytest.mark.parametrize("n,k", [(1, 1), (2, 3), (3, 5), (5, 9), (16, 31)])
def test_smallest_sizes(n, k):
    """Degenerate sizes: one pixel (A = P[0,0] I, so x = P b / (P^2 + lambda^2)
    in closed form), and PSF supports larger than the image (K up to 2n - 1),
    against the oracle's dense Cholesky solve; FP32 PCG and FP16 FPCG."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_FPCG, KP_OK, KP_P16, KP_P32, KP_PCG, Plan
    rng = np.random.default_rng(70 + n)
    psf = rng.uniform(0.2, 1.0, (k, k))
    psf = (psf / psf.sum()).astype(np.float32).astype(np.float64)
    b = rng.uniform(0.0, 1.0, (n, n)).astype(np.float32)
    lam = 0.05
    ref = SV.x_lambda_dense(psf, b.astype(np.float64), lam)
    if n == 1:
        p0 = psf[0, 0]
        assert abs(ref[0, 0] - p0 * b[0, 0] / (p0 * p0 + lam * lam)) <= 1e-12
    say(f"smallest n={n} k={k}")
    with Plan(psf, n) as plan:
        for mode, bar in ((KP_PCG | KP_P32, 1e-5), (KP_FPCG | KP_P16, 1e-4)):
            x, info = plan.solve(to_dev(b), lam, tol=1e-9, maxit=100, mode=mode)
            err = rel(to_host(x), ref)
            say(f"  mode={mode:#x} iters={info.iters} err={err:.2e}")
            assert info.status == KP_OK and err <= bar


def test_maximum_size():
    """The largest image the library accepts (2048 x 2048) with the largest
    PSF support (K = 63): the FP16-KP FPCG solve reaches the oracle's
    x_lambda."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_FPCG, KP_OK, KP_P16, Plan
    prob = S.large_moffat(3, n=2048, k=63)
    lam = 0.03
    say("maximum size 2048^2, K = 63")
    ref = SV.x_lambda(prob.psf, prob.b.astype(np.float64), lam)
    with Plan(prob.psf, prob.n) as plan:
        x, info = plan.solve(to_dev(prob.b), lam, tol=1e-6, maxit=100, mode=KP_FPCG | KP_P16)
        got = to_host(x)
    err = rel(got, ref)
    say(f"  iters={info.iters} relres_true={info.relres_true:.2e} err={err:.2e}")
    assert info.status == KP_OK and err <= 1e-4


def test_edge_cases():
    torch = require_gpu()
    from paper_2311_15393_amd import (KP_BREAKDOWN, KP_ERR_ARG, KP_FPCG, KP_MAXIT, KP_OK, KP_P16,
                                      KP_PCG, KP_WARM, KPError, Plan)
    prob = S.small_gaussian(1)
    with Plan(prob.psf, prob.n) as plan:
        say("edge: zero data")
        z = torch.zeros((prob.n, prob.n), device="cuda")
        x, info = plan.solve(z, 0.02, mode=KP_FPCG | KP_P16)
        assert info.status == KP_OK and info.iters == 0 and not to_host(x).any()
        say("edge: maxit = 1")
        x, info = plan.solve(to_dev(prob.b), 0.02, tol=1e-12, maxit=1, mode=0)
        assert info.status == KP_MAXIT and info.iters == 1
        say("edge: warm start from the converged solution")
        x, info = plan.solve(to_dev(prob.b), 0.02, tol=1e-7, maxit=50, mode=KP_PCG)
        x2, info2 = plan.solve(to_dev(prob.b), 0.02, tol=1e-6, maxit=50,
                               mode=KP_PCG | KP_WARM, x=x.clone())
        assert info2.status == KP_OK and info2.iters == 0
        say("edge: invalid arguments")
        for kw in ({"lam": -1.0}, {"lam": 0.0}, {"lam": float("nan")}, {"tol": 0.0},
                   {"maxit": 0}, {"mode": 3}, {"mode": 0x30}, {"mode": 0x2000}):
            args = {"lam": 0.02, "tol": 1e-6, "maxit": 10, "mode": KP_PCG}
            args.update(kw)
            with pytest.raises(KPError) as ei:
                plan.solve(to_dev(prob.b), args["lam"], tol=args["tol"],
                           maxit=args["maxit"], mode=args["mode"])
            assert ei.value.status == KP_ERR_ARG
        say("edge: non-finite data")
        bad = to_dev(prob.b)
        bad[3, 5] = float("nan")
        with pytest.raises(KPError) as ei:
            plan.solve(bad, 0.02, mode=KP_PCG)
        assert ei.value.status == KP_BREAKDOWN


@pytest.mark.parametrize("tol,cfg", [(1e-6, 6), (1e-6, 7), (1e-6, 0), (5e-8, 6)])
def test_reported_true_residual_matches_oracle(tol, cfg):
    """The certificate: relres_true, formed on the device as
    A^T (b - A x) - lambda^2 x with b - A x in FP64 and A^T on the MFMA blur
    (cfg 6) or the FP32 VALU blur (cfg 0) for tol >= 1e-7, in FP64 below,
    equals the oracle's FP64 ||c - H x|| / ||c|| at the returned x (eq.
    (tik:normal2)), to within a tenth of the tolerance."""
    require_gpu()
    from paper_2311_15393_amd import KP_FPCG, KP_OK, KP_P16, Plan
    from oracle import operator as O
    prob = S.mid_anisotropic(0)
    say(f"true residual certificate tol={tol:.0e} cfg={cfg}")
    b64 = prob.b.astype(np.float64)
    fb = O.FFTBlur(prob.psf, prob.n)
    c = fb.blur_t(b64)
    with Plan(prob.psf, prob.n) as plan:
        plan.set_blur_config(cfg)
        x, info = plan.solve(to_dev(prob.b), prob.lam, tol=tol, maxit=200,
                             mode=KP_FPCG | KP_P16)
        got = to_host(x).astype(np.float64)
    r = c - O.normal_op(prob.psf, prob.lam, got, fft=fb)
    ref = float(np.linalg.norm(r) / np.linalg.norm(c))
    say(f"  iters={info.iters} repl={info.replacements} relres_true={info.relres_true:.4e} "
        f"oracle={ref:.4e}")
    assert info.status == KP_OK and info.relres_true <= tol
    assert abs(info.relres_true - ref) <= 0.1 * tol
    assert abs(info.rhs_norm - np.linalg.norm(c)) <= 1e-5 * np.linalg.norm(c)


def test_nonfinite_data_on_mfma_blur():
    """Inf or NaN anywhere in b ends the solve with KP_BREAKDOWN also when the
    right-hand side runs on the MFMA blur (per-tile scaling must not hide it)."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_BREAKDOWN, KP_FPCG, KP_P16, KPError, Plan
    prob = S.mid_anisotropic(1)
    with Plan(prob.psf, prob.n) as plan:
        plan.set_blur_config(6)
        for bad_value in (float("inf"), float("-inf"), float("nan")):
            say(f"non-finite data {bad_value} on the MFMA blur")
            bad = to_dev(prob.b)
            bad[100, 37] = bad_value
            with pytest.raises(KPError) as ei:
                plan.solve(bad, prob.lam, tol=1e-6, maxit=50, mode=KP_FPCG | KP_P16)
            assert ei.value.status == KP_BREAKDOWN


@pytest.mark.parametrize("mode,tol,bar", [("fpcg16", 1e-7, 1e-4), ("pcg32", 1e-8, 1e-5)])
def test_exact_diag_solve_matches_oracle(mode, tol, bar):
    """KP_EXACT_DIAG changes only the preconditioner: the solve still reaches
    the oracle's x_lambda, and on the rotated anisotropic Gaussian (a
    non-separable PSF, one-term KP error 0.29) in fewer iterations than the
    one-term diagonal."""
    require_gpu()
    from paper_2311_15393_amd import KP_EXACT_DIAG, KP_OK, Plan
    prob = S.mid_anisotropic(0)
    ref = _xlam(prob)
    say(f"exact diagonal solve {mode}")
    with Plan(prob.psf, prob.n) as plan:
        x, info = plan.solve(to_dev(prob.b), prob.lam, tol=tol, maxit=400,
                             mode=_modes()[mode] | KP_EXACT_DIAG)
        got = to_host(x)
        _, info1 = plan.solve(to_dev(prob.b), prob.lam, tol=tol, maxit=400, mode=_modes()[mode])
    err = rel(got, ref)
    say(f"  iters={info.iters} (one-term {info1.iters}) relres_true={info.relres_true:.2e} "
        f"err={err:.2e}")
    assert info.status == KP_OK and info.relres_true <= tol and err <= bar
    assert info.iters < 0.75 * info1.iters


def test_gcv_and_discrepancy_match_oracle():
    """KP-basis GCV and discrepancy on the 32-point grid (eqs. (GCVTikSVD),
    (DSCTikSVD)): same grid choice as the oracle, scores to 1e-5 relative
    (b_hat from FP32 factors and FP32 MFMA GEMMs)."""
    torch = require_gpu()
    from paper_2311_15393_amd import Plan
    prob = S.mid_anisotropic(2)
    grid = S.lambda_grid()
    kp = KP.kp_svd(prob.psf, prob.n)
    s2, bh2 = L.spectrum(kp, prob.b.astype(np.float64))
    g_ref = L.gcv(s2, bh2, grid)
    d_ref = L.discrepancy(s2, bh2, grid, prob.noise_norm)
    with Plan(prob.psf, prob.n) as plan:
        lam_g, g = plan.gcv(to_dev(prob.b), grid)
        lam_w, gw = plan.gcv(to_dev(prob.b), grid, omega=3.0)
        lam_d, d = plan.discrepancy(to_dev(prob.b), grid, prob.noise_norm)
    say(f"gcv lam={lam_g:.4g} dp lam={lam_d:.4g}")
    assert lam_g == grid[L.grid_argmin(g_ref)]
    assert np.allclose(g, g_ref, rtol=1e-5)
    assert np.allclose(gw, L.gcv(s2, bh2, grid, 3.0), rtol=1e-5)
    assert lam_w == grid[L.grid_argmin(L.gcv(s2, bh2, grid, 3.0))]
    assert np.allclose(d, d_ref, rtol=1e-5, atol=1e-6 * prob.noise_norm ** 2)
    assert lam_d == grid[L.grid_discrepancy(d_ref)]


@pytest.mark.parametrize("kind", ["defocus", "motion"])
def test_weighted_gcv_and_modified_discrepancy_match_oracle(kind):
    """wGCV at omega = 2, 5, 8 (eq. (wGCVTikSVD)) and the discrepancy
    principle with epsilon = eta ||eps||, eta = 2, 5, 15 (Section 5.1) on
    non-separable blurs: the GPU's grid choice equals the oracle's, and the
    discrepancy choice never decreases with eta."""
    require_gpu()
    from paper_2311_15393_amd import Plan
    prob = S.study_problem(kind, 128, 0.01, 0)
    grid = S.lambda_grid(48)
    kp = KP.kp_svd(prob.psf, prob.n)
    s2, bh2 = L.spectrum(kp, prob.b.astype(np.float64))
    say(f"wgcv / modified dp on {prob.kind}")
    with Plan(prob.psf, prob.n) as plan:
        b = to_dev(prob.b)
        for omega in (2.0, 5.0, 8.0):
            lam, sc = plan.gcv(b, grid, omega=omega)
            ref = L.gcv(s2, bh2, grid, omega)
            assert np.allclose(sc, ref, rtol=1e-5)
            assert lam == grid[L.grid_argmin(ref)]
        prev = 0.0
        for eta in (2.0, 5.0, 15.0):
            lam, d = plan.discrepancy(b, grid, prob.noise_norm, eta=eta)
            ref = L.discrepancy(s2, bh2, grid, eta * prob.noise_norm)
            assert np.allclose(d, ref, rtol=1e-5, atol=1e-6 * (eta * prob.noise_norm) ** 2)
            assert lam == grid[L.grid_discrepancy(ref)]
            assert lam >= prev
            prev = lam


def test_lambda_study_runs():
    """The parameter study end to end on four small problems: every rule has
    a lambda on the grid and a finite error no smaller than the grid's best,
    and the optimal-error choice in the KP basis stays within 1.5x of it."""
    require_gpu()
    from paper_2311_15393_amd import lambda_study as LS
    probs = [S.study_problem(kind, 64, 0.01, 0) for kind in LS.KINDS]
    grid = S.lambda_grid(32)
    rows = LS.study(probs, grid, tol=1e-6)
    summary = LS.summarize(rows)
    say(LS.table(summary))
    for r in rows:
        assert set(r["lam"]) == set(LS.rule_names())
        assert all(lam in grid for lam in r["lam"].values())
        assert all(0.0 < e < 1.0 for e in r["err"].values())
        assert min(r["err"].values()) == r["err"]["best"]
        assert r["err"]["opt"] <= 1.5 * r["err"]["best"]


def _xlam_large(prob, lam, kp):
    """The oracle's settled x_lambda for a large problem: FP64 KP-PCG to a
    true residual of 1e-13, accepted only if a run at a 100x looser
    tolerance agrees with it (check=True), converged, with its true
    residual at or below 1e-12."""
    key = ("large", prob.seed, lam)
    if key not in _XLAM:
        x, info = SV.x_lambda_iterative(prob.psf, prob.b.astype(np.float64), lam, kp=kp,
                                        check=True)
        say(f"  oracle x_lambda: iters={info['iters']} status={info['status']} "
            f"true relres={info['true_relres']:.1e} loose agreement "
            f"{info['loose_agreement']:.1e}")
        assert info["status"] == "converged" and info["true_relres"] <= 1e-12
        _XLAM[key] = x
    return _XLAM[key]


# (mode, tol, bar): the FP32 modes are held to 1e-5 at a tolerance whose
# true residuals use the FP64 data misfit b - A x; the reduced-precision
# preconditioners to 1e-4
LARGE_CASES = [("fpcg16", 1e-6, 1e-4), ("fpcg8", 1e-6, 1e-4), ("pcg32", 1e-7, 1e-5),
               ("fpcg32", 1e-7, 1e-5)]


@pytest.mark.parametrize("mode,tol,bar", LARGE_CASES)
def test_large_moffat_full_size(mode, tol, bar):
    """1024 x 1024, Moffat + motion PSF (K = 63), lambda from the GPU's KP-GCV
    (same grid index as the oracle): the benchmark's configuration, checked
    against the oracle's x_lambda at full size."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_OK, Plan
    prob = S.large_moffat(0)
    grid = S.lambda_grid()
    say(f"large moffat {mode} tol={tol:g}")
    with Plan(prob.psf, prob.n) as plan:
        b = to_dev(prob.b)
        lam, _ = plan.gcv(b, grid)
        kp = KP.kp_svd(prob.psf, prob.n)
        s2, bh2 = L.spectrum(kp, prob.b.astype(np.float64))
        assert lam == grid[L.grid_argmin(L.gcv(s2, bh2, grid))]
        ref = _xlam_large(prob, lam, kp)
        x, info = plan.solve(b, lam, tol=tol, maxit=300, mode=_modes()[mode])
        err = rel(to_host(x), ref)
    say(f"  lam={lam:.4g} iters={info.iters} repl={info.replacements} err={err:.2e}")
    assert info.status == KP_OK and err <= bar


def test_fp32_fallback_after_reduced_precision_failure():
    """pcg_solve restarts a failed FP16/FP8 solve from its last iterate with
    the FP32 preconditioner: at 1024^2 the FP8 preconditioner needs more than
    10 iterations to reach 1e-6 (about 29), so with maxit = 10 the FP8 run
    stops at KP_MAXIT, and the FP32 restart (about 6 iterations from
    scratch) converges within its own 10.  KP_NO_FALLBACK keeps the failure."""
    require_gpu()
    from paper_2311_15393_amd import (KP_FPCG, KP_MAXIT, KP_NO_FALLBACK, KP_OK_FALLBACK, KP_P8,
                                      Plan)
    prob = S.large_moffat(0)
    grid = S.lambda_grid()
    with Plan(prob.psf, prob.n) as plan:
        b = to_dev(prob.b)
        lam, _ = plan.gcv(b, grid)
        x, info = plan.solve(b, lam, tol=1e-6, maxit=10, mode=KP_FPCG | KP_P8 | KP_NO_FALLBACK,
                             raise_on_fail=False)
        say(f"  fp8, no fallback: status={info.status} iters={info.iters}")
        assert info.status == KP_MAXIT and info.iters == 10 and info.fallback == 0
        x, info = plan.solve(b, lam, tol=1e-6, maxit=10, mode=KP_FPCG | KP_P8)
        say(f"  fp8 + fallback: status={info.status} iters={info.iters} "
            f"relres={info.relres_true:.2e}")
        assert info.status == KP_OK_FALLBACK and info.fallback == 1
        assert 10 < info.iters <= 20 and info.relres_true <= 1e-6
        ref = _xlam_large(prob, lam, KP.kp_svd(prob.psf, prob.n))
        assert rel(to_host(x), ref) <= 1e-4
