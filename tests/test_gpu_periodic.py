"""Periodic boundary (KP_BC_PERIODIC) through the C ABI, against the FP64
periodic oracle (oracle/periodic.py): blur kernels elementwise, circulant
factor SVDs, KP-basis GCV, solves against the DFT closed-form x_lambda, and
the modes a periodic plan refuses."""
import numpy as np
import pytest

import synthetic as S
from oracle import kp as KP
from oracle import lam as L
from oracle import periodic as PB
from tests.gpu_util import rel, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _psf(kind, k, seed=0):
    rng = np.random.default_rng(seed)
    if kind == "gauss":
        return S.psf_gaussian(k, 2.0 + k / 20, 1.5, 0.4)
    if kind == "moffat":
        return S.psf_moffat_motion(k, rng.uniform(3, 8), 2.5, rng.uniform(3, 9),
                                   rng.uniform(0, np.pi))
    p = rng.uniform(0, 1, (k, k))
    return (p / p.sum()).astype(np.float32).astype(np.float64)


def _problem(n, k, kind, seed, noise=0.02):
    """b = A x_true + e with the periodic A, ||e|| = noise ||A x_true||,
    rounded to FP32 (the device's input)."""
    rng = np.random.default_rng(1000 + seed)
    psf = _psf(kind, k, seed)
    x = S.true_image(rng, n)
    ax = PB.blur_fft(psf, x)
    e = rng.standard_normal((n, n))
    b = ax + noise * np.linalg.norm(ax) / np.linalg.norm(e) * e
    return psf, x, b.astype(np.float32)


BLUR_CASES = [(64, 15, "gauss"), (100, 15, "rand"), (131, 63, "moffat"), (37, 9, "rand"),
              (15, 15, "rand"), (200, 31, "moffat"), (1024, 63, "moffat")]


@pytest.mark.parametrize("n,k,kind", BLUR_CASES)
@pytest.mark.parametrize("cfg", [0, 6, 7])
def test_periodic_blur_matches_oracle(n, k, kind, cfg):
    """Periodic A and A^T vs FP64, elementwise, with the bounds of the
    zero-boundary blur test (the wrap changes which inputs enter a sum, not
    how it is formed):
      VALU:  |y - y64| <= gamma_{K^2+1} (|P| * |x|) + u |y|
      MFMA:  |y - y64| <= (gamma_{3K^2+1} + 2^-20) (|P| * |x|) + u |y|
                          + 2^-30 max|x| sum|P|
    with * the periodic convolution.  (15, 15) has K = n: every tap wraps."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_BC_PERIODIC, Plan
    say(f"periodic blur n={n} k={k} {kind} cfg={cfg}")
    psf = _psf(kind, k, n)
    x = S.random_image(np.random.default_rng(n + k), n)
    x64 = x.astype(np.float64)
    if cfg in (6, 7):
        t = 3 * k * k + 4
        g = t * U32 / (1 - t * U32) + 2.0 ** -20
    else:
        g = (k * k + 1) * U32 / (1 - (k * k + 1) * U32)
    fwd = PB.blur_fft if n > 200 else PB.blur
    adj = PB.blur_t_fft if n > 200 else PB.blur_t
    with Plan(psf, n, bc=KP_BC_PERIODIC) as plan:
        plan.set_blur_config(cfg)
        for tr in (False, True):
            y = torch.empty_like(to_dev(x))
            plan.blur(to_dev(x), y, transpose=tr)
            got = to_host(y)
            ref = adj(psf, x64) if tr else fwd(psf, x64)
            absref = (adj if tr else fwd)(np.abs(psf), np.abs(x64))
            bound = g * absref + U32 * np.abs(ref)
            if cfg in (6, 7):
                bound = bound + 2.0 ** -30 * np.abs(x64).max() * np.abs(psf).sum()
            # the DFT reference itself carries ~1e-15 relative error
            bound = bound + 1e-13 * np.abs(absref).max()
            assert np.all(np.abs(got - ref) <= bound), (tr, np.max(np.abs(got - ref) / bound))


@pytest.mark.parametrize("n,k,kind", [(64, 15, "moffat"), (100, 31, "rand"), (256, 31, "moffat"),
                                      (63, 63, "gauss")])
def test_periodic_factors_match_oracle(n, k, kind):
    """Circulant factor singular values (device FP64 SVD) and the KP error
    match the oracle; V through the sign- and rotation-free projector
    V diag(s^2) V^T = A^T A (a real circulant's singular values come in
    equal pairs, so V itself is not unique)."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_PERIODIC, Plan
    say(f"periodic factors n={n} k={k} {kind}")
    psf = _psf(kind, k, 5)
    kp = PB.kp_svd(psf, n)
    with Plan(psf, n, bc=KP_BC_PERIODIC) as plan:
        info = plan.query()
        sc, sr, vc, vr = plan.factors()
    assert np.allclose(sc, kp.sc, rtol=1e-10, atol=1e-13 * kp.sc[0])
    assert np.allclose(sr, kp.sr, rtol=1e-10, atol=1e-13 * kp.sr[0])
    assert abs(info["kp_rel_error"] - KP.kp_error(kp.s_psf)) <= 1e-10
    assert np.allclose((vc * sc ** 2) @ vc.T, kp.Ac.T @ kp.Ac, atol=1e-5 * sc[0] ** 2)
    assert np.allclose((vr * sr ** 2) @ vr.T, kp.Ar.T @ kp.Ar, atol=1e-5 * sr[0] ** 2)


def test_periodic_gcv_matches_oracle():
    """KP-basis GCV (eq. (GCVTikSVD)) with the circulant factors: the same
    grid choice and scores to 1e-5 (sums of b_hat^2 within a pair of equal
    singular values do not depend on the basis chosen for the pair)."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_PERIODIC, Plan
    psf, _, b = _problem(256, 31, "moffat", 3)
    grid = S.lambda_grid()
    kp = PB.kp_svd(psf, 256)
    s2, bh2 = L.spectrum(kp, b.astype(np.float64))
    g_ref = L.gcv(s2, bh2, grid)
    with Plan(psf, 256, bc=KP_BC_PERIODIC) as plan:
        lam_g, g = plan.gcv(to_dev(b), grid)
    say(f"periodic gcv lam={lam_g:.4g}")
    assert lam_g == grid[L.grid_argmin(g_ref)]
    assert np.allclose(g, g_ref, rtol=1e-5)


@pytest.mark.parametrize("mode", ["fpcg16", "pcg32", "cg", "fpcg8", "fpcg16diag"])
def test_periodic_solve_matches_closed_form(mode):
    """Solves at 256^2 (K = 31) reach the DFT closed-form x_lambda to 1e-4,
    and the reported true residual agrees with the oracle's ||c - H x|| /
    ||c|| at the returned x to a tenth of the tolerance plus twice the
    residual that rounding x_lambda to FP32 causes (the returned x is FP32,
    the certificate is for the FP64 iterate)."""
    require_gpu()
    from paper_2311_15393_amd import (KP_BC_PERIODIC, KP_CG, KP_FPCG, KP_OK, KP_P16, KP_P32,
                                      KP_PCG, KP_P8, KP_EXACT_DIAG, Plan)
    n, k, lam, tol = 256, 31, 0.01, 1e-7
    psf, _, b = _problem(n, k, "moffat", 1)
    b64 = b.astype(np.float64)
    m = {"fpcg16": KP_FPCG | KP_P16, "pcg32": KP_PCG | KP_P32, "cg": KP_CG,
         "fpcg8": KP_FPCG | KP_P8, "fpcg16diag": KP_FPCG | KP_P16 | KP_EXACT_DIAG}[mode]
    with Plan(psf, n, bc=KP_BC_PERIODIC) as plan:
        x, info = plan.solve(to_dev(b), lam, tol=tol, maxit=3000, mode=m)
        got = to_host(x)
    ref = PB.x_lambda(psf, b64, lam)
    op = PB.NormalOperator(psf, n, lam)
    c = op.At(b64)
    rr = float(np.linalg.norm(c - op.H(got)) / np.linalg.norm(c))
    # the device certifies its FP64 iterate and returns it in FP32: the
    # residual of fl32(x_lambda) measures what that rounding alone adds
    floor = float(np.linalg.norm(c - op.H(ref.astype(np.float32).astype(np.float64)))
                  / np.linalg.norm(c))
    err = rel(got, ref)
    say(f"periodic {mode}: iters={info.iters} err={err:.2e} relres_true={info.relres_true:.3e} "
        f"oracle={rr:.3e} fp32 floor={floor:.1e}")
    assert info.status == KP_OK and err <= 1e-4
    assert abs(info.relres_true - rr) <= 0.1 * tol + 2 * floor


def test_periodic_full_size_fp16():
    """1024^2, K = 63 Moffat + motion, 2% noise, lambda by the device's
    KP-GCV on the 32-point grid: FP16-KP FPCG at tol 2e-6 reaches the DFT
    closed form to 1e-4 (the benchmark's bar)."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_PERIODIC, KP_FPCG, KP_OK, KP_P16, Plan
    n, k = 1024, 63
    psf, _, b = _problem(n, k, "moffat", 0)
    with Plan(psf, n, bc=KP_BC_PERIODIC) as plan:
        lam, _ = plan.gcv(to_dev(b), S.lambda_grid())
        x, info = plan.solve(to_dev(b), lam, tol=2e-6, maxit=500, mode=KP_FPCG | KP_P16)
        got = to_host(x)
    err = rel(got, PB.x_lambda(psf, b.astype(np.float64), lam))
    say(f"periodic 1024: lam={lam:.4g} iters={info.iters} err={err:.2e}")
    assert info.status == KP_OK and err <= 1e-4


def test_periodic_exact_diag_matches_oracle():
    """kp_setup's exact KP-basis diagonal for a periodic plan against the
    oracle's circulant form.  A real circulant's singular vectors are not
    unique within its pairs of equal singular values, so the oracle's D0 is
    formed in the device's own basis (its FP32 V): FP32 rounding of V and of
    D0 bound the difference by 1e-6 relative plus 1e-9 max(D0)."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_PERIODIC, Plan
    for n, k, kind in ((64, 15, "moffat"), (100, 9, "rand"), (128, 63, "moffat")):
        psf = _psf(kind, k, 21)
        kp = PB.kp_svd(psf, n)
        with Plan(psf, n, bc=KP_BC_PERIODIC) as plan:
            got = plan.exact_diag().astype(np.float64)
            sc, sr, vc, vr = plan.factors()
        kp.Vc, kp.Vr = vc.astype(np.float64), vr.astype(np.float64)
        ref = PB.exact_diag(kp, psf)
        err = np.abs(got - ref)
        say(f"periodic exact diagonal n={n} k={k}: max err / max {err.max() / ref.max():.2e}")
        assert np.all(err <= 1e-6 * np.abs(ref) + 1e-9 * ref.max())


def test_periodic_exact_diag_solve_and_batch():
    """A periodic solve with KP_EXACT_DIAG reaches the DFT closed form, and a
    batch mixing periodic and zero-boundary plans (FP16-KP FPCG, one-term
    and exact-diagonal S) reaches every item's own x_lambda to 1e-4."""
    require_gpu()
    from paper_2311_15393_amd import (KP_BC_PERIODIC, KP_EXACT_DIAG, KP_FPCG, KP_OK, KP_P16, Plan,
                                      solve_batched)
    from oracle import solvers as SV
    pa, _, ba = _problem(128, 15, "moffat", 4)
    pb, _, bb = _problem(200, 31, "gauss", 5)
    pz = S.mid_anisotropic(1, n=128)
    plans = [Plan(pa, 128, bc=KP_BC_PERIODIC), Plan(pb, 200, bc=KP_BC_PERIODIC),
             Plan(pz.psf, 128)]
    x, info = plans[0].solve(to_dev(ba), 0.01, tol=1e-7, maxit=500,
                             mode=KP_FPCG | KP_P16 | KP_EXACT_DIAG)
    err = rel(to_host(x), PB.x_lambda(pa, ba.astype(np.float64), 0.01))
    say(f"periodic exact-diag solve: iters={info.iters} err={err:.2e}")
    assert info.status == KP_OK and err <= 1e-4
    items = [(0, 0.01), (0, 0.003), (1, 0.02), (2, 0.01)]
    bs = [to_dev([ba, bb, pz.b][p]) for p, _ in items]
    refs = [PB.x_lambda(pa, ba.astype(np.float64), lam) if p == 0 else
            PB.x_lambda(pb, bb.astype(np.float64), lam) if p == 1 else
            SV.x_lambda(pz.psf, pz.b.astype(np.float64), lam) for p, lam in items]
    for extra in (0, KP_EXACT_DIAG):
        xs, infos, st = solve_batched(plans, bs, [l for _, l in items], [p for p, _ in items],
                                      tol=1e-8, maxit=2000, mode=KP_FPCG | KP_P16 | extra)
        for (p, lam), xd, inf, ref in zip(items, xs, infos, refs):
            e = rel(to_host(xd), ref)
            say(f"  batch{'+diag' if extra else ''} plan {p} lam={lam}: iters={inf.iters} "
                f"err={e:.2e}")
            assert inf.status == KP_OK and e <= 1e-4
        assert st == KP_OK
    for pl in plans:
        pl.close()


def test_periodic_refusals():
    """kp_setup refuses a periodic PSF larger than the image (it would wrap
    onto itself) and an unknown boundary value."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_PERIODIC, KPError, Plan
    from paper_2311_15393_amd.kpcg import KP_ERR_ARG, KP_ERR_UNSUPPORTED
    with pytest.raises(KPError) as ei:
        Plan(_psf("rand", 17, 0), 15, bc=KP_BC_PERIODIC)
    assert ei.value.status == KP_ERR_ARG
    with pytest.raises(KPError) as ei:
        Plan(_psf("gauss", 15, 0), 64, bc=3)
    assert ei.value.status == KP_ERR_UNSUPPORTED
