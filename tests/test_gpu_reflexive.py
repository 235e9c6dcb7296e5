"""Reflexive boundary (KP_BC_REFLEXIVE, PSFs symmetric in both axes) through
the C ABI, against the FP64 reflexive oracle (oracle/reflexive.py): blur
kernels elementwise (A and A^T, equal here), reflexive factor SVDs, solves
against the DCT closed-form x_lambda, the exact diagonal, a mixed batch,
the refusals, and the largest image size under both non-zero boundaries."""
import numpy as np
import pytest

import synthetic as S
from oracle import kp as KP
from oracle import reflexive as RB
from tests.gpu_util import rel, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _psf(kind, k, seed=0):
    rng = np.random.default_rng(seed)
    if kind == "defocus":
        return S.psf_defocus(k, min(6.0, (k - 1) / 2.0))
    if kind == "gauss":
        return S.psf_gaussian(k, 2.0 + k / 20, 1.5, 0.0)
    p = rng.uniform(0, 1, (k, k))
    p = p + p[::-1, :] + p[:, ::-1] + p[::-1, ::-1]
    return (p / p.sum()).astype(np.float32).astype(np.float64)


def _problem(n, k, kind, seed, noise=0.02):
    rng = np.random.default_rng(2000 + seed)
    psf = _psf(kind, k, seed)
    x = S.true_image(rng, n)
    ax = RB.blur_dct(psf, x)
    e = rng.standard_normal((n, n))
    b = ax + noise * np.linalg.norm(ax) / np.linalg.norm(e) * e
    return psf, b.astype(np.float32)


@pytest.mark.parametrize("n,k,kind", [(64, 15, "sym"), (100, 15, "defocus"), (131, 63, "sym"),
                                      (37, 9, "sym"), (15, 15, "sym"), (1024, 63, "defocus")])
@pytest.mark.parametrize("cfg", [0, 6, 7])
def test_reflexive_blur_matches_oracle(n, k, kind, cfg):
    """Both orientations of the blur against the reflexive A (A^T = A for
    these PSFs), with the bounds of the zero-boundary blur test; (15, 15)
    has K = n: every tap reflects somewhere."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, Plan
    say(f"reflexive blur n={n} k={k} {kind} cfg={cfg}")
    psf = _psf(kind, k, n)
    x = S.random_image(np.random.default_rng(n + k), n)
    x64 = x.astype(np.float64)
    if cfg in (6, 7):
        t = 3 * k * k + 4
        g = t * U32 / (1 - t * U32) + 2.0 ** -20
    else:
        g = (k * k + 1) * U32 / (1 - (k * k + 1) * U32)
    op = RB.blur_dct if n > 200 else RB.blur
    ref = op(psf, x64)
    absref = op(np.abs(psf), np.abs(x64))
    bound = g * absref + U32 * np.abs(ref) + 1e-13 * np.abs(absref).max()
    if cfg in (6, 7):
        bound = bound + 2.0 ** -30 * np.abs(x64).max() * np.abs(psf).sum()
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        plan.set_blur_config(cfg)
        for tr in (False, True):
            y = torch.empty_like(to_dev(x))
            plan.blur(to_dev(x), y, transpose=tr)
            got = to_host(y)
            assert np.all(np.abs(got - ref) <= bound), (tr, np.max(np.abs(got - ref) / bound))


@pytest.mark.parametrize("n,k,kind", [(64, 15, "sym"), (100, 31, "defocus"), (256, 31, "sym")])
def test_reflexive_factors_match_oracle(n, k, kind):
    """Reflexive (Toeplitz-plus-Hankel) factor singular values and Gram
    matrices V diag(s^2) V^T = A^T A against the oracle."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, Plan
    psf = _psf(kind, k, 5)
    kp = RB.kp_svd(psf, n)
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        sc, sr, vc, vr = plan.factors()
    assert np.allclose(sc, kp.sc, rtol=1e-10, atol=1e-13 * kp.sc[0])
    assert np.allclose(sr, kp.sr, rtol=1e-10, atol=1e-13 * kp.sr[0])
    assert np.allclose((vc * sc ** 2) @ vc.T, kp.Ac.T @ kp.Ac, atol=1e-5 * sc[0] ** 2)
    assert np.allclose((vr * sr ** 2) @ vr.T, kp.Ar.T @ kp.Ar, atol=1e-5 * sr[0] ** 2)


@pytest.mark.parametrize("mode", ["fpcg16", "pcg32", "cg", "fpcg8", "fpcg16diag"])
def test_reflexive_solve_matches_closed_form(mode):
    """Solves at 256^2 (K = 31, random doubly symmetric PSF) reach the DCT
    closed-form x_lambda to 1e-4, and the reported true residual agrees with
    the oracle's ||c - H x|| / ||c|| to a tenth of the tolerance plus twice
    the residual that rounding x_lambda to FP32 causes (the returned x is
    FP32, the certificate is for the FP64 iterate).  The broad
    random PSF at lambda = 0.01 is worse conditioned than the Moffat case of
    the other boundaries: tol 1e-7 left x at 1.04e-4, so tol is 2e-8."""
    require_gpu()
    from paper_2311_15393_amd import (KP_BC_REFLEXIVE, KP_CG, KP_FPCG, KP_OK, KP_P16, KP_P32,
                                      KP_PCG, KP_P8, KP_EXACT_DIAG, Plan)
    n, k, lam, tol = 256, 31, 0.01, 2e-8
    psf, b = _problem(n, k, "sym", 1)
    b64 = b.astype(np.float64)
    m = {"fpcg16": KP_FPCG | KP_P16, "pcg32": KP_PCG | KP_P32, "cg": KP_CG,
         "fpcg8": KP_FPCG | KP_P8, "fpcg16diag": KP_FPCG | KP_P16 | KP_EXACT_DIAG}[mode]
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        x, info = plan.solve(to_dev(b), lam, tol=tol, maxit=3000, mode=m)
        got = to_host(x)
    ref = RB.x_lambda(psf, b64, lam)
    op = RB.NormalOperator(psf, n, lam)
    c = op.At(b64)
    rr = float(np.linalg.norm(c - op.H(got)) / np.linalg.norm(c))
    # the device certifies its FP64 iterate and returns it in FP32: the
    # residual of fl32(x_lambda) measures what that rounding alone adds
    floor = float(np.linalg.norm(c - op.H(ref.astype(np.float32).astype(np.float64)))
                  / np.linalg.norm(c))
    err = rel(got, ref)
    say(f"reflexive {mode}: iters={info.iters} err={err:.2e} relres_true={info.relres_true:.3e} "
        f"oracle={rr:.3e} fp32 floor={floor:.1e}")
    assert info.status == KP_OK and err <= 1e-4
    assert abs(info.relres_true - rr) <= 0.1 * tol + 2 * floor


def test_reflexive_full_size_fp16():
    """1024^2, K = 63 defocus disk, 2% noise, lambda by the device's KP-GCV:
    FP16-KP FPCG reaches the DCT closed form to 1e-4, and its reported true
    residual agrees with the oracle's to a tenth of the tolerance.  The disk
    is far from rank one (the one-term preconditioner's weak case), so the
    solve needs tol 2e-7 where the Moffat + motion workload needs 2e-6."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, KP_FPCG, KP_OK, KP_P16, Plan
    n, k, tol = 1024, 63, 2e-7
    psf, b = _problem(n, k, "defocus", 0)
    b64 = b.astype(np.float64)
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        lam, _ = plan.gcv(to_dev(b), S.lambda_grid())
        x, info = plan.solve(to_dev(b), lam, tol=tol, maxit=500, mode=KP_FPCG | KP_P16)
        got = to_host(x)
    err = rel(got, RB.x_lambda(psf, b64, lam))
    op = RB.NormalOperator(psf, n, lam)
    c = op.At(b64)
    rr = float(np.linalg.norm(c - op.H(got)) / np.linalg.norm(c))
    say(f"reflexive 1024: lam={lam:.4g} iters={info.iters} err={err:.2e} "
        f"relres_true={info.relres_true:.3e} oracle={rr:.3e}")
    assert info.status == KP_OK and err <= 1e-4
    assert abs(info.relres_true - rr) <= 0.1 * tol


def test_reflexive_exact_diag_and_batch():
    """The exact diagonal against the oracle's formed in the device's basis
    (FP32 V: 1e-6 relative plus 1e-9 max), and a batch mixing reflexive,
    periodic and zero-boundary plans reaching every item's x_lambda.  The
    reflexive items use the defocus disk at lambda 0.01 and 0.03: at 0.003
    the one-term preconditioner of the disk leaves more than 2000 iterations
    to tol 1e-8."""
    require_gpu()
    from paper_2311_15393_amd import (KP_BC_PERIODIC, KP_BC_REFLEXIVE, KP_FPCG, KP_OK, KP_P16,
                                      Plan, solve_batched)
    from oracle import periodic as PB
    from oracle import solvers as SV
    psf = _psf("sym", 15, 21)
    kp = RB.kp_svd(psf, 96)
    with Plan(psf, 96, bc=KP_BC_REFLEXIVE) as plan:
        got = plan.exact_diag().astype(np.float64)
        _, _, vc, vr = plan.factors()
    kp.Vc, kp.Vr = vc.astype(np.float64), vr.astype(np.float64)
    ref = RB.exact_diag(kp, psf)
    assert np.all(np.abs(got - ref) <= 1e-6 * np.abs(ref) + 1e-9 * ref.max())
    pr, br = _problem(128, 15, "defocus", 4)
    pp = _psf("sym", 31, 6)
    bp = S.random_image(np.random.default_rng(9), 160)
    pz = S.mid_anisotropic(1, n=128)
    plans = [Plan(pr, 128, bc=KP_BC_REFLEXIVE), Plan(pp, 160, bc=KP_BC_PERIODIC),
             Plan(pz.psf, 128)]
    items = [(0, 0.01), (1, 0.02), (2, 0.01), (0, 0.03)]
    datas = [br, bp, pz.b]
    refs = [RB.x_lambda(pr, br.astype(np.float64), lam) if p == 0 else
            PB.x_lambda(pp, bp.astype(np.float64), lam) if p == 1 else
            SV.x_lambda(pz.psf, pz.b.astype(np.float64), lam) for p, lam in items]
    xs, infos, st = solve_batched(plans, [to_dev(datas[p]) for p, _ in items],
                                  [l for _, l in items], [p for p, _ in items], tol=1e-8,
                                  maxit=2000, mode=KP_FPCG | KP_P16)
    for (p, lam), xd, inf, r in zip(items, xs, infos, refs):
        e = rel(to_host(xd), r)
        say(f"  batch plan {p} lam={lam}: iters={inf.iters} err={e:.2e}")
        assert inf.status == KP_OK and e <= 1e-4
    assert st == KP_OK
    for pl in plans:
        pl.close()


def test_reflexive_refusals():
    """K > n is refused; a PSF not symmetric in both axes is accepted and
    takes the FFT form of the normal operator (its A^T is no blur)."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, KP_NORMAL_FFT, KPError, Plan
    from paper_2311_15393_amd.kpcg import KP_ERR_ARG
    asym = S.psf_moffat_motion(15, 4.0, 2.5, 6.0, 0.7)
    with Plan(asym, 64, bc=KP_BC_REFLEXIVE) as plan:
        assert plan.query()["normal_op"] == KP_NORMAL_FFT
    with pytest.raises(KPError) as ei:
        Plan(_psf("sym", 17, 0), 15, bc=KP_BC_REFLEXIVE)
    assert ei.value.status == KP_ERR_ARG


@pytest.mark.parametrize("bc_name", ["periodic", "reflexive"])
def test_maximum_size_other_boundaries(bc_name):
    """The largest image (2048 x 2048) with the largest PSF (K = 63) under
    the periodic and the reflexive boundary: FP16-KP FPCG reaches the
    closed-form x_lambda (2-D DFT or DCT) to 1e-4."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_PERIODIC, KP_BC_REFLEXIVE, KP_FPCG, KP_OK, KP_P16, Plan
    from oracle import periodic as PB
    if bc_name == "periodic":
        prob, bc, ref_mod = S.large_moffat_periodic(3, n=2048, k=63), KP_BC_PERIODIC, PB
    else:
        prob, bc, ref_mod = S.large_moffat_reflexive(3, n=2048, k=63), KP_BC_REFLEXIVE, RB
    lam = 0.03
    say(f"maximum size 2048^2, K = 63, {bc_name}")
    ref = ref_mod.x_lambda(prob.psf, prob.b.astype(np.float64), lam)
    with Plan(prob.psf, prob.n, bc=bc) as plan:
        x, info = plan.solve(to_dev(prob.b), lam, tol=1e-6, maxit=200, mode=KP_FPCG | KP_P16)
        got = to_host(x)
    err = rel(got, ref)
    say(f"  iters={info.iters} relres_true={info.relres_true:.2e} err={err:.2e}")
    assert info.status == KP_OK and err <= 1e-4
