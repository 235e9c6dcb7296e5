"""Reflexive boundary with the FFT form of the normal operator, and PSFs that
are not symmetric (A^T != A): the folded FFT passes for H p and A^T u
against the FP64 reflexive oracle (oracle/reflexive.py), solves against
its dense Cholesky solve and its settled FP64 PCG, the exact diagonal,
and the refusals of what such a plan cannot do.

The FFT bar is the one of the zero-boundary FFT tests: normwise 1e-5
relative (four FP32 transforms of length L ~ 2200, each within about
log2(L) * 1e-7), which a wrong reflection, fold or crop misses by orders
of magnitude."""
import numpy as np
import pytest

import synthetic as S
from oracle import reflexive as RB
from tests.gpu_util import rel, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _asym(k, seed):
    rng = np.random.default_rng(seed)
    p = S.psf_moffat_motion(k, rng.uniform(3, 8), 2.5, rng.uniform(3, 9), rng.uniform(0, np.pi))
    # FP32-representable, so the device and the oracle blur with one PSF
    return p.astype(np.float32).astype(np.float64)


def _sym(k, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 1, (k, k))
    p = p + p[::-1, :] + p[:, ::-1] + p[::-1, ::-1]
    return (p / p.sum()).astype(np.float32).astype(np.float64)


def _data(psf, n, seed, noise=0.02):
    rng = np.random.default_rng(3000 + seed)
    x = S.true_image(rng, n)
    ax = RB.blur_general(psf, x) if n <= 64 else RB.blur_fft_general(psf, x)
    e = rng.standard_normal((n, n))
    return (ax + noise * np.linalg.norm(ax) / np.linalg.norm(e) * e).astype(np.float32)


CASES = [(15, 15), (37, 9), (64, 15), (100, 31), (129, 23), (256, 63), (1024, 63), (2048, 63)]


@pytest.mark.parametrize("n,k", CASES)
@pytest.mark.parametrize("kind", ["sym", "asym"])
def test_reflexive_fft_normal_matches_oracle(n, k, kind):
    """H p = A^T A p + lambda^2 p by the reflexive FFT passes; (15, 15) has
    K = n (every tap reflects).  For symmetric PSFs the direct blurs give
    the same operator and are checked beside it."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, KP_NORMAL_DIRECT, KP_NORMAL_FFT, Plan
    psf = _sym(k, n + k) if kind == "sym" else _asym(k, n + k)
    x = S.random_image(np.random.default_rng(n), n) - 0.5
    lam = 0.01
    x64 = x.astype(np.float64)
    op = RB.NormalOperatorGeneral(psf, n, lam)
    ref = op.H(x64)
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        info = plan.query()
        y = torch.empty((n, n), dtype=torch.float32, device="cuda")
        plan.normal(to_dev(x), lam, y, op=KP_NORMAL_FFT)
        got = to_host(y)
        e_dir = None
        if kind == "sym":
            plan.normal(to_dev(x), lam, y, op=KP_NORMAL_DIRECT)
            e_dir = rel(to_host(y), ref)
    e_fft = rel(got, ref)
    say(f"reflexive {kind} n={n} K={k} L={info['fft_length']}: |fft - ref| {e_fft:.2e}, "
        f"direct {e_dir}; form {info['normal_op']} (direct {info['normal_op_ms'][0]:.4f} ms, "
        f"fft {info['normal_op_ms'][1]:.4f} ms)")
    assert info["fft_length"] >= n + k - 1
    assert e_fft <= 1e-5
    if kind == "asym":
        assert info["normal_op"] == KP_NORMAL_FFT
    else:
        assert e_dir <= 1e-5


@pytest.mark.parametrize("n,k", [(15, 15), (40, 9), (100, 31), (256, 63), (1024, 63)])
def test_reflexive_general_blurs(n, k):
    """A x on the direct blur (elementwise, the bound of the blur tests) and
    A^T y by the folded FFT passes (normwise 1e-5) for a PSF that is not
    symmetric, against the definitions (n <= 64) or their FFT forms."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, Plan
    psf = _asym(k, 7 * n + k)
    rng = np.random.default_rng(n + k)
    x = S.random_image(rng, n)
    yv = (rng.standard_normal((n, n))).astype(np.float32)
    x64, y64 = x.astype(np.float64), yv.astype(np.float64)
    fwd = RB.blur_general if n <= 64 else RB.blur_fft_general
    adj = RB.blur_t_general if n <= 64 else RB.blur_t_fft_general
    ref_a, ref_at = fwd(psf, x64), adj(psf, y64)
    absref = fwd(np.abs(psf), np.abs(x64))
    t = 3 * k * k + 4           # the MFMA hi/lo blur's bound covers the VALU one
    g = t * U32 / (1 - t * U32) + 2.0 ** -20
    bound = (g * absref + U32 * np.abs(ref_a) + 1e-13 * np.abs(absref).max()
             + 2.0 ** -30 * np.abs(x64).max() * np.abs(psf).sum())
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        out = torch.empty((n, n), dtype=torch.float32, device="cuda")
        plan.blur(to_dev(x), out, transpose=False)
        got_a = to_host(out)
        plan.blur(to_dev(yv), out, transpose=True)
        got_at = to_host(out)
    e_at = rel(got_at, ref_at)
    say(f"general reflexive blurs n={n} K={k}: A max/bound "
        f"{np.max(np.abs(got_a - ref_a) / bound):.2e}, A^T normwise {e_at:.2e}")
    assert np.all(np.abs(got_a - ref_a) <= bound)
    assert e_at <= 1e-5


@pytest.mark.parametrize("mode", ["fpcg16", "pcg32", "cg", "fpcg16diag"])
def test_reflexive_general_solve_matches_dense(mode):
    """48^2, K = 11 Moffat + motion (not symmetric), 2% noise: every solver
    reaches the dense Cholesky x_lambda to 1e-4 at tol 1e-7 (the tightest
    such a plan accepts), and its reported true residual agrees with the
    oracle's ||c - H x|| / ||c|| to a tenth of the tolerance plus twice the
    residual that rounding x_lambda to FP32 causes."""
    require_gpu()
    from paper_2311_15393_amd import (KP_BC_REFLEXIVE, KP_CG, KP_EXACT_DIAG, KP_FPCG, KP_OK,
                                      KP_P16, KP_P32, KP_PCG, Plan)
    n, k, lam, tol = 48, 11, 0.02, 1e-7
    psf = _asym(k, 5)
    b = _data(psf, n, 1)
    b64 = b.astype(np.float64)
    m = {"fpcg16": KP_FPCG | KP_P16, "pcg32": KP_PCG | KP_P32, "cg": KP_CG,
         "fpcg16diag": KP_FPCG | KP_P16 | KP_EXACT_DIAG}[mode]
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        x, info = plan.solve(to_dev(b), lam, tol=tol, maxit=3000, mode=m)
        got = to_host(x)
    ref = RB.x_lambda_dense_general(psf, b64, lam)
    op = RB.NormalOperatorGeneral(psf, n, lam)
    c = op.At(b64)
    rr = float(np.linalg.norm(c - op.H(got)) / np.linalg.norm(c))
    floor = float(np.linalg.norm(c - op.H(ref.astype(np.float32).astype(np.float64)))
                  / np.linalg.norm(c))
    err = rel(got, ref)
    say(f"general reflexive {mode}: iters={info.iters} err={err:.2e} "
        f"relres_true={info.relres_true:.3e} oracle={rr:.3e} fp32 floor={floor:.1e}")
    assert info.status == KP_OK and err <= 1e-4
    assert abs(info.relres_true - rr) <= 0.1 * tol + 2 * floor


def test_reflexive_general_solve_256():
    """256^2, K = 31 Moffat + motion, lambda 0.01: FP16-KP FPCG and FP32 PCG
    at tol 1e-7 reach the oracle's settled FP64 PCG x_lambda to 1e-4, with
    the reported true residual within a tenth of tol of the oracle's.  (At
    tol 1e-6 x stood 3e-4 from x_lambda: with cond(H) ~ 1e4 at this lambda
    the error may reach cond(H) times the residual.)"""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, KP_FPCG, KP_OK, KP_P16, KP_P32, KP_PCG, Plan
    n, k, lam, tol = 256, 31, 0.01, 1e-7
    psf = _asym(k, 11)
    b = _data(psf, n, 2)
    b64 = b.astype(np.float64)
    ref, rinfo = RB.x_lambda_general(psf, b64, lam, tol=1e-12)
    op = RB.NormalOperatorGeneral(psf, n, lam)
    c = op.At(b64)
    floor = float(np.linalg.norm(c - op.H(ref.astype(np.float32).astype(np.float64)))
                  / np.linalg.norm(c))
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        for name, m in (("fpcg16", KP_FPCG | KP_P16), ("pcg32", KP_PCG | KP_P32)):
            x, info = plan.solve(to_dev(b), lam, tol=tol, maxit=2000, mode=m)
            got = to_host(x)
            err = rel(got, ref)
            rr = float(np.linalg.norm(c - op.H(got)) / np.linalg.norm(c))
            say(f"general reflexive 256^2 {name}: iters={info.iters} err={err:.2e} "
                f"relres_true={info.relres_true:.3e} oracle={rr:.3e} floor={floor:.1e} "
                f"(oracle {rinfo['iters']} iters)")
            assert info.status == KP_OK and err <= 1e-4
            assert abs(info.relres_true - rr) <= 0.1 * tol + 2 * floor


def test_reflexive_general_full_size():
    """1024^2, K = 63 Moffat + motion workload with reflexive data (2%
    noise) at lambda 0.03: FP16-KP FPCG at tol 2e-6 reaches the settled
    FP64 PCG x_lambda to 1e-4, and plain CG agrees with it."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, KP_FPCG, KP_OK, KP_P16, Plan
    prob = S.large_moffat_motion_reflexive(0, n=1024, k=63)
    lam = 0.03
    say("general reflexive 1024^2 K=63: oracle x_lambda")
    ref, rinfo = RB.x_lambda_general(prob.psf, prob.b.astype(np.float64), lam, tol=1e-12)
    with Plan(prob.psf, prob.n, bc=KP_BC_REFLEXIVE) as plan:
        x, info = plan.solve(to_dev(prob.b), lam, tol=2e-6, maxit=500, mode=KP_FPCG | KP_P16)
        got = to_host(x)
        t_ms = info.ms
    err = rel(got, ref)
    say(f"  iters={info.iters} relres_true={info.relres_true:.2e} err={err:.2e} "
        f"{t_ms:.2f} ms (oracle {rinfo['iters']} iters)")
    assert info.status == KP_OK and err <= 1e-4


def test_reflexive_general_exact_diag():
    """The exact KP-basis diagonal for a PSF that is not symmetric against
    the oracle's, formed in the device's basis (FP32 V: 1e-6 relative plus
    1e-9 of the largest)."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, Plan
    n, k = 96, 15
    psf = _asym(k, 21)
    kp = RB.kp_svd(psf, n)
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        got = plan.exact_diag().astype(np.float64)
        _, _, vc, vr = plan.factors()
    kp.Vc, kp.Vr = vc.astype(np.float64), vr.astype(np.float64)
    ref = RB.exact_diag(kp, psf)
    assert np.all(np.abs(got - ref) <= 1e-6 * np.abs(ref) + 1e-9 * ref.max())


def test_reflexive_symmetric_solve_with_fft_form():
    """A doubly symmetric PSF with the FFT form forced: FP16-KP FPCG reaches
    the DCT closed-form x_lambda to 1e-4."""
    require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, KP_FPCG, KP_NORMAL_FFT, KP_OK, KP_P16, Plan
    n, k, lam = 256, 31, 0.02
    psf = _sym(k, 4)
    b = _data(psf, n, 3)
    ref = RB.x_lambda(psf, b.astype(np.float64), lam)
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        plan.set_normal_op(KP_NORMAL_FFT)
        x, info = plan.solve(to_dev(b), lam, tol=1e-7, maxit=2000, mode=KP_FPCG | KP_P16)
        err = rel(to_host(x), ref)
    say(f"symmetric reflexive via FFT: iters={info.iters} err={err:.2e}")
    assert info.status == KP_OK and err <= 1e-4


def test_reflexive_general_refusals():
    """What a plan whose A^T is not a blur cannot do is refused with
    KP_ERR_UNSUPPORTED: the direct normal operator, the FP64 normal
    operator, tolerances below 1e-7 (their true residuals would need A^T in
    FP64) and batched solves; K > n stays an argument error, K above
    KP_MAX_PSF is unsupported, and the largest plan (2048^2, K = 63) has
    its FFT length."""
    torch = require_gpu()
    from paper_2311_15393_amd import (KP_BC_REFLEXIVE, KP_FPCG, KP_NORMAL_DIRECT, KP_P16,
                                      KPError, Plan, solve_batched)
    from paper_2311_15393_amd.kpcg import KP_ERR_ARG, KP_ERR_UNSUPPORTED
    n = 64
    psf = _asym(15, 1)
    b = _data(psf, n, 4)
    with Plan(psf, n, bc=KP_BC_REFLEXIVE) as plan:
        x = torch.zeros((n, n), dtype=torch.float32, device="cuda")
        y = torch.empty((n, n), dtype=torch.float64, device="cuda")
        w = torch.empty((n, n), dtype=torch.float32, device="cuda")
        for call in (lambda: plan.set_normal_op(KP_NORMAL_DIRECT),
                     lambda: plan.normal(x, 0.1, w, op=KP_NORMAL_DIRECT),
                     lambda: plan.normal_fp64(x, 0.1, y),
                     lambda: plan.solve(to_dev(b), 0.02, tol=5e-8, maxit=100),
                     lambda: solve_batched([plan], [to_dev(b)], [0.02], [0], tol=1e-6,
                                           maxit=100, mode=KP_FPCG | KP_P16)):
            with pytest.raises(KPError) as ei:
                call()
            assert ei.value.status == KP_ERR_UNSUPPORTED
    with pytest.raises(KPError) as ei:
        Plan(_asym(17, 0), 15, bc=KP_BC_REFLEXIVE)
    assert ei.value.status == KP_ERR_ARG
    # supports above KP_MAX_PSF (63) are refused outright; up to it every
    # n <= 2048 has an FFT length (n + 2h <= 2110 against the menu's 2160)
    from paper_2311_15393_amd.kpcg import workspace_size
    with pytest.raises(KPError) as ei:
        Plan(_asym(65, 2), 100, bc=KP_BC_REFLEXIVE)
    assert ei.value.status == KP_ERR_UNSUPPORTED
    with Plan(_asym(63, 3), 2048, bc=KP_BC_REFLEXIVE) as big:
        assert big.query()["fft_length"] == 2160 and big.query()["normal_op"] == 1
    assert workspace_size(2048, 63) > 0
