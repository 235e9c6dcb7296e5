"""Kernel-level parity of the HIP library against the FP64 oracle, through
the C ABI.  Tolerances are derived from the arithmetic (standard
floating-point summation bounds) and written in each test."""
import numpy as np
import pytest

import synthetic as S
from oracle import kp as KP
from oracle import operator as O
from oracle import quant as Q
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
    p = rng.uniform(0, 1, (k, k))                       # dense random PSF
    return (p / p.sum()).astype(np.float32).astype(np.float64)


BLUR_CASES = [(64, 15, "gauss"), (100, 15, "rand"), (256, 31, "gauss"), (131, 63, "moffat"),
              (37, 9, "rand"), (8, 15, "rand"), (1024, 63, "moffat")]


@pytest.mark.parametrize("n,k,kind", BLUR_CASES)
@pytest.mark.parametrize("cfg", [0, 6, 7])
def test_blur_matches_oracle(n, k, kind, cfg):
    """Blur vs FP64, elementwise.
    VALU shapes (cfg 0..5), FP32 products and sums in any order:
        |y - y64| <= gamma_{K^2+1} (|P| * |x|) + u |y|.
    MFMA kernels (cfg 6: 16x16x32, cfg 7: 32x32x16 instructions): x and P
    are split into FP16 hi + lo (scaled by
    powers of two), the hi*hi, hi*lo, lo*hi products are exact in FP32 and
    summed in FP32 (3 K^2 terms); the representation error and the dropped
    lo*lo term are each at most 2^-22 relative per product, and FP16
    underflow costs at most 2^-25 of the scaled unit per entry:
        |y - y64| <= (gamma_{3K^2+1} + 2^-20) (|P| * |x|) + u |y|
                     + 2^-30 max|x| sum|P|."""
    torch = require_gpu()
    from paper_2311_15393_amd import Plan
    say(f"blur n={n} k={k} {kind} cfg={cfg}")
    psf = _psf(kind, k, n)
    x = S.random_image(np.random.default_rng(n + k), n)
    xd = to_dev(x)
    if cfg in (6, 7):
        t = 3 * k * k + 4
        g = t * U32 / (1 - t * U32) + 2.0 ** -20
    else:
        g = (k * k + 1) * U32 / (1 - (k * k + 1) * U32)
    with Plan(psf, n) as plan:
        plan.set_blur_config(cfg)
        for tr in (False, True):
            y = torch.empty_like(xd)
            plan.blur(xd, y, transpose=tr)
            got = to_host(y)
            x64 = x.astype(np.float64)
            ref = O.blur_t(psf, x64) if tr else O.blur(psf, x64)
            absref = O.blur_t(np.abs(psf), np.abs(x64)) if tr else O.blur(np.abs(psf), np.abs(x64))
            bound = g * absref + U32 * np.abs(ref)
            if cfg in (6, 7):
                bound = bound + 2.0 ** -30 * np.abs(x64).max() * np.abs(psf).sum()
            assert np.all(np.abs(got - ref) <= bound), (tr, np.max(np.abs(got - ref) / bound))


@pytest.mark.parametrize("cfg", [6, 7])
def test_blur_mfma_high_dynamic_range(cfg):
    """MFMA blurs on an image whose tiles mix values of 1 and 1e-6 (worst case
    for a per-tile scale): the error stays within the MFMA bound above."""
    torch = require_gpu()
    from paper_2311_15393_amd import Plan
    n, k = 200, 31
    psf = _psf("moffat", k, 4)
    rng = np.random.default_rng(3)
    x = (rng.uniform(0, 1, (n, n)) * np.where(rng.uniform(size=(n, n)) < 0.5, 1.0, 1e-6))
    x = x.astype(np.float32)
    t = 3 * k * k + 4
    g = t * U32 / (1 - t * U32) + 2.0 ** -20
    with Plan(psf, n) as plan:
        plan.set_blur_config(cfg)
        y = torch.empty_like(to_dev(x))
        plan.blur(to_dev(x), y)
        x64 = x.astype(np.float64)
        ref = O.blur(psf, x64)
        bound = (g * O.blur(np.abs(psf), np.abs(x64)) + U32 * np.abs(ref)
                 + 2.0 ** -30 * np.abs(x64).max() * np.abs(psf).sum())
        err = np.abs(to_host(y) - ref)
        say(f"hdr: max err/bound {np.max(err / bound):.3f}")
        assert np.all(err <= bound)


@pytest.mark.parametrize("cfg", [0, 6, 7])
def test_solve_with_each_blur_kernel(cfg):
    """The FP16-KP FPCG solve at 256^2 reaches the same x_lambda with the VALU
    and the MFMA blur."""
    require_gpu()
    from paper_2311_15393_amd import KP_FPCG, KP_OK, KP_P16, Plan
    from oracle import solvers as SV
    prob = S.mid_anisotropic(0)
    with Plan(prob.psf, prob.n) as plan:
        plan.set_blur_config(cfg)
        x, info = plan.solve(to_dev(prob.b), prob.lam, tol=1e-7, maxit=3000,
                             mode=KP_FPCG | KP_P16)
    ref = SV.x_lambda(prob.psf, prob.b.astype(np.float64), prob.lam)
    err = rel(to_host(x), ref)
    say(f"cfg={cfg}: iters={info.iters} err={err:.2e}")
    assert info.status == KP_OK and err <= 1e-4


@pytest.mark.parametrize("n,k", [(64, 15), (100, 31), (256, 63)])
def test_normal_fp64_matches_oracle(n, k):
    """(A^T A + lambda^2 I) x with FP64 accumulation: products of FP32 data
    are exact in FP64, so the error is FP64 summation only."""
    torch = require_gpu()
    from paper_2311_15393_amd import Plan
    say(f"normal64 n={n} k={k}")
    psf = _psf("moffat", k, 3)
    x = S.random_image(np.random.default_rng(7), n)
    lam = 0.03
    with Plan(psf, n) as plan:
        y = torch.empty((n, n), dtype=torch.float64, device="cuda")
        plan.normal_fp64(to_dev(x), lam, y)
        got = to_host(y)
    x64 = x.astype(np.float64)
    ref = O.normal_op(psf, lam, x64)
    absref = O.blur_t(np.abs(psf), O.blur(np.abs(psf), np.abs(x64))) + lam * lam * np.abs(x64)
    u64 = 2.0 ** -53
    assert np.all(np.abs(got - ref) <= 4 * k * k * u64 * absref + 1e-300)


@pytest.mark.parametrize("n,k,kind", [(64, 15, "moffat"), (100, 31, "moffat"),
                                      (256, 31, "moffat"), (96, 15, "rand"), (200, 31, "rand")])
def test_factor_svd_matches_oracle(n, k, kind):
    """Singular values of the Kronecker factors (device FP64 SVD) and the
    quality measure of Table 1 match the oracle; V is compared through the
    sign-free projector V diag(s^2) V^T = A_c^T A_c."""
    require_gpu()
    from paper_2311_15393_amd import Plan
    say(f"factors n={n} k={k} {kind}")
    psf = _psf(kind, k, 5)
    kp = KP.kp_svd(psf, n)
    with Plan(psf, n) as plan:
        info = plan.query()
        sc, sr, vc, vr = plan.factors()
    assert np.allclose(sc, kp.sc, rtol=1e-10, atol=1e-13 * kp.sc[0])
    assert np.allclose(sr, kp.sr, rtol=1e-10, atol=1e-13 * kp.sr[0])
    assert abs(info["kp_rel_error"] - KP.kp_error(kp.s_psf)) <= 1e-10
    gram_c = (vc * sc ** 2) @ vc.T                      # V_c S^2 V_c^T (FP32 V)
    assert np.allclose(gram_c, kp.Ac.T @ kp.Ac, atol=1e-5 * sc[0] ** 2)
    gram_r = (vr * sr ** 2) @ vr.T
    assert np.allclose(gram_r, kp.Ar.T @ kp.Ar, atol=1e-5 * sr[0] ** 2)


def _gpu_factors(plan):
    sc, sr, vc, vr = plan.factors()
    return sc, sr, vc, vr


@pytest.mark.parametrize("n,k,lam", [(64, 15, 0.02), (100, 31, 0.01), (256, 31, 0.005)])
def test_precond_fp32_within_accumulation_bound(n, k, lam):
    """FP32 preconditioner (four MFMA FP32 GEMMs) vs the same chain with exact
    products, on the GPU's own factors: elementwise within the first-order
    FP32 accumulation bound."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_P32, Plan
    say(f"precond32 n={n} k={k}")
    psf = _psf("moffat", k, 9)
    r = S.random_image(np.random.default_rng(11), n)
    with Plan(psf, n) as plan:
        sc, sr, vc, vr = _gpu_factors(plan)
        z = torch.empty((n, n), dtype=torch.float32, device="cuda")
        plan.precond(to_dev(r), lam, KP_P32, z)
        got = to_host(z)
    ref = Q.precond_fp32(vc, vr, sc, sr, lam, r)
    bound = Q.fp32_chain_bound(vc, vr, sc, sr, lam, r)
    assert np.all(np.abs(got - ref) <= bound + 1e-30)
    # and close to the exact FP64 preconditioner of the oracle
    kp = KP.kp_svd(psf, n)
    assert rel(got, KP.precond_solve(kp, lam, r.astype(np.float64))) < 1e-4


@pytest.mark.parametrize("n,k,lam", [(64, 15, 0.02), (256, 31, 0.01), (1024, 63, 0.003)])
def test_precond_fp16_matches_emulated_chain(n, k, lam):
    """FP16 chain on MFMA vs the oracle's emulation of the same rounding
    points (FP16 storage of V, of the power-of-two-scaled residual and of
    each intermediate; exact products).
    Elementwise: |z_gpu - z_emul| <= Q.fp16_chain_bound, the worst-case bound
    for FP32 accumulation in any order plus, at each stored intermediate, the
    neighbouring FP16 value wherever the accumulated value may lie on the
    other side of a rounding boundary, propagated through |V|.
    Normwise (sharper, since the worst case is loose at large n): the GPU's
    error against exact arithmetic is of the emulation's size (0.5x-1.5x)
    and its distance to the emulation at most half that size.  A wrong
    operand, transposition or scale gives O(1) errors."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_P16, Plan
    say(f"precond16 n={n} k={k}")
    psf = _psf("moffat", k, 13)
    r = S.random_image(np.random.default_rng(17), n) * 1e-3
    r64 = r.astype(np.float64)
    # the device picks its scale from its own FP64 ||r||: keep clear of a
    # power-of-two boundary so both sides take the same one
    m = np.frexp(np.linalg.norm(r64))[0]
    assert 0.5 + 1e-9 < m < 1.0 - 1e-9
    with Plan(psf, n) as plan:
        sc, sr, vc, vr = _gpu_factors(plan)
        z = torch.empty((n, n), dtype=torch.float32, device="cuda")
        plan.precond(to_dev(r), lam, KP_P16, z)
        got = to_host(z)
    emul = Q.precond_fp16(vc, vr, sc, sr, lam, r64)
    bound = Q.fp16_chain_bound(vc, vr, sc, sr, lam, r64)
    exact = Q.precond_fp32(vc, vr, sc, sr, lam, r)
    e_emul = rel(emul, exact)
    e_gpu = rel(got, exact)
    d = rel(got, emul)
    worst = float(np.max(np.abs(got - emul) / bound))
    say(f"  |gpu-exact|={e_gpu:.3e} |emul-exact|={e_emul:.3e} |gpu-emul|={d:.3e} "
        f"max |gpu-emul|/bound={worst:.3e}")
    assert np.all(np.abs(got - emul) <= bound)
    assert 0.5 * e_emul <= e_gpu <= 1.5 * e_emul
    assert d <= 0.5 * e_emul
    assert 1e-5 < e_emul < 2e-2


@pytest.mark.parametrize("n,k,lam", [(128, 15, 0.02), (256, 31, 0.01), (1024, 63, 0.003)])
def test_precond_fp8_matches_emulated_chain(n, k, lam):
    """FP8 e4m3 chain with 32-entry block exponents on the block-scaled MFMA,
    vs the oracle's emulation with the same block structure (exponent from
    the block's largest magnitude, e4m3 round-to-nearest-even, exact
    products), quantising the same FP32 copies of V the device quantises.
    Elementwise: |z_gpu - z_emul| <= Q.fp8_chain_bound (FP32 accumulation
    in any order; at each stored intermediate the neighbouring e4m3 value,
    or a neighbouring block exponent, wherever the accumulated values allow
    it).  Normwise as for FP16."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_P8, Plan
    say(f"precond8 n={n} k={k}")
    psf = _psf("moffat", k, 21)
    r = S.random_image(np.random.default_rng(23), n) * 1e-3
    r64 = r.astype(np.float64)
    with Plan(psf, n) as plan:
        sc, sr, vc, vr = _gpu_factors(plan)
        z = torch.empty((n, n), dtype=torch.float32, device="cuda")
        plan.precond(to_dev(r), lam, KP_P8, z)
        got = to_host(z)
    vc32, vr32 = Q.round_fp32(vc), Q.round_fp32(vr)
    emul = Q.precond_fp8(vc32, vr32, sc, sr, lam, r64)
    bound = Q.fp8_chain_bound(vc32, vr32, sc, sr, lam, r64)
    exact = Q.precond_fp32(vc, vr, sc, sr, lam, r)
    e_emul = rel(emul, exact)
    e_gpu = rel(got, exact)
    d = rel(got, emul)
    worst = float(np.max(np.abs(got - emul) / bound))
    say(f"  |gpu-exact|={e_gpu:.3e} |emul-exact|={e_emul:.3e} |gpu-emul|={d:.3e} "
        f"max |gpu-emul|/bound={worst:.3e}")
    assert np.all(np.abs(got - emul) <= bound)
    assert 0.5 * e_emul <= e_gpu <= 1.5 * e_emul
    assert d <= 0.5 * e_emul
    assert 1e-3 < e_emul < 0.2


@pytest.mark.parametrize("lam", [1.0, 0.5])
def test_precond_lowp_exact_products_bit_for_bit(lam):
    """An identity PSF (K = 1) gives A = I: both Kronecker factors are the
    identity, their singular values 1 and V = I.  Every product of the
    chain then has one nonzero term and is exact in FP32, so the device
    must reproduce the rounding points of the emulation bit for bit: the
    power-of-two residual scale and its FP16 (or block-scaled e4m3)
    rounding, the stored intermediates, S' = lambda^2 / (1 + lambda^2)
    in FP32 and the final 1 / (scale lambda^2).  lambda = 1 makes S' = 1/2
    (exact); lambda = 1/2 makes S' = 0.2 (rounded to FP32 first, then the
    FP16 product is rounded from its FP32 value, as on the device)."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_P8, KP_P16, KP_P32, Plan
    n = 256
    say(f"precond exact products lambda={lam}")
    r = S.random_image(np.random.default_rng(41), n).astype(np.float64) - 0.5
    r[5, :40] *= 2.0 ** -20                              # some subnormal FP16 entries
    r = r.astype(np.float32)
    r64 = r.astype(np.float64)
    with Plan(np.array([[1.0]]), n) as plan:
        sc, sr, vc, vr = _gpu_factors(plan)
        if not (np.array_equal(np.abs(vc), np.eye(n)) and np.array_equal(np.abs(vr), np.eye(n))
                and np.all(sc == 1.0) and np.all(sr == 1.0)):
            pytest.skip("device SVD of the identity factor is not a signed identity")
        outs = {}
        for prec in (KP_P32, KP_P16, KP_P8):
            z = torch.empty((n, n), dtype=torch.float32, device="cuda")
            plan.precond(to_dev(r), lam, prec, z)
            outs[prec] = to_host(z).astype(np.float64)
    f32 = np.float32
    sp = f32(lam * lam) / (f32(1.0) + f32(lam * lam))     # S' in FP32
    # FP32: each product is one exact term; S' applied in FP32
    t = vc.T @ r64 @ vr
    t2 = Q.round_fp32(np.float64(sp) * t)
    want32 = Q.round_fp32((vc @ t2 @ vr.T) * np.float64(f32(1.0 / (lam * lam))))
    assert np.array_equal(outs[KP_P32], want32)
    if lam == 1.0:
        emul16 = Q.precond_fp16(vc, vr, sc, sr, lam, r64)
        emul8 = Q.precond_fp8(vc, vr, sc, sr, lam, r64)
        assert np.array_equal(outs[KP_P16], Q.round_fp32(emul16))
        assert np.array_equal(outs[KP_P8], Q.round_fp32(emul8))
    else:
        tr = {}
        Q.precond_fp16(vc, vr, sc, sr, lam, r64, trace=tr)
        t1 = vc.T @ tr["rt"] @ vr                         # exact: one term each
        t2 = Q.round_fp16(Q.round_fp32(np.float64(sp) * t1))
        zs = np.float64(f32(1.0 / (tr["scale"] * lam * lam)))
        want16 = Q.round_fp32((vc @ t2 @ vr.T) * zs)
        assert np.array_equal(outs[KP_P16], want16)


def test_fp8_rejects_unsupported_size():
    torch = require_gpu()
    from paper_2311_15393_amd import KP_ERR_UNSUPPORTED, KP_FPCG, KP_P8, KPError, Plan
    psf = _psf("gauss", 9)
    with Plan(psf, 96) as plan:
        z = torch.empty((96, 96), dtype=torch.float32, device="cuda")
        r = to_dev(S.random_image(np.random.default_rng(1), 96))
        with pytest.raises(KPError) as ei:
            plan.precond(r, 0.01, KP_P8, z)
        assert ei.value.status == KP_ERR_UNSUPPORTED
        with pytest.raises(KPError) as ei:
            plan.solve(r, 0.01, mode=KP_FPCG | KP_P8)
        assert ei.value.status == KP_ERR_UNSUPPORTED


def test_symmetric_and_general_factor_paths_agree(monkeypatch):
    """Point-symmetric PSFs take the symmetric eigensolver path; forcing the
    general SVD must give the same preconditioner (V and s are unique up to
    signs and rotations inside repeated singular values, M^{-1} is not)."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_P32, Plan
    n, k, lam = 128, 31, 0.01
    psf = _psf("moffat", k, 31)
    r = to_dev(S.random_image(np.random.default_rng(3), n))
    outs = []
    for general in ("0", "1"):
        monkeypatch.setenv("KPCG_GENERAL_SVD", general)
        with Plan(psf, n) as plan:
            z = torch.empty((n, n), dtype=torch.float32, device="cuda")
            plan.precond(r, lam, KP_P32, z)
            outs.append(to_host(z))
    assert rel(outs[0], outs[1]) < 1e-5


@pytest.mark.parametrize("n,k,kind", [(64, 15, "moffat"), (100, 9, "rand"), (256, 31, "moffat"),
                                      (128, 63, "moffat"), (64, 15, "gauss")])
def test_exact_diag_matches_oracle(n, k, kind):
    """kp_setup's exact KP-basis diagonal D0 = diag(V^T A^T A V) (all terms of
    eq. (KronSumDecomp), FP64 Gram sums on the device, stored FP32) against
    the oracle's, elementwise: FP32 rounding of each entry plus an absolute
    1e-9 max(D0) for the entries far below the largest (FP64 cancellation
    in the sum over term pairs, and the device's own FP64 V)."""
    require_gpu()
    from paper_2311_15393_amd import Plan
    say(f"exact diagonal n={n} k={k} {kind}")
    psf = _psf(kind, k, 21)
    kp = KP.kp_svd(psf, n)
    ref = KP.exact_diag(kp, psf)
    with Plan(psf, n) as plan:
        got = plan.exact_diag().astype(np.float64)
    err = np.abs(got - ref)
    say(f"  max rel (entries > 1e-3 max) "
        f"{(err / ref)[ref > 1e-3 * ref.max()].max():.2e}, max abs / max {err.max() / ref.max():.2e}")
    assert np.all(err <= 2.0 ** -23 * np.abs(ref) + 1e-9 * ref.max())


@pytest.mark.parametrize("n,k,lam", [(64, 15, 0.02), (256, 31, 0.01)])
def test_precond_exact_diag_matches_oracle(n, k, lam):
    """z = V (S .* V^T r V) V^T with S = 1 / (D0 + lambda^2) on the device's
    FP32 and FP16 chains vs the oracle's FP64 application with its own D0."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_EXACT_DIAG, KP_P16, KP_P32, Plan
    say(f"precond exact diagonal n={n} k={k}")
    psf = _psf("moffat", k, 23)
    r = S.random_image(np.random.default_rng(29), n)
    kp = KP.kp_svd(psf, n)
    ref = KP.precond_solve(kp, lam, r.astype(np.float64), KP.exact_diag(kp, psf))
    one = KP.precond_solve(kp, lam, r.astype(np.float64))
    with Plan(psf, n) as plan:
        z = torch.empty((n, n), dtype=torch.float32, device="cuda")
        plan.precond(to_dev(r), lam, KP_P32 | KP_EXACT_DIAG, z)
        e32 = rel(to_host(z), ref)
        plan.precond(to_dev(r), lam, KP_P16 | KP_EXACT_DIAG, z)
        e16 = rel(to_host(z), ref)
        plan.precond(to_dev(r), lam, KP_P32, z)
        e_one = rel(to_host(z), one)
    say(f"  fp32 {e32:.2e} fp16 {e16:.2e} (one-term fp32 {e_one:.2e}; "
        f"the two S differ by {rel(one, ref):.2e})")
    assert e32 < 1e-4 and e16 < 2e-2 and e_one < 1e-4
    assert rel(one, ref) > 10 * e32        # the test can tell the two tables apart
