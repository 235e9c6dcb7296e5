"""Reduced-precision construction of S, V_r, V_c (KP_SETUP_LOWP): each
Kronecker factor scaled by a power of two, rounded to FP16 and factorised by
FP32 rocSOLVER, against the oracle's exact SVD of the same FP16-rounded
factors (kp.kp_svd_fp16_factors)."""
import numpy as np
import pytest

import synthetic as S
from oracle import kp as KP
from oracle import periodic as PB
from oracle import reflexive as RB
from tests.gpu_util import rel, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _psf(kind, k, seed=0):
    rng = np.random.default_rng(seed)
    if kind == "gauss":
        return S.psf_gaussian(k, 2.0 + k / 20, 1.5, 0.0)      # separable, symmetric factors
    if kind == "moffat":
        return S.psf_moffat_motion(k, rng.uniform(3, 8), 2.5, rng.uniform(3, 9),
                                   rng.uniform(0, np.pi))
    p = rng.uniform(0, 1, (k, k))
    return (p / p.sum()).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("n,k,kind,bc", [(64, 15, "moffat", 0), (100, 31, "rand", 0),
                                         (256, 31, "moffat", 0), (128, 63, "gauss", 0),
                                         (96, 15, "moffat", 1), (112, 31, "gauss", 2)])
def test_lowp_factors_match_fp16_oracle(n, k, kind, bc):
    """FP32 SVD (general path) or FP32 symmetric eigensolver (symmetric
    profiles) of the FP16 factor: a backward-stable factorisation in FP32
    moves singular values by at most c n u ||A||_2 and the Gram matrix
    V diag(s^2) V^T = A^T A by c n u ||A||_2^2 (c = 4 here); compared with the
    exact SVD of the same FP16 factor.  The FP64 construction's singular
    values differ by the FP16 rounding itself, which the test also sees, so
    the reduced path is the one that ran."""
    require_gpu()
    from paper_2311_15393_amd import KP_SETUP_LOWP, Plan
    say(f"lowp factors n={n} k={k} {kind} bc={bc}")
    psf = _psf(kind, k, 7)
    kp = (PB.kp_svd(psf, n) if bc == 1 else RB.kp_svd(psf, n) if bc == 2
          else KP.kp_svd(psf, n))
    ref = KP.kp_svd_fp16_factors(kp)
    with Plan(psf, n, bc=bc | KP_SETUP_LOWP) as plan:
        sc, sr, vc, vr = plan.factors()
    with Plan(psf, n, bc=bc) as full:
        sc64, _, _, _ = full.factors()
    for s_gpu, s_ref, v_gpu, a16 in ((sc, ref.sc, vc, ref.Ac), (sr, ref.sr, vr, ref.Ar)):
        smax = s_ref[0]
        tol = 4 * n * U32 * smax
        assert np.all(np.abs(s_gpu - s_ref) <= tol), np.abs(s_gpu - s_ref).max() / tol
        gram = (v_gpu.astype(np.float64) * s_gpu ** 2) @ v_gpu.T.astype(np.float64)
        assert np.abs(gram - a16.T @ a16).max() <= 4 * n * U32 * smax ** 2
    d_lowp, d_round = np.abs(sc - sc64).max(), np.abs(ref.sc - kp.sc).max()
    say(f"  |s_lowp - s_fp64| {d_lowp:.2e}, FP16 rounding moves s by {d_round:.2e}")
    assert d_lowp > 0.0


@pytest.mark.parametrize("bc", [0, 1])
def test_lowp_solve_reaches_x_lambda(bc):
    """FP16-KP FPCG with the reduced-precision factors still reaches the
    exact x_lambda (the factors only change the preconditioner): 256^2,
    K = 31 Moffat + motion, to 1e-4."""
    require_gpu()
    from paper_2311_15393_amd import KP_FPCG, KP_OK, KP_P16, KP_SETUP_LOWP, Plan
    from oracle import solvers as SV
    n, k, lam = 256, 31, 0.01
    psf = _psf("moffat", k, 3)
    rng = np.random.default_rng(5)
    x = S.true_image(rng, n)
    if bc:
        ax = PB.blur_fft(psf, x)
    else:
        ax = S.problems._blur_for_data(psf, x)
    e = rng.standard_normal((n, n))
    b = (ax + 0.01 * np.linalg.norm(ax) / np.linalg.norm(e) * e).astype(np.float32)
    ref = (PB.x_lambda(psf, b.astype(np.float64), lam) if bc
           else SV.x_lambda(psf, b.astype(np.float64), lam))
    with Plan(psf, n, bc=bc | KP_SETUP_LOWP) as plan:
        xg, info = plan.solve(to_dev(b), lam, tol=1e-7, maxit=500, mode=KP_FPCG | KP_P16)
        got = to_host(xg)
    with Plan(psf, n, bc=bc) as full:
        _, info64 = full.solve(to_dev(b), lam, tol=1e-7, maxit=500, mode=KP_FPCG | KP_P16)
    err = rel(got, ref)
    say(f"lowp solve bc={bc}: iters {info.iters} (FP64 factors {info64.iters}) err {err:.2e}")
    assert info.status == KP_OK and err <= 1e-4
