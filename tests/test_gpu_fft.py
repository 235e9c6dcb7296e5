"""The FFT form of the normal operator (KP_NORMAL_FFT) against the FP64
oracle operator, and solves that use it.

FP32 FFT error analysis (Higham, Accuracy and Stability of Numerical
Algorithms, ch. 24): a radix-based FFT of length L computed in precision u
has normwise relative error at most about log2(L) (u + gamma_4 (sqrt 2 + mu))
with mu the twiddle error (here one FP32 rounding of FP64 values), about
1e-6 for L ~ 2100.  H p applies four transforms of that length and two
pointwise products: the bar is 1e-5 normwise (relative to ||H p||), which a
wrong twiddle, radix butterfly, packing or crop misses by orders of
magnitude."""
import numpy as np
import pytest

import synthetic as S
from oracle import operator as O
from oracle import solvers as SV
from tests.gpu_util import rel, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [(37, 9), (64, 15), (100, 31), (129, 23), (256, 63), (1024, 15), (1024, 63),
         (2048, 63)]


def _psf(k, seed):
    rng = np.random.default_rng(seed)
    return S.psf_moffat_motion(k, rng.uniform(3, 8), 2.5, rng.uniform(3, 9),
                               rng.uniform(0, np.pi))


@pytest.mark.parametrize("n,k", CASES)
def test_fft_normal_matches_oracle(n, k):
    torch = require_gpu()
    from paper_2311_15393_amd import KP_NORMAL_DIRECT, KP_NORMAL_FFT, Plan
    psf = _psf(k, n + k)
    x = S.random_image(np.random.default_rng(n), n) - 0.5
    lam = 0.01
    with Plan(psf, n) as plan:
        info = plan.query()
        y = torch.empty((n, n), dtype=torch.float32, device="cuda")
        plan.normal(to_dev(x), lam, y, op=KP_NORMAL_FFT)
        got_fft = to_host(y)
        plan.normal(to_dev(x), lam, y, op=KP_NORMAL_DIRECT)
        got_dir = to_host(y)
    x64 = x.astype(np.float64)
    fft = O.FFTBlur(psf, n) if n > 256 else None
    ref = O.normal_op(psf, lam, x64, fft)
    e_fft, e_dir = rel(got_fft, ref), rel(got_dir, ref)
    say(f"n={n} K={k} L={info['fft_length']}: |fft - ref| {e_fft:.2e}, |direct - ref| "
        f"{e_dir:.2e}; autotuned form {info['normal_op']} (direct {info['normal_op_ms'][0]:.4f} "
        f"ms, fft {info['normal_op_ms'][1]:.4f} ms)")
    assert e_fft <= 1e-5
    assert e_dir <= 1e-5


@pytest.mark.parametrize("n,k,mode_name", [(256, 31, "fpcg16"), (1024, 63, "fpcg16"),
                                           (1536, 31, "fpcg16"), (200, 15, "pcg32"),
                                           (129, 23, "fpcg16"), (64, 15, "cg")])
def test_solve_with_fft_normal(n, k, mode_name):
    """Solves whose iterations use the FFT form reach x_lambda (1e-4 for the
    FP16 preconditioner and CG, 1e-5 for FP32), certified by true
    residuals on the blurs; n = 129 leaves the last line of every row pass
    (the one that also takes the direction step) with a single real row,
    and n = 1536 (L = 1600) runs the passes with one line per workgroup, 192
    threads summing the 576 partials of r.z and z.Hp of the GEMM tiles.  The
    preconditioned solves take the same steps as with the direct form (whose
    direction update is a launch of its own): recurrence residuals within
    2e-2 over the first five iterations (the two forms' rounding, through the
    FP16 preconditioner, moves them by up to 4e-3 at the fourth), iteration
    counts within one.  A direction step that dropped partials of r.z had a
    step length and beta wrong from the first iteration on: a first residual
    70 times the direct form's and 21 iterations against 9 at n = 1536, while
    FPCG still converged.
    CG runs to a tighter tolerance: without a preconditioner the error is up
    to cond(H) times the relative residual (about 2.5e3 here)."""
    torch = require_gpu()
    from paper_2311_15393_amd import (KP_CG, KP_FPCG, KP_NORMAL_DIRECT, KP_NORMAL_FFT, KP_OK,
                                      KP_P16, KP_P32, KP_PCG)
    from paper_2311_15393_amd import Plan
    mode = {"fpcg16": KP_FPCG | KP_P16, "pcg32": KP_PCG | KP_P32, "cg": KP_CG}[mode_name]
    bar = 1e-5 if mode_name == "pcg32" else 1e-4
    # the error is up to cond(H) ~ 2.5e3 times the relative residual: 1e-7
    # keeps the FP16 solves' error under the 1e-4 bar (at 1e-6 the 1536^2
    # solve stops at 1.4e-4)
    tol = {"pcg32": 1e-8, "cg": 1e-9}.get(mode_name, 1e-7)
    psf = _psf(k, 7 * n + k)
    prob = S.make_problem(n, psf, np.random.default_rng(n + 1), 0.01, None, n + 1, "fft")
    lam = 0.02
    with Plan(psf, n) as plan:
        plan.set_normal_op(KP_NORMAL_FFT)
        x, info = plan.solve(to_dev(prob.b), lam, tol=tol, maxit=3000, mode=mode, history=True)
        got = to_host(x)
        if mode_name != "cg":
            plan.set_normal_op(KP_NORMAL_DIRECT)
            _, info_d = plan.solve(to_dev(prob.b), lam, tol=tol, maxit=3000, mode=mode,
                                   history=True)
            m = min(5, info.iters, info_d.iters)
            h_f, h_d = info.history_rec[1:m + 1], info_d.history_rec[1:m + 1]
            say(f"  FFT form {info.iters} iterations, direct {info_d.iters}; first residuals "
                f"{np.array2string(h_f, precision=4)} vs {np.array2string(h_d, precision=4)}")
            assert abs(info.iters - info_d.iters) <= 1
            np.testing.assert_allclose(h_f, h_d, rtol=2e-2)
    if n >= 1024:
        ref = SV.x_lambda_iterative(psf, prob.b.astype(np.float64), lam, check=True)[0]
    else:
        ref = SV.x_lambda(psf, prob.b.astype(np.float64), lam)
    err = rel(got, ref)
    say(f"{mode_name} n={n} K={k} via FFT: iters={info.iters} status={info.status} err={err:.2e}")
    assert info.status == KP_OK and err <= bar


def test_fft_form_refused_off_the_zero_boundary():
    torch = require_gpu()
    from paper_2311_15393_amd import (KP_BC_PERIODIC, KP_ERR_UNSUPPORTED, KP_NORMAL_FFT, KPError,
                                      Plan)
    n, k = 64, 9
    with Plan(_psf(k, 1), n, bc=KP_BC_PERIODIC) as plan:
        assert plan.query()["normal_op"] == 0
        with pytest.raises(KPError) as ei:
            plan.set_normal_op(KP_NORMAL_FFT)
        assert ei.value.status == KP_ERR_UNSUPPORTED


# every transform length the library's FFT menu holds (each is its own set of
# kernels), with its three Stockham radices; the two largest are reached by
# n = 2048 with K = 63 (zero boundary 2100, reflexive 2160)
MENU = [64, 96, 128, 144, 192, 256, 320, 384, 480, 540, 560, 576, 672, 768, 896, 960, 1024,
        1050, 1080, 1152, 1296, 1440, 1600, 1728, 1920, 2016, 2100, 2160]


@pytest.mark.parametrize("L", MENU)
def test_fft_normal_every_menu_length(L):
    """H p by the FFT passes at n = L - h (so that L is the plan's length)
    for every length of the menu against the oracle's operator (normwise
    1e-5): n odd (K = 15; the last row pair has one row) below 2048, and the
    two largest lengths at n = 2048, K = 63 (zero and reflexive boundary)."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_BC_REFLEXIVE, KP_NORMAL_FFT, Plan
    from oracle import reflexive as RB
    if L == 2100:
        n, k, bc = 2048, 63, 0
    elif L == 2160:
        n, k, bc = 2048, 63, KP_BC_REFLEXIVE
    else:
        n, k, bc = L - 7, 15, 0
    psf = _psf(k, L)
    x = S.random_image(np.random.default_rng(L), n) - 0.5
    lam = 0.02
    with Plan(psf, n, bc=bc) as plan:
        assert plan.query()["fft_length"] == L
        y = torch.empty((n, n), dtype=torch.float32, device="cuda")
        plan.normal(to_dev(x), lam, y, op=KP_NORMAL_FFT)
        got = to_host(y)
    x64 = x.astype(np.float64)
    if bc == KP_BC_REFLEXIVE:
        ref = RB.NormalOperatorGeneral(psf, n, lam).H(x64)
    else:
        ref = O.normal_op(psf, lam, x64, O.FFTBlur(psf, n) if n > 256 else None)
    e = rel(got, ref)
    say(f"menu L={L} n={n} K={k} bc={bc}: |fft - ref| {e:.2e}")
    assert e <= 1e-5


# (solver, preconditioner, tol, bar): at lambda = 0.02 cond(H) is about
# 2.5e3, so the tolerances sit 1-2 decades below the bars
FFT_MODES = {"pcg16": ("KP_PCG", "KP_P16", 1e-7, 1e-4), "fpcg16": ("KP_FPCG", "KP_P16", 1e-7, 1e-4),
             "pcg32": ("KP_PCG", "KP_P32", 1e-8, 1e-5), "fpcg32": ("KP_FPCG", "KP_P32", 1e-8, 1e-5),
             "fpcg8": ("KP_FPCG", "KP_P8", 1e-7, 1e-4), "fpcg16_diag": ("KP_FPCG", "KP_P16", 1e-7, 1e-4)}


@pytest.mark.parametrize("mode_name", list(FFT_MODES))
def test_fft_solves_every_preconditioned_mode(mode_name):
    """PCG and FPCG with H p by the FFT passes on a zero-boundary plan, where
    the direction step p = z + beta p of each iteration runs in the first
    pass of the next H p: every preconditioner precision (and the exact
    diagonal) reaches x_lambda at 256^2, K = 21 with one history entry per
    iteration; a solve cut at maxit = 3 stops at KP_MAXIT after exactly three
    iterations, reporting the oracle's ||c - H x|| / ||c|| of its x; a warm
    start from the solution converges again within a few iterations."""
    torch = require_gpu()
    import paper_2311_15393_amd as K
    solver, prec, tol, bar = FFT_MODES[mode_name]
    mode = getattr(K, solver) | getattr(K, prec)
    if mode_name.endswith("_diag"):
        mode |= K.KP_EXACT_DIAG
    n, k, lam = 256, 21, 0.02            # n: a multiple of the FP8 GEMM tiles
    psf = _psf(k, 11)
    prob = S.make_problem(n, psf, np.random.default_rng(5), 0.01, None, 6, "fft")
    b64 = prob.b.astype(np.float64)
    ref = SV.x_lambda(psf, b64, lam)
    c = O.blur_t(psf, b64)
    with K.Plan(psf, n) as plan:
        plan.set_normal_op(K.KP_NORMAL_FFT)
        b = to_dev(prob.b)
        x, info = plan.solve(b, lam, tol=tol, maxit=3000, mode=mode, history=True)
        err = rel(to_host(x), ref)
        say(f"{mode_name} via FFT: iters={info.iters} repl={info.replacements} err={err:.2e}")
        assert info.status == K.KP_OK and err <= bar
        assert info.history_rec.size == info.iters + 1 and np.all(np.isfinite(info.history_rec))
        x3, info3 = plan.solve(b, lam, tol=tol, maxit=3, mode=mode | K.KP_NO_FALLBACK,
                               raise_on_fail=False)
        x3_64 = to_host(x3).astype(np.float64)
        r_or = np.linalg.norm(c - O.normal_op(psf, lam, x3_64)) / np.linalg.norm(c)
        say(f"  maxit 3: status={info3.status} relres {info3.relres_true:.4e} oracle {r_or:.4e}")
        assert info3.status == K.KP_MAXIT and info3.iters == 3
        assert abs(info3.relres_true - r_or) <= 1e-2 * r_or
        xw = x.clone()
        xw, infow = plan.solve(b, lam, tol=tol, maxit=3000, mode=mode | K.KP_WARM, x=xw)
        say(f"  warm start: iters={infow.iters}")
        assert infow.status == K.KP_OK and infow.iters <= 3 and rel(to_host(xw), ref) <= bar


@pytest.mark.parametrize("n,k", [(1024, 63), (1536, 31)])
def test_fft_solves_are_bitwise_reproducible(n, k):
    """Two FP16-KP FPCG solves of one problem through the FFT form, each
    from x = 0, give the same x bit for bit and the same iteration count:
    every reduction (the folds in the direction step, the first GEMM and the
    update, each in the scalar step's order) is deterministic, and no kernel
    reads LDS or partials another workgroup may still be writing.  n = 1536
    runs the direction step's fold in blocks of 192 threads."""
    torch = require_gpu()
    import paper_2311_15393_amd as K
    psf = _psf(k, 3 * n + k)
    prob = S.make_problem(n, psf, np.random.default_rng(n + 7), 0.01, None, n + 7, "fft")
    with K.Plan(psf, n) as plan:
        plan.set_normal_op(K.KP_NORMAL_FFT)
        b = to_dev(prob.b)
        outs = []
        for _ in range(2):
            x = torch.zeros_like(b)
            x, info = plan.solve(b, 0.02, tol=1e-6, maxit=500, mode=K.KP_FPCG | K.KP_P16, x=x)
            outs.append((to_host(x), info.iters, info.status))
    say(f"n={n} K={k}: iterations {outs[0][1]}, {outs[1][1]}")
    assert outs[0][2] == K.KP_OK and outs[1][2] == K.KP_OK
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0].view(np.uint32), outs[1][0].view(np.uint32))
