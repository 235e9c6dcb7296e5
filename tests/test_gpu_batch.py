"""Batched solves (pcg_solve_batched) against the FP64 oracle: uneven image
sizes and PSF supports, several lambda per problem, one set of launches."""
import numpy as np
import pytest

import synthetic as S
from oracle import operator as O
from oracle import solvers as SV
from tests.gpu_util import rel, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu

_CACHE = {}


def _small_batch():
    """Five problems, uneven sizes (one ragged), two lambda each."""
    if "probs" not in _CACHE:
        specs = [(64, 15, "g"), (100, 9, "m"), (128, 31, "m"), (192, 21, "g"), (256, 31, "m")]
        probs = []
        for idx, (n, k, kind) in enumerate(specs):
            rng = np.random.default_rng(500 + idx)
            psf = (S.psf_gaussian(k, 1.5 + idx * 0.5, 2.5, 0.3 * idx) if kind == "g"
                   else S.psf_moffat_motion(k, 3.0 + idx, 2.5, 3.0 + idx, 0.5 * idx))
            probs.append(S.make_problem(n, psf, rng, 0.01 + 0.005 * idx, None, 500 + idx,
                                        f"batch{idx}"))
        lams = [0.01, 0.05]
        items = [(p, lam) for p in range(len(probs)) for lam in lams]
        _CACHE["probs"] = probs
        _CACHE["items"] = items
    return _CACHE["probs"], _CACHE["items"]


def _xlam(probs, p, lam):
    key = (p, lam)
    if key not in _CACHE:
        prob = probs[p]
        _CACHE[key] = SV.x_lambda(prob.psf, prob.b.astype(np.float64), lam)
    return _CACHE[key]


def _run(plans, probs, items, mode, tol, maxit=500):
    from paper_2311_15393_amd import solve_batched
    bs = [to_dev(probs[p].b) for p, _ in items]
    lams = [lam for _, lam in items]
    poi = [p for p, _ in items]
    xs, infos, st = solve_batched(plans, bs, lams, poi, tol=tol, maxit=maxit, mode=mode)
    return [to_host(x) for x in xs], infos, st


@pytest.mark.parametrize("mode_name,bar,tol", [("fpcg16", 1e-4, 1e-8), ("pcg32", 1e-5, 1e-9),
                                               ("cg", 1e-4, 1e-8)])
def test_batched_items_match_oracle(mode_name, bar, tol):
    require_gpu()
    from paper_2311_15393_amd import KP_CG, KP_FPCG, KP_OK, KP_P16, KP_P32, KP_PCG, Plan
    mode = {"fpcg16": KP_FPCG | KP_P16, "pcg32": KP_PCG | KP_P32, "cg": KP_CG}[mode_name]
    probs, items = _small_batch()
    plans = [Plan(p.psf, p.n) for p in probs]
    say(f"batched {mode_name}: {len(items)} items")
    xs, infos, st = _run(plans, probs, items, mode, tol, maxit=2000)
    for (p, lam), x, inf in zip(items, xs, infos):
        err = rel(x, _xlam(probs, p, lam))
        say(f"  n={probs[p].n} k={probs[p].k} lam={lam} iters={inf.iters} "
            f"status={inf.status} err={err:.2e}")
        assert inf.status == KP_OK and inf.relres_true <= tol
        assert err <= bar
    assert st == KP_OK
    for pl in plans:
        pl.close()


def test_graph_replay_matches_eager_launches():
    """The captured iteration block, replayed with host synchronisation and
    true-residual work between replays, gives bit-identical results to
    launching every kernel eagerly (all reductions are deterministic)."""
    require_gpu()
    from paper_2311_15393_amd import KP_BATCH_EAGER, KP_FPCG, KP_P16, Plan
    probs, items = _small_batch()
    plans = [Plan(p.psf, p.n) for p in probs]
    mode = KP_FPCG | KP_P16
    xg, ig, _ = _run(plans, probs, items, mode, 1e-8)
    xe, ie, _ = _run(plans, probs, items, mode | KP_BATCH_EAGER, 1e-8)
    for a, b, i1, i2 in zip(xg, xe, ig, ie):
        assert i1.iters == i2.iters and i1.replacements == i2.replacements
        assert np.array_equal(a, b)
    assert max(i.iters for i in ig) > 8          # more than one replay happened
    for pl in plans:
        pl.close()


def test_batched_misfit_report():
    """infos[i].misfit = ||A x_i - b_i|| (FP64-accumulated blur of the result)."""
    require_gpu()
    from paper_2311_15393_amd import KP_FPCG, KP_P16, Plan
    probs, items = _small_batch()
    plans = [Plan(p.psf, p.n) for p in probs]
    xs, infos, _ = _run(plans, probs, items, KP_FPCG | KP_P16, 1e-7)
    for (p, lam), x, inf in zip(items, xs, infos):
        prob = probs[p]
        ref = float(np.linalg.norm(O.blur(prob.psf, x.astype(np.float32).astype(np.float64))
                                   - prob.b.astype(np.float64)))
        assert abs(inf.misfit - ref) <= 1e-6 * ref
    for pl in plans:
        pl.close()


def test_batched_rejects_bad_arguments():
    require_gpu()
    import torch
    from paper_2311_15393_amd import (KP_ERR_ARG, KP_ERR_UNSUPPORTED, KP_FPCG, KP_P8, KP_P16,
                                      KPError, Plan, solve_batched)
    probs, items = _small_batch()
    plan = Plan(probs[0].psf, probs[0].n)
    b = to_dev(probs[0].b)
    with pytest.raises(KPError) as ei:
        solve_batched([plan], [b], [-1.0], [0], mode=KP_FPCG | KP_P16)
    assert ei.value.status == KP_ERR_ARG
    # the FP8 chain needs n to be a multiple of 128 (this item: 64)
    with pytest.raises(KPError) as ei:
        solve_batched([plan], [b], [0.01], [0], mode=KP_FPCG | KP_P8)
    assert ei.value.status == KP_ERR_UNSUPPORTED
    plan.close()


def test_batched_fp8_items_match_oracle():
    """FP8-KP FPCG in the batch (items of 128^2 and 256^2, two lambda each):
    every item meets the FP16 bar against x_lambda, and takes about as many
    iterations as the same solve by pcg_solve with the plan's FP8 chain (a
    wrong stage, exponent block or tile mapping in the batched chain would
    change the preconditioner and with it the iteration count)."""
    require_gpu()
    from paper_2311_15393_amd import KP_FPCG, KP_NO_FALLBACK, KP_OK, KP_P8, Plan
    probs, items = _small_batch()
    items = [(p, lam) for p, lam in items if probs[p].n % 128 == 0]
    assert len(items) == 4
    plans = [Plan(p.psf, p.n) for p in probs]
    tol = 1e-8
    xs, infos, st = _run(plans, probs, items, KP_FPCG | KP_P8, tol, maxit=2000)
    assert st == KP_OK
    for (p, lam), x, inf in zip(items, xs, infos):
        _, one = plans[p].solve(to_dev(probs[p].b), lam, tol=tol, maxit=2000,
                                mode=KP_FPCG | KP_P8 | KP_NO_FALLBACK)
        err = rel(x, _xlam(probs, p, lam))
        say(f"  fp8 n={probs[p].n} lam={lam}: batch iters={inf.iters} single iters={one.iters} "
            f"err={err:.2e}")
        assert inf.status == KP_OK and inf.relres_true <= tol and err <= 1e-4
        assert abs(inf.iters - one.iters) <= max(3, 0.3 * one.iters)
    for pl in plans:
        pl.close()


def test_uneven_batch_sample_full_sizes():
    """Five problems of the uneven-size workload (sizes 128, 384, 1024, 256
    and 768, supports 15..63, Gaussian or Moffat), three lambda around each
    problem's KP-GCV choice: every item converges, and the middle item of
    every problem (the 768^2 and 1024^2 ones included) meets the FP16 bar
    against the oracle's settled x_lambda."""
    require_gpu()
    from paper_2311_15393_amd import KP_FPCG, KP_OK, KP_P16, Plan
    probs = [S.batch_problem(i) for i in (0, 1, 2, 3, 9)]
    plans = [Plan(p.psf, p.n) for p in probs]
    grid = S.lambda_grid()
    items = []
    for pi, (prob, plan) in enumerate(zip(probs, plans)):
        lam_g, _ = plan.gcv(to_dev(prob.b), grid)
        for f in (0.3, 1.0, 3.0):
            items.append((pi, float(np.clip(lam_g * f, 1e-4, 1.0))))
    say(f"uneven sample: sizes {[p.n for p in probs]} supports {[p.k for p in probs]}")
    xs, infos, st = _run(plans, probs, items, KP_FPCG | KP_P16, 1e-7, maxit=1000)
    checked = 0
    for (p, lam), x, inf in zip(items, xs, infos):
        assert inf.status == KP_OK, (p, lam, inf)
        if lam == items[3 * p + 1][1]:
            ref, rinfo = SV.x_lambda_iterative(probs[p].psf, probs[p].b.astype(np.float64), lam,
                                               check=True)
            assert rinfo["status"] == "converged" and rinfo["true_relres"] <= 1e-12, rinfo
            err = rel(x, ref)
            say(f"  n={probs[p].n} k={probs[p].k} lam={lam:.3g} iters={inf.iters} err={err:.2e}")
            assert err <= 1e-4
            checked += 1
    assert checked == len(probs)
    for pl in plans:
        pl.close()


def test_batch_mixes_valu_and_mfma_items():
    """Items whose plans use the VALU blur and items on the MFMA blur (all
    three chunk counts) in one batch: each item still reaches the oracle's
    x_lambda."""
    require_gpu()
    from paper_2311_15393_amd import KP_BLUR_MFMA, KP_FPCG, KP_OK, KP_P16, Plan
    probs, _ = _small_batch()
    plans = [Plan(p.psf, p.n) for p in probs]
    # K = 15, 9, 31, 21, 31: chunk counts 1, 1, 2, 2, 2; alternate the kernels
    # (a plan on the 32x32x16 blur runs the 16x16x32 one in batched solves)
    for i, pl in enumerate(plans):
        pl.set_blur_config((KP_BLUR_MFMA if i % 4 == 0 else 7) if i % 2 == 0 else 0)
    big = S.batch_problem(7)                       # n = 128, K = 55: three chunks
    extra = Plan(big.psf, big.n)
    extra.set_blur_config(KP_BLUR_MFMA)
    allp = probs + [big]
    allplans = plans + [extra]
    items = [(i, lam) for i in range(len(allp)) for lam in (0.02,)]
    xs, infos, st = _run(allplans, allp, items, KP_FPCG | KP_P16, 1e-7, maxit=1000)
    for (p, lam), x, inf in zip(items, xs, infos):
        assert inf.status == KP_OK, (allp[p].n, allp[p].k, inf)
        if allp[p].n <= 256:
            err = rel(x, _xlam(allp, p, lam))
            say(f"  n={allp[p].n} k={allp[p].k} mfma={p % 2 == 0 or p == len(allp) - 1} "
                f"iters={inf.iters} err={err:.2e}")
            assert err <= 1e-4
    for pl in allplans:
        pl.close()


@pytest.mark.parametrize("tol", [1e-6, 5e-8])
def test_batched_true_residual_matches_oracle(tol):
    """relres_true of every batched item (A^T of the FP64 data residual on
    each item's fast blur for tol >= 1e-7, in FP64 below) equals the oracle's
    FP64 ||c - H x|| / ||c|| at the returned x, to within a tenth of tol plus
    the effect of returning x in FP32: the device certifies its FP64
    iterate, and rounding it to FP32 (|dx_i| <= 2^-24 |x_i|) moves the
    residual by at most ||H||_2 2^-24 ||x|| / ||c||, with ||H||_2 <=
    (sum |P|)^2 + lambda^2 (zero-boundary convolution).  Plans alternate
    between the MFMA and the VALU blur."""
    require_gpu()
    from paper_2311_15393_amd import KP_BLUR_MFMA, KP_FPCG, KP_OK, KP_P16, Plan
    probs, items = _small_batch()
    plans = [Plan(p.psf, p.n) for p in probs]
    for i, pl in enumerate(plans):
        pl.set_blur_config(KP_BLUR_MFMA if i % 2 == 0 else 0)
    try:
        say(f"batched certificate tol={tol:.0e}: {len(items)} items")
        xs, infos, st = _run(plans, probs, items, KP_FPCG | KP_P16, tol, 400)
        assert st == KP_OK
        for (pi, lam), x, info in zip(items, xs, infos):
            pr = probs[pi]
            c = O.blur_t(pr.psf, pr.b.astype(np.float64))
            r = c - O.normal_op(pr.psf, lam, x.astype(np.float64))
            ref = float(np.linalg.norm(r) / np.linalg.norm(c))
            say(f"  n={pr.n} k={pr.k} lam={lam:.3g} iters={info.iters} "
                f"relres_true={info.relres_true:.4e} oracle={ref:.4e}")
            x64 = x.astype(np.float64)
            rounding = ((np.abs(pr.psf).sum() ** 2 + lam * lam) * 2.0 ** -24
                        * np.linalg.norm(x64) / np.linalg.norm(c))
            assert info.status == KP_OK and info.relres_true <= tol
            assert abs(info.relres_true - ref) <= 0.1 * tol + rounding
    finally:
        for p in plans:
            p.close()


def test_batched_exact_diag_items_match_oracle():
    """pcg_solve_batched with KP_EXACT_DIAG: every item reaches the oracle's
    x_lambda, with no more iterations than with the one-term diagonal."""
    require_gpu()
    from paper_2311_15393_amd import KP_EXACT_DIAG, KP_FPCG, KP_OK, KP_P16, Plan
    probs, items = _small_batch()
    plans = [Plan(p.psf, p.n) for p in probs]
    try:
        say(f"batched exact diagonal: {len(items)} items")
        xs, infos, st = _run(plans, probs, items, KP_FPCG | KP_P16 | KP_EXACT_DIAG, 1e-8, 400)
        _, infos1, _ = _run(plans, probs, items, KP_FPCG | KP_P16, 1e-8, 400)
        assert st == KP_OK
        for (pi, lam), x, info, info1 in zip(items, xs, infos, infos1):
            err = rel(x, _xlam(probs, pi, lam))
            say(f"  n={probs[pi].n} k={probs[pi].k} lam={lam} iters={info.iters} "
                f"(one-term {info1.iters}) err={err:.2e}")
            assert info.status == KP_OK and err <= 1e-4
            assert info.iters <= info1.iters + 1
    finally:
        for p in plans:
            p.close()


def test_batched_warm_start_continuation():
    """KP_WARM in pcg_solve_batched: each item of a lambda = 0.01 batch starts
    from the item's own solution at lambda = 0.05 (continuation along a
    sweep).  Every item reaches the oracle's x_lambda at 0.01 in no more
    iterations than from x_0 = 0; an item started from its own converged
    solution is certified by its first true residual (no iteration)."""
    require_gpu()
    import torch
    from paper_2311_15393_amd import KP_FPCG, KP_OK, KP_P16, KP_WARM, Plan, solve_batched
    probs, _ = _small_batch()
    plans = [Plan(p.psf, p.n) for p in probs]
    try:
        bs = [to_dev(p.b) for p in probs]
        poi = list(range(len(probs)))
        mode = KP_FPCG | KP_P16
        say("batched warm start: cold solves at 0.05, then 0.01 from them")
        x05, inf05, st = solve_batched(plans, bs, [0.05] * len(probs), poi, tol=1e-8, maxit=500,
                                       mode=mode)
        assert st == KP_OK
        _, cold, _ = solve_batched(plans, bs, [0.01] * len(probs), poi, tol=1e-8, maxit=500,
                                   mode=mode)
        xw = [x.clone() for x in x05]
        xw, warm, st = solve_batched(plans, bs, [0.01] * len(probs), poi, tol=1e-8, maxit=500,
                                     mode=mode | KP_WARM, xs=xw)
        assert st == KP_OK
        for i, (x, c, w) in enumerate(zip(xw, cold, warm)):
            err = rel(to_host(x), _xlam(probs, i, 0.01))
            say(f"  n={probs[i].n} k={probs[i].k}: cold {c.iters} warm {w.iters} err={err:.2e}")
            assert w.status == KP_OK and err <= 1e-4
            assert w.iters <= c.iters
        # restart from the converged solutions themselves: nothing left to do
        # (at a tolerance above the effect of their rounding to FP32)
        xr = [x.clone() for x in xw]
        xr, again, st = solve_batched(plans, bs, [0.01] * len(probs), poi, tol=1e-6, maxit=500,
                                      mode=mode | KP_WARM, xs=xr)
        for x0, x1, a in zip(xw, xr, again):
            assert a.status == KP_OK and a.iters == 0, a
            assert torch.equal(x0, x1)
    finally:
        for p in plans:
            p.close()
