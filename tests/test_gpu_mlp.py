"""The learned-lambda kernels against the FP64 oracle: spectral features,
optimal-error scores, network gradients (at the same FP16-rounded weights),
Adam updates, batched prediction, the feature normaliser, argument checks."""
import math

import numpy as np
import pytest

import synthetic as S
from oracle import kp as KP
from oracle import lam as L
from oracle import mlp as OM
from tests.gpu_util import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

SIZES = (128, 256, 256, 256, 1)


def _unflatten(flat):
    """Flat FP32 parameters -> oracle [(W, b)] in FP64 (same values)."""
    out, off = [], 0
    for fan_in, fan_out in zip(SIZES[:-1], SIZES[1:]):
        W = flat[off:off + fan_in * fan_out].astype(np.float64).reshape(fan_out, fan_in)
        off += fan_in * fan_out
        b = flat[off:off + fan_out].astype(np.float64)
        off += fan_out
        out.append((W, b))
    assert off == flat.size
    return out


def _flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def _random_params(seed):
    from paper_2311_15393_amd.lambda_net import init_params
    flat = init_params(seed)
    rng = np.random.default_rng(seed + 1)
    # non-zero biases so that their gradients and the bias add are exercised
    params = _unflatten(flat)
    params = [(W, rng.uniform(-0.1, 0.1, b.shape)) for W, b in params]
    return _flatten(params).astype(np.float32)


@pytest.mark.parametrize("case", [(100, 31, "m"), (256, 15, "g"), (128, 63, "m")])
def test_features_match_oracle(case):
    require_gpu()
    from paper_2311_15393_amd import Plan
    n, k, kind = case
    rng = np.random.default_rng(n + k)
    psf = (S.psf_gaussian(k, 2.5, 1.7, 0.4) if kind == "g"
           else S.psf_moffat_motion(k, 4.0, 2.5, 5.0, 1.1))
    prob = S.make_problem(n, psf, rng, 0.01, None, n + k, kind)
    plan = Plan(psf, n)
    f = plan.features(to_dev(prob.b)).cpu().numpy().astype(np.float64)
    kp = KP.kp_svd(psf, n)
    c = kp.Vc.T @ prob.b.astype(np.float64) @ kp.Vr
    ref = OM.spectral_features(c, kp.sc, kp.sr)
    say(f"features n={n} k={k}: max |d power| {np.abs(f[:64] - ref[:64]).max():.2e}, "
        f"bins used {(ref[64:] > -11).sum()}")
    # bin counts are integers: the density features must agree to FP32 rounding
    assert np.allclose(f[64:], ref[64:].astype(np.float32), rtol=0, atol=1e-6)
    # power features: log10 of FP64 means of FP32-GEMM coefficients
    assert np.abs(f[:64] - ref[:64]).max() <= 1e-4
    plan.close()


def test_opt_lambda_matches_oracle():
    require_gpu()
    from paper_2311_15393_amd import Plan
    from paper_2311_15393_amd.lambda_net import OPT_GRID
    for prob in S.training_group(7, per_psf=2, n=192):
        plan = Plan(prob.psf, prob.n)
        lam, sc = plan.opt(to_dev(prob.b), to_dev(prob.x_true.astype(np.float32)), OPT_GRID)
        kp = KP.kp_svd(prob.psf, prob.n)
        ref = L.optimal_error(kp, prob.b.astype(np.float64),
                              prob.x_true.astype(np.float32).astype(np.float64), OPT_GRID)
        rel = np.max(np.abs(sc - ref) / ref)
        say(f"opt n={prob.n} {prob.kind}: lam {lam:.3g} vs {OPT_GRID[L.grid_argmin(ref)]:.3g}, "
            f"max rel score diff {rel:.1e}")
        assert rel <= 1e-5
        assert lam == OPT_GRID[L.grid_argmin(ref)]
        plan.close()


def _grad_case(nb, seed):
    import torch
    from paper_2311_15393_amd import Mlp
    rng = np.random.default_rng(seed)
    flat = _random_params(seed)
    X = rng.standard_normal((nb, 128)).astype(np.float32)
    t = rng.uniform(-4, 0, nb).astype(np.float32)
    m = Mlp(max_batch=max(nb, 64))
    m.set_params(flat)
    loss, g = m.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda())
    m.close()
    ref_loss, ref = OM.loss_and_grads(_unflatten(flat), X.astype(np.float64),
                                      t.astype(np.float64), fp16=True)
    return loss, _unflatten(g), ref_loss, ref


@pytest.mark.parametrize("nb", [1, 100, 256])
def test_gradients_match_oracle(nb):
    """Device loss and gradients vs the oracle's FP64 backward pass through
    the same FP16-rounded weights and activations.  Differences come from
    FP32 accumulation (K <= 256: ~1e-6 relative) and from activations whose
    FP32 and FP64 pre-activations round to neighbouring FP16 values (one
    FP16 ulp, 2^-11 relative, for a small fraction of entries); 1e-3 per
    tensor bounds both with a wide margin.  Entry by entry, no gradient may
    be off by more than 1e-3 of its tensor's largest entry (a single wrong
    entry of a 256 x 256 tensor could hide in the normwise figure; measured
    at most 3.5e-5)."""
    require_gpu()
    loss, g, ref_loss, ref = _grad_case(nb, 11 + nb)
    assert abs(loss - ref_loss) <= 1e-5 * max(ref_loss, 1e-12)
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(g, ref)):
        eW = np.linalg.norm(gW - rW) / np.linalg.norm(rW)
        eb = np.linalg.norm(gb - rb) / max(np.linalg.norm(rb), 1e-30)
        mW = np.abs(gW - rW).max() / np.abs(rW).max()
        mb = np.abs(gb - rb).max() / max(np.abs(rb).max(), 1e-30)
        say(f"nb={nb} layer {li + 1}: dW rel {eW:.1e} (entrywise {mW:.1e}), "
            f"db rel {eb:.1e} (entrywise {mb:.1e})")
        assert eW <= 1e-3 and eb <= 1e-3
        assert mW <= 1e-3 and mb <= 1e-3


def test_adam_steps_match_oracle():
    """Two Adam steps: the device's new master weights equal the oracle's
    Adam update applied to the device's own gradients."""
    require_gpu()
    import torch
    from paper_2311_15393_amd import Mlp
    rng = np.random.default_rng(5)
    flat = _random_params(5)
    X = torch.from_numpy(rng.standard_normal((64, 128)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.uniform(-4, 0, 64).astype(np.float32)).cuda()
    m = Mlp(max_batch=64)
    m.set_params(flat)
    params = _unflatten(flat)
    mom, vel = OM.zeros_like(params), OM.zeros_like(params)
    for step in (1, 2):
        _, g = m.gradients(X, t)
        lr = 1e-3 * step
        m.train_step(X, t, lr)
        params, mom, vel = OM.adam_step(params, _unflatten(g), mom, vel, step, lr=lr)
        got = m.get_params().astype(np.float64)
        d = np.abs(got - _flatten(params)).max()
        say(f"adam step {step}: max |dp| {d:.2e}")
        assert d <= 1e-6
        params = _unflatten(got.astype(np.float32))   # continue from the device's weights
    m.close()


def test_predict_matches_oracle_with_normaliser():
    """lambda_predict over more rows than the model's batch (chunked), with a
    non-trivial normaliser, vs the oracle forward at the same rounding."""
    require_gpu()
    import torch
    from paper_2311_15393_amd import Mlp
    rng = np.random.default_rng(9)
    flat = _random_params(9)
    nb = 1000
    X = (rng.standard_normal((nb, 128)) * 3 + 1).astype(np.float32)
    mu = rng.uniform(-1, 2, 128).astype(np.float32)
    sc = rng.uniform(1, 4, 128).astype(np.float32)
    m = Mlp(max_batch=384)
    m.set_params(flat)
    m.set_normalizer(mu, sc)
    y = m.predict(torch.from_numpy(X).cuda()).cpu().numpy()
    # the device standardises in FP32 before rounding to FP16: give the
    # oracle the same FP32-standardised input
    Xn = ((X - mu) / sc).astype(np.float32).astype(np.float64)
    ref, _ = OM.forward(_unflatten(flat), Xn, fp16=True)
    d = np.abs(y - ref).max()
    say(f"predict: max |dy| {d:.2e} (|y| up to {np.abs(ref).max():.2f})")
    assert d <= 1e-3 * max(1.0, np.abs(ref).max())
    m.close()


def test_fit_normalizer():
    require_gpu()
    import torch
    from paper_2311_15393_amd import Mlp
    rng = np.random.default_rng(2)
    X = (rng.standard_normal((777, 128)) * rng.uniform(0.1, 5, 128)
         + rng.uniform(-10, 10, 128)).astype(np.float32)
    X[:, 5] = -12.0                                  # constant feature
    m = Mlp(max_batch=64)
    m.fit_normalizer(torch.from_numpy(X).cuda())
    mu, sc = m.get_normalizer()
    X64 = X.astype(np.float64)
    ref_sd = X64.std(axis=0)
    ref_sd[5] = 1.0
    assert np.allclose(mu, X64.mean(axis=0), rtol=1e-6, atol=1e-5)
    assert np.allclose(sc, ref_sd, rtol=1e-5)
    m.close()


def test_training_overfits_small_batch():
    """64 samples, 400 Adam steps: the training loss falls by 100x."""
    require_gpu()
    import torch
    from paper_2311_15393_amd import Mlp
    from paper_2311_15393_amd.lambda_net import init_params
    rng = np.random.default_rng(4)
    X = torch.from_numpy(rng.standard_normal((64, 128)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.uniform(-4, 0, 64).astype(np.float32)).cuda()
    m = Mlp(max_batch=64)
    m.set_params(init_params(4))
    first = m.train_step(X, t, 1e-3, want_loss=True)
    for _ in range(400):
        last = m.train_step(X, t, 1e-3, want_loss=False)
    last = m.train_step(X, t, 1e-4, want_loss=True)
    say(f"overfit: loss {first:.3e} -> {last:.3e}")
    assert last <= first / 100
    m.close()


def test_mlp_rejects_bad_arguments():
    require_gpu()
    import torch
    from paper_2311_15393_amd import KP_ERR_ARG, KPError, Mlp, Plan
    from paper_2311_15393_amd.lambda_net import init_params
    m = Mlp(max_batch=32)
    bad = init_params(0)
    bad[17] = np.nan
    with pytest.raises(KPError) as ei:
        m.set_params(bad)
    assert ei.value.status == KP_ERR_ARG
    X = torch.zeros((40, 128), device="cuda")
    t = torch.zeros(40, device="cuda")
    with pytest.raises(KPError):
        m.train_step(X, t, 1e-3)                       # 40 rows > max_batch 32
    with pytest.raises(KPError):
        m.train_step(X, t, 1e-3, rows=np.array([0, 40]))
    with pytest.raises(KPError):
        m.set_normalizer(np.zeros(128), np.zeros(128))
    prob = S.small_gaussian(0)
    plan = Plan(prob.psf, prob.n)
    with pytest.raises(KPError):
        plan.lambda_learned(m, to_dev(prob.b), S.lambda_grid(64), tau=0.1)
    with pytest.raises(KPError):
        plan.lambda_learned(m, to_dev(prob.b), S.lambda_grid(), tau=-1.0)
    plan.close()
    m.close()


def test_lambda_learned_fallback_rule():
    """kp_lambda_learned: lambda_pred is 10^(network output) clipped to the
    grid, the GCV ratio is G(lambda_pred)/min G - 1 with G from gcv_lambda's
    own scores, and the choice falls back exactly when ratio > tau."""
    require_gpu()
    from paper_2311_15393_amd import Mlp, Plan
    prob = S.mid_anisotropic(1)
    plan = Plan(prob.psf, prob.n)
    b = to_dev(prob.b)
    grid = S.lambda_grid()
    m = Mlp(max_batch=8)
    params = np.zeros(164865, dtype=np.float32)
    for y in (-2.7, 0.5, -9.0):
        params[-1] = y                       # output bias only: y is the prediction
        m.set_params(params)
        info = plan.lambda_learned(m, b, grid, tau=0.05)
        lp = min(max(10.0 ** y, grid[0]), grid[-1])
        assert math.isclose(info["lambda_pred"], lp, rel_tol=1e-6)
        lam_g, g = plan.gcv(b, grid)
        _, gp = plan.gcv(b, [info["lambda_pred"]])
        ratio = gp[0] / g.min() - 1
        assert math.isclose(info["gcv_ratio"], ratio, rel_tol=1e-9, abs_tol=1e-12)
        assert info["lambda_gcv"] == lam_g
        assert info["fell_back"] == (ratio > 0.05)
        assert info["lambda"] == (lam_g if ratio > 0.05 else info["lambda_pred"])
        say(f"y={y}: pred {info['lambda_pred']:.3g} ratio {ratio:.3g} "
            f"fell_back {info['fell_back']}")
    m.close()
    plan.close()
