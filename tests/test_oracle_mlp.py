"""Pins for the oracle's network and features."""
import numpy as np
import pytest

from oracle import kp as KP
from oracle import mlp as M
import synthetic as S


def _small(rng):
    return M.init_params(rng, sizes=(6, 5, 4, 1))


def test_gradcheck_central_differences():
    rng = np.random.default_rng(0)
    params = _small(rng)
    X = rng.standard_normal((7, 6))
    t = rng.standard_normal(7)
    loss, grads = M.loss_and_grads(params, X, t)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gf = g.reshape(-1)
            for idx in rng.choice(flat.size, min(flat.size, 6), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = M.loss_and_grads(params, X, t)
                flat[idx] = old - h
                lm, _ = M.loss_and_grads(params, X, t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gf[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_gelu_matches_definition():
    from scipy.stats import norm
    z = np.linspace(-5, 5, 41)
    assert np.allclose(M.gelu(z), z * norm.cdf(z), atol=1e-15)
    h = 1e-6
    assert np.allclose(M.gelu_grad(z), (M.gelu(z + h) - M.gelu(z - h)) / (2 * h), atol=1e-8)


def test_adam_first_step_is_signed_lr():
    """With zero moments, Adam's bias-corrected first step is lr * sign(g)
    (up to eps)."""
    rng = np.random.default_rng(1)
    params = _small(rng)
    grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    new, _, _ = M.adam_step(params, grads, M.zeros_like(params), M.zeros_like(params), 1,
                            lr=0.01)
    for (W, b), (W2, b2), (gW, gb) in zip(params, new, grads):
        assert np.allclose(W - W2, 0.01 * np.sign(gW), atol=1e-9)


def test_one_sample_overfit():
    rng = np.random.default_rng(2)
    params = M.init_params(rng, sizes=(8, 16, 16, 16, 1))
    X = rng.standard_normal((1, 8))
    t = np.array([-2.3])
    m, v = M.zeros_like(params), M.zeros_like(params)
    for step in range(1, 301):
        _, g = M.loss_and_grads(params, X, t)
        params, m, v = M.adam_step(params, g, m, v, step, lr=1e-2)
    loss, _ = M.loss_and_grads(params, X, t)
    assert loss < 1e-6


def test_features_by_brute_force():
    rng = np.random.default_rng(3)
    n = 12
    psf = S.psf_moffat_motion(5, 2.0, 2.5, 3.0, 0.4)
    kp = KP.kp_svd(psf, n)
    c = rng.standard_normal((n, n))
    f = M.spectral_features(c, kp.sc, kp.sr)
    acc = [[] for _ in range(M.NBINS)]
    for i in range(n):
        for j in range(n):
            s = kp.sc[i] * kp.sr[j]
            k = 0 if s <= 0 else int(np.floor((np.log10(s) + 8) / 8 * 64))
            acc[min(max(k, 0), 63)].append(c[i, j] ** 2)
    for k in range(M.NBINS):
        mean = np.mean(acc[k]) if acc[k] else 0.0
        assert np.isclose(f[k], np.log10(max(mean, 1e-30)))
        assert np.isclose(f[64 + k], np.log10(len(acc[k]) / n / n + 1e-12))


def test_fp16_forward_matches_per_layer_half_casts():
    """forward(..., fp16=True) against torch's own layers in float64 with an
    explicit half-precision cast of each hidden layer's input and weight
    (the cast rounds the double straight to binary16; torch's own float64 ->
    float16 conversion goes through float32 and can double-round, so the
    cast is numpy's).  The output layer stays unrounded, as on the device.
    The check also shows the rounding is visible (differs from the FP64
    forward) and that rounding the output layer too would differ."""
    import torch

    rng = np.random.default_rng(4)
    params = M.init_params(rng)
    X = rng.standard_normal((9, M.NFEAT)) * 3.0
    mu = rng.standard_normal(M.NFEAT)
    scale = rng.uniform(0.5, 2.0, M.NFEAT)

    def half(t):
        return torch.from_numpy(t.numpy().astype(np.float16).astype(np.float64))

    def reference(round_last):
        h = (torch.from_numpy(X) - torch.from_numpy(mu)) / torch.from_numpy(scale)
        for li, (W, b) in enumerate(params):
            last = li == len(params) - 1
            Wt, bt = torch.from_numpy(W), torch.from_numpy(b)
            if not last or round_last:
                h, Wt = half(h), half(Wt)
            z = torch.nn.functional.linear(h, Wt, bt)
            h = z if last else torch.nn.functional.gelu(z, approximate="none")
        return h[:, 0].numpy()

    y16, _ = M.forward(params, X, mu, scale, fp16=True)
    y64, _ = M.forward(params, X, mu, scale, fp16=False)
    ref = reference(False)
    assert np.allclose(y16, ref, rtol=1e-12, atol=1e-12)
    assert not np.allclose(y64, ref, rtol=1e-7, atol=0)
    assert not np.allclose(reference(True), ref, rtol=1e-9, atol=0)
