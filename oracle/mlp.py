"""FP64 reference of the lambda-predicting network and its input features.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper chooses lambda by GCV, weighted GCV or the discrepancy principle
in the Kronecker basis (Section 2.2, Section 5.1) and ends by asking for a
more systematic way to choose these parameters (Section 5.1, last paragraph;
Section 6).  The network here is this library's own answer to that, not a
method from the paper: it maps spectral features of the data in the KP-SVD
basis to log10(lambda).  Parity status: pinned by central finite differences
(tests/test_oracle_mlp.py); the FP16 forward by torch's own layers with an
explicit binary16 cast of each hidden layer's operands; the features by
brute-force binning.

Features (128 per problem), from the coefficients c = V_c^T B V_r and the
singular values s_ij = s_c[i] s_r[j] of the Kronecker approximation:
  * 64 bins of log10(s) over [-8, 0] (s below 1e-8 go to bin 0, s >= 1 to
    bin 63);
  * f[k]      = log10(max(mean of c^2 over bin k, 1e-30)), empty bins 1e-30;
  * f[64 + k] = log10(count of bin k / N + 1e-12).
They are standardised with per-feature mean and scale stored in the model.

Network: 128 -> 256 -> 256 -> 256 -> 1, exact GELU, g(z) = z Phi(z), after
each hidden layer, linear output.  Loss: mean over the batch of (y - t)^2.
Adam with bias correction.  Weights are stored [out][in].  The device runs
the hidden layers with FP16 weights and FP16 activations (FP32 accumulation);
`forward(..., fp16=True)` rounds the same operands to FP16 so its output and
gradients are those of the function the device computes.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

NBINS = 64
NFEAT = 2 * NBINS
LOGS_LO, LOGS_HI = -8.0, 0.0


def spectral_features(c: np.ndarray, sc: np.ndarray, sr: np.ndarray) -> np.ndarray:
    """The 128 raw features of one problem (see module docstring)."""
    s = np.outer(sc, sr).ravel()
    c2 = np.asarray(c, dtype=np.float64).ravel() ** 2
    with np.errstate(divide="ignore"):
        ls = np.log10(s)
    b = np.floor((ls - LOGS_LO) / (LOGS_HI - LOGS_LO) * NBINS)
    b = np.clip(np.nan_to_num(b, nan=0.0, neginf=0.0), 0, NBINS - 1).astype(int)
    cnt = np.bincount(b, minlength=NBINS).astype(np.float64)
    pw = np.bincount(b, weights=c2, minlength=NBINS)
    mean = np.where(cnt > 0, pw / np.maximum(cnt, 1), 0.0)
    f = np.empty(NFEAT)
    f[:NBINS] = np.log10(np.maximum(mean, 1e-30))
    f[NBINS:] = np.log10(cnt / s.size + 1e-12)
    return f


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def round16(x):
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def init_params(rng: np.random.Generator, sizes=(128, 256, 256, 256, 1)):
    """He-uniform weights, zero biases; returns a list of (W[out][in], b[out])."""
    params = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        bound = math.sqrt(6.0 / fan_in)
        W = rng.uniform(-bound, bound, (fan_out, fan_in))
        params.append((W, np.zeros(fan_out)))
    return params


def forward(params, X, mu=None, scale=None, fp16=False):
    """Returns (y, cache).  X is (batch, 128) raw features."""
    h = np.asarray(X, dtype=np.float64)
    if mu is not None:
        h = (h - mu) / scale
    cache = []
    L = len(params)
    for li, (W, b) in enumerate(params):
        last = li == L - 1
        hin = round16(h) if (fp16 and not last) else h
        Wl = round16(W) if (fp16 and not last) else W
        z = hin @ Wl.T + b
        cache.append((hin, Wl, z))
        h = z if last else gelu(z)
    return h[:, 0], cache


def loss_and_grads(params, X, t, mu=None, scale=None, fp16=False):
    """MSE loss mean((y - t)^2) and its gradients (list of (dW, db))."""
    y, cache = forward(params, X, mu, scale, fp16)
    B = y.shape[0]
    dz = (2.0 / B) * (y - np.asarray(t, dtype=np.float64))[:, None]
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        hin, Wl, z = cache[li]
        if li != len(params) - 1:
            dz = dh * gelu_grad(z)
        grads[li] = (dz.T @ hin, dz.sum(axis=0))
        dh = dz @ Wl
    loss = float(np.mean((y - t) ** 2))
    return loss, grads


def adam_step(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (in place on copies); returns new (params, m, v)."""
    out, mo, vo = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        new = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = b1 * mm + (1 - b1) * g
            vv = b2 * vv + (1 - b2) * g * g
            mhat = mm / (1 - b1 ** step)
            vhat = vv / (1 - b2 ** step)
            new.append((p - lr * mhat / (np.sqrt(vhat) + eps), mm, vv))
        out.append((new[0][0], new[1][0]))
        mo.append((new[0][1], new[1][1]))
        vo.append((new[0][2], new[1][2]))
    return out, mo, vo


def zeros_like(params):
    return [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
