"""Training and use of the lambda-predicting network.

Orchestration only: the features, the optimal-error targets, the forward and
backward passes, Adam and the GCV check all run in libkpcg (kp_features,
opt_lambda, mlp_train_step, lambda_predict, kp_lambda_learned in
include/kpcg.h).  This module picks problems, minibatch order, the learning
rate schedule and the fallback threshold.

The paper chooses lambda with GCV / weighted GCV / the discrepancy principle
in the KP-SVD basis (Section 2.2, Section 5.1) and leaves a more systematic
choice open (Section 5.1, Section 6); the network is this library's answer,
with GCV kept as the judge: a prediction whose GCV score exceeds the grid
minimum by more than a threshold tau falls back to the GCV grid choice.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .kpcg import KP_MLP_HIDDEN, KP_MLP_NFEAT, KP_MLP_NPARAM, Mlp, Plan

# 64-point grid of the optimal-error targets and 32-point GCV grid, both on
# [1e-4, 1]
OPT_GRID = np.logspace(-4.0, 0.0, 64)
GCV_GRID = np.logspace(-4.0, 0.0, 32)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, in the flat
    FP32 layout of include/kpcg.h."""
    rng = np.random.default_rng(seed)
    sizes = (KP_MLP_NFEAT, KP_MLP_HIDDEN, KP_MLP_HIDDEN, KP_MLP_HIDDEN, 1)
    parts = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        bound = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-bound, bound, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == KP_MLP_NPARAM
    return flat


@dataclasses.dataclass
class Dataset:
    features: object          # CUDA float32 (N, 128)
    targets: object           # CUDA float32 (N,): log10 lambda_opt
    log_gcv: np.ndarray       # log10 of the GCV grid choice per problem
    sizes: np.ndarray         # image size per problem


def _same_psf(a, b) -> bool:
    return a is not None and a.shape == b.shape and np.array_equal(a, b)


def build_dataset(problems, device, opt_grid=OPT_GRID, gcv_grid=GCV_GRID) -> Dataset:
    """Features of each problem's data and its optimal-error lambda (the
    target).  Consecutive problems with the same PSF and size share a plan."""
    import torch
    problems = list(problems)
    N = len(problems)
    feats = torch.empty((N, KP_MLP_NFEAT), device=device, dtype=torch.float32)
    tgt = np.empty(N, dtype=np.float32)
    lg = np.empty(N)
    plan, plan_psf, plan_n = None, None, None
    for i, p in enumerate(problems):
        if plan is None or plan_n != p.n or not _same_psf(plan_psf, p.psf):
            if plan is not None:
                plan.close()
            plan, plan_psf, plan_n = Plan(p.psf, p.n), p.psf, p.n
        b = torch.from_numpy(p.b).to(device)
        xt = torch.from_numpy(p.x_true.astype(np.float32)).to(device)
        plan.features(b, out=feats[i])
        lam_opt, _ = plan.opt(b, xt, opt_grid)
        lam_gcv, _ = plan.gcv(b, gcv_grid)
        tgt[i] = math.log10(lam_opt)
        lg[i] = math.log10(lam_gcv)
    if plan is not None:
        plan.close()
    return Dataset(feats, torch.from_numpy(tgt).to(device), lg,
                   np.array([p.n for p in problems]))


def train(mlp: Mlp, data: Dataset, epochs: int = 300, batch: int = 256, lr: float = 1e-3,
          lr_final: float = 1e-5, seed: int = 0, fit_normalizer: bool = True):
    """Adam on shuffled minibatches, learning rate decayed geometrically
    from lr to lr_final over the run.  Returns the per-epoch loss of the last
    minibatch."""
    N = int(data.features.shape[0])
    if fit_normalizer:
        mlp.fit_normalizer(data.features)
    rng = np.random.default_rng(seed)
    steps_per_epoch = max(1, (N + batch - 1) // batch)
    total = epochs * steps_per_epoch
    decay = (lr_final / lr) ** (1.0 / max(1, total - 1))
    hist = []
    step = 0
    for _ in range(epochs):
        perm = rng.permutation(N).astype(np.int32)
        loss = None
        for s in range(steps_per_epoch):
            rows = perm[s * batch:(s + 1) * batch]
            last = s == steps_per_epoch - 1
            loss = mlp.train_step(data.features, data.targets, lr * decay ** step, rows=rows,
                                  want_loss=last)
            step += 1
        hist.append(loss)
    return hist


def predict_log10(mlp: Mlp, data: Dataset) -> np.ndarray:
    return mlp.predict(data.features).cpu().numpy()


def calibrate_tau(mlp: Mlp, problems, device, q: float = 0.95, grid=GCV_GRID) -> float:
    """tau = the q-quantile over held-out problems of G(lambda_pred) / min G - 1
    (the GCV excess of the network's choice)."""
    import torch
    ratios = []
    plan, plan_psf, plan_n = None, None, None
    for p in problems:
        if plan is None or plan_n != p.n or not _same_psf(plan_psf, p.psf):
            if plan is not None:
                plan.close()
            plan, plan_psf, plan_n = Plan(p.psf, p.n), p.psf, p.n
        info = plan.lambda_learned(mlp, torch.from_numpy(p.b).to(device), grid, tau=1e300)
        ratios.append(info["gcv_ratio"])
    if plan is not None:
        plan.close()
    return float(np.quantile(np.asarray(ratios), q))
