"""Train the lambda-predicting network on generated problems and report its
gain over GCV on held-out problems of the uneven-size batch.

    python -m paper_2311_15393_amd.train_lambda [--groups 2500] [--per-psf 8]
        [--epochs 60] [--test 48] [--out model.npz]

Training problems: `groups` PSFs drawn from the uneven batch's mix, each
with `per-psf` 256 x 256 images and noise levels (2500 x 8 = 20,000
problems); targets are the optimal-error lambda in the KP-SVD basis on a
64-point grid.  Validation problems (held out, their own seeds) set the GCV
fallback threshold tau.  Test problems: the first `test` problems of the
uneven batch (sizes 128..1024), each solved at the GCV lambda, the learned
lambda (with fallback) and the optimal-error lambda.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def run(groups: int, per_psf: int, epochs: int, ntest: int, val_groups: int = 64,
        seed: int = 0, log=print):
    import torch
    import synthetic as S
    from . import Mlp
    from . import lambda_net as LN

    dev = torch.device("cuda:0")
    t0 = time.time()
    train = [p for g in range(groups) for p in S.training_group(g, per_psf=per_psf)]
    data = LN.build_dataset(train, dev)
    val = [p for g in range(val_groups)
           for p in S.training_group(g, per_psf=4, seed0=S.VAL_SEED0)]
    vdata = LN.build_dataset(val, dev)
    t1 = time.time()
    log(f"[train_lambda] {len(train)} training / {len(val)} validation problems "
        f"built in {t1 - t0:.1f}s")
    mlp = Mlp(max_batch=512)
    mlp.set_params(LN.init_params(seed))
    torch.cuda.synchronize()
    t2 = time.time()
    hist = LN.train(mlp, data, epochs=epochs, batch=256, lr=1e-3, seed=seed)
    torch.cuda.synchronize()
    t3 = time.time()
    steps = epochs * ((len(train) + 255) // 256)
    tt = data.targets.cpu().numpy()
    vt = vdata.targets.cpu().numpy()
    rmse = lambda a, b: float(np.sqrt(np.mean((np.asarray(a) - np.asarray(b)) ** 2)))
    out = {
        "train_problems": len(train), "val_problems": len(val), "epochs": epochs,
        "train_s": t3 - t2, "adam_steps": steps, "loss_last": hist[-1],
        "rmse_train": rmse(LN.predict_log10(mlp, data), tt),
        "rmse_val": rmse(LN.predict_log10(mlp, vdata), vt),
        "rmse_val_gcv": rmse(vdata.log_gcv, vt),
    }
    tau = LN.calibrate_tau(mlp, val, dev)
    out["tau"] = tau
    log(f"[train_lambda] trained in {t3 - t2:.1f}s ({steps} Adam steps); log10-lambda rmse "
        f"train {out['rmse_train']:.3f} val {out['rmse_val']:.3f} (GCV {out['rmse_val_gcv']:.3f}); "
        f"tau {tau:.3f}")
    if ntest:
        out.update(gain(mlp, tau, ntest, dev, log))
    return mlp, out


def gain(mlp, tau: float, ntest: int, dev, log=print) -> dict:
    """Relative error ||x - x_true|| / ||x_true|| of the FP16-KP FPCG solution
    at the GCV, learned (with fallback) and optimal-error lambda, for the
    first `ntest` problems of the uneven batch."""
    import torch
    import synthetic as S
    from . import KP_FPCG, KP_P16, Plan, solve_batched
    from . import lambda_net as LN
    test = [S.batch_problem(i) for i in range(ntest)]
    tdata = LN.build_dataset(test, dev)
    topt = tdata.targets.cpu().numpy()
    plans = [Plan(p.psf, p.n) for p in test]
    bs = [torch.from_numpy(p.b).to(dev) for p in test]
    learned, fell = [], 0
    for p, pl, b in zip(test, plans, bs):
        info = pl.lambda_learned(mlp, b, LN.GCV_GRID, tau)
        learned.append(info["lambda"])
        fell += int(info["fell_back"])
    pred = LN.predict_log10(mlp, tdata)
    lams = {"gcv": 10.0 ** tdata.log_gcv, "learned": np.asarray(learned), "opt": 10.0 ** topt}
    errs = {}
    for name, lam in lams.items():
        xs, infos, _ = solve_batched(plans, bs, list(lam), list(range(ntest)), tol=1e-6,
                                     maxit=1000, mode=KP_FPCG | KP_P16)
        errs[name] = np.array([np.linalg.norm(x.cpu().numpy() - p.x_true) /
                               np.linalg.norm(p.x_true) for x, p in zip(xs, test)])
    for pl in plans:
        pl.close()
    rmse = lambda a, b: float(np.sqrt(np.mean((np.asarray(a) - np.asarray(b)) ** 2)))
    res = {
        "test_problems": ntest, "fell_back": fell,
        "rmse_test_net": rmse(pred, topt), "rmse_test_gcv": rmse(tdata.log_gcv, topt),
        "err_gcv": float(errs["gcv"].mean()), "err_learned": float(errs["learned"].mean()),
        "err_opt": float(errs["opt"].mean()),
        "wins": int((errs["learned"] < errs["gcv"]).sum()),
        "worst_ratio": float(np.max(errs["learned"] / errs["gcv"])),
    }
    log(f"[train_lambda] uneven batch ({ntest} problems): log10-lambda rmse vs the "
        f"optimal-error choice: network {res['rmse_test_net']:.3f}, GCV {res['rmse_test_gcv']:.3f}; "
        f"mean ||x - x_true||/||x_true||: learned {res['err_learned']:.4f}, GCV "
        f"{res['err_gcv']:.4f}, optimal-error {res['err_opt']:.4f}; learned better on "
        f"{res['wins']}/{ntest}; {fell} fallbacks")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--groups", type=int, default=2500)
    ap.add_argument("--per-psf", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--test", type=int, default=48)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None, help="save parameters, normaliser and tau (.npz)")
    args = ap.parse_args()
    mlp, out = run(args.groups, args.per_psf, args.epochs, args.test, seed=args.seed)
    if args.out:
        mean, scale = mlp.get_normalizer()
        np.savez(args.out, params=mlp.get_params(), mean=mean, scale=scale, tau=out["tau"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
