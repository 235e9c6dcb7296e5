"""Parameter study of the KP-basis regularisation-parameter rules: weighted
GCV with weight omega and the discrepancy principle with safety factor eta.

    python -m paper_2311_15393_amd.lambda_study [--sizes 128,256] [--per 3]
        [--noise 0.01,0.1] [--json out.json]

The paper evaluates GCV, wGCV (eq. (wGCVTikSVD)) and the discrepancy
principle (eq. (DSCTikSVD)) with the singular values of the Kronecker
approximation (Section 5.1).  It reports that GCV can pick lambda too small
for non-Gaussian blurs, that wGCV with omega > 1 repairs this and is
insensitive to omega between about 2 and 8, and that the discrepancy
principle needs eta > 1 and is sensitive to it, with the best eta up to 15.

Here every rule picks lambda on the same log grid with the library's own
selectors (gcv_lambda with omega, discrepancy_lambda with eta, and
opt_lambda, the optimal-error choice in the KP basis that needs the true
image), each choice is solved with the FP16 KP-preconditioned flexible PCG,
and the reconstruction error ||x - x_true|| / ||x_true|| is reported per
rule, relative to the best error on the grid (every grid lambda is solved:
the optimal-error rule works with the Kronecker model, so it is not always
the true best).  Problems are the synthetic
stand-ins of study_problem (Gaussian, defocus, motion and Moffat + motion
blurs, 1% and 10% noise).
"""
from __future__ import annotations

import argparse
import json

import numpy as np

OMEGAS = (1.0, 2.0, 3.0, 5.0, 8.0)
ETAS = (1.0, 2.0, 3.0, 5.0, 10.0, 15.0)
KINDS = ("gauss", "defocus", "motion", "moffat")


def rule_names(omegas=OMEGAS, etas=ETAS):
    return (["best", "opt"] + [f"wgcv{w:g}" for w in omegas] + [f"dp{e:g}" for e in etas])


def study(problems, grid, omegas=OMEGAS, etas=ETAS, tol: float = 1e-6, maxit: int = 500,
          log=None):
    """For each problem: a solve at every grid lambda and its error against
    the true image, the lambda of every rule and its error ("best" is the
    grid lambda with the smallest error).  Returns one dict per problem."""
    import torch
    from . import KP_FPCG, KP_P16, Plan

    dev = torch.device("cuda:0")
    grid = np.asarray(grid, dtype=np.float64)
    rows = []
    for prob in problems:
        with Plan(prob.psf, prob.n) as plan:
            b = torch.from_numpy(prob.b).to(dev)
            xt = torch.from_numpy(prob.x_true.astype(np.float32)).to(dev)
            lams = {"opt": plan.opt(b, xt, grid)[0]}
            for w in omegas:
                lams[f"wgcv{w:g}"] = plan.gcv(b, grid, omega=w)[0]
            for e in etas:
                lams[f"dp{e:g}"] = plan.discrepancy(b, grid, prob.noise_norm, eta=e)[0]
            solved = {}
            for lam in grid:
                x, info = plan.solve(b, float(lam), tol=tol, maxit=maxit,
                                     mode=KP_FPCG | KP_P16, raise_on_fail=False)
                err = float(torch.linalg.vector_norm(x - xt) / torch.linalg.vector_norm(xt))
                solved[float(lam)] = (err, int(info.iters))
            lams["best"] = min(solved, key=lambda l: solved[l][0])
        row = {"kind": prob.kind, "n": prob.n, "noise": prob.noise_level, "seed": prob.seed,
               "lam": lams, "err": {r: solved[l][0] for r, l in lams.items()},
               "iters": {r: solved[l][1] for r, l in lams.items()}}
        rows.append(row)
        if log:
            e = row["err"]
            log(f"[lambda_study] {prob.kind} n={prob.n} noise={prob.noise_level:g}: best "
                f"{e['best']:.4f} opt {e['opt']:.4f} gcv {e['wgcv1']:.4f} "
                f"wgcv3 {e.get('wgcv3', float('nan')):.4f} "
                f"dp1 {e['dp1']:.4f} dp2 {e.get('dp2', float('nan')):.4f}")
    return rows


def summarize(rows, omegas=OMEGAS, etas=ETAS):
    """Per rule, over all problems and per blur family: the median and the
    worst ratio of its error to the grid's best, and how often it is within
    10% of it.  Also the spread of wGCV over omega in [2, 8] and of
    the discrepancy principle over eta in [2, 5] (max / min error per problem,
    median over problems)."""
    names = rule_names(omegas, etas)
    fams = sorted({r["kind"].rstrip("0123456789") for r in rows})
    out = {"rules": {}, "families": {}, "spread": {}}
    for name in names:
        ratio = np.array([r["err"][name] / r["err"]["best"] for r in rows])
        out["rules"][name] = {"median_ratio": float(np.median(ratio)),
                              "worst_ratio": float(ratio.max()),
                              "within_10pct": float(np.mean(ratio <= 1.1))}
    for fam in fams:
        sub = [r for r in rows if r["kind"].rstrip("0123456789") == fam]
        out["families"][fam] = {
            name: float(np.median([r["err"][name] / r["err"]["best"] for r in sub]))
            for name in names}
    w = [f"wgcv{x:g}" for x in omegas if 2.0 <= x <= 8.0]
    d = [f"dp{x:g}" for x in etas if 2.0 <= x <= 5.0]
    for key, cols in (("wgcv_omega_2_8", w), ("dp_eta_2_5", d)):
        if cols:
            sp = [max(r["err"][c] for c in cols) / min(r["err"][c] for c in cols) for r in rows]
            out["spread"][key] = float(np.median(sp))
    best_eta = []
    for r in rows:
        best = min((r["err"][f"dp{e:g}"], e) for e in etas)
        best_eta.append(best[1])
    out["best_eta_counts"] = {f"{e:g}": int(sum(1 for b in best_eta if b == e)) for e in etas}
    return out


def table(summary, omegas=OMEGAS, etas=ETAS) -> str:
    names = rule_names(omegas, etas)
    fams = list(summary["families"])
    lines = ["| rule | median err / best | worst | within 10% | " +
             " | ".join(f"{f} (median)" for f in fams) + " |",
             "|---|---:|---:|---:|" + "---:|" * len(fams)]
    for name in names:
        s = summary["rules"][name]
        lines.append(f"| {name} | {s['median_ratio']:.3f} | {s['worst_ratio']:.2f} | "
                     f"{100 * s['within_10pct']:.0f}% | " +
                     " | ".join(f"{summary['families'][f][name]:.3f}" for f in fams) + " |")
    return "\n".join(lines)


def main():
    import synthetic as S
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="128,256")
    ap.add_argument("--per", type=int, default=3, help="problems per (blur, size, noise)")
    ap.add_argument("--noise", default="0.01,0.1")
    ap.add_argument("--grid", type=int, default=48, help="points of the log grid on [1e-4, 1]")
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    sizes = [int(v) for v in args.sizes.split(",")]
    noises = [float(v) for v in args.noise.split(",")]
    probs = [S.study_problem(kind, n, nu, i) for kind in KINDS for n in sizes for nu in noises
             for i in range(args.per)]
    rows = study(probs, S.lambda_grid(args.grid), log=print)
    summary = summarize(rows)
    print(table(summary))
    print("spread (median over problems of max/min error):", json.dumps(summary["spread"]))
    print("best eta per problem:", json.dumps(summary["best_eta_counts"]))
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"rows": rows, "summary": summary}, f)


if __name__ == "__main__":
    main()
