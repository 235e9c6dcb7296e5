"""Benchmark: 1024^2 deblurring solves/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--seed S]

Workload: 1024 x 1024 synthetic image, Moffat turbulence (beta = 2.5) blur
convolved with a short motion segment on a 63 x 63 support, zero boundary,
2% noise; lambda chosen by GCV on the 32-point log grid [1e-4, 1] in the
KP-SVD basis (the GPU's choice must equal the CPU oracle's).  A step is one
pcg_solve of (A^T A + lambda^2 I) x = A^T b with the FP16 KP-SVD
preconditioner and flexible PCG, from b resident in HBM to x resident in
HBM, at the loosest tolerance (1e-5, tightened 10x at a time) whose solution
is within 1e-4 relative error of the FP64 oracle's x_lambda.  The same
measurement is made for the FP32 preconditioner (PCG), the FP8 one and for
no preconditioner (CG), and for the FP16 / FP32 preconditioners with the
exact KP-basis diagonal (KP_EXACT_DIAG) in place of the one-term singular
values; their numbers are reported beside the headline value.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "1024^2 deblur PCG solves/s at rel err <=1e-4 vs FP64; FP16-KP vs FP32-KP vs none"
HBM_PEAK = 8.0e12
FP32_VALU_PEAK = 157.3e12
FP16_MFMA_PEAK = 2.5e15
# solver modes and their iteration caps
MODES = {"fp16_kp_fpcg": 200, "fp32_kp_pcg": 200, "fp8_kp_fpcg": 400, "none_cg": 3000,
         "fp16_kpdiag_fpcg": 200, "fp32_kpdiag_pcg": 200}
# --profile-only skips the oracle, so it cannot search the tolerance ladder;
# it uses the tolerances the full run picks on this workload (seed 0)
PROFILE_TOLS = {"fp16_kp_fpcg": 2e-6, "fp32_kp_pcg": 1e-5, "fp8_kp_fpcg": 1e-6,
                "none_cg": 5e-7, "fp16_kpdiag_fpcg": 1e-6, "fp32_kpdiag_pcg": 5e-6}
# Bytes of the plain copy launched by --profile-only to calibrate the HBM
# counters (FETCH_SIZE / WRITE_SIZE): 64 Mi floats read, 64 Mi written.
COPY_CALIB_FLOATS = 64 * 1024 * 1024

# HBM traffic of one forward-blur launch at the 1024^2, K=63 workload, from
# two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) of
# `python bench.py --profile-only --modes fp16_kp_fpcg --steps 2 --warmup 1`,
# each divided by the same counter's reading per byte of the calibration copy.
# `sources_sha256` is the hash of the blur sources the counters were taken
# on; when the sources differ the figure no longer describes the kernel and
# is reported as null.
BLUR_TRAFFIC = {
    "kernel": "blur_mfma_kernel<3, EpiStoreF32>",
    "fetch_kib_raw": 5366.8, "write_kib_raw": 4096.0,       # per launch, as counted
    "fetch_scale": 1.99979, "write_scale": 1.0,              # copy bytes / counter
    "bytes_per_launch": 15184347,
    "sources_sha256": "4ffeead0c3a59a727fac05e52b7aac61c7e1735f28b633607da9bda1729ab4ed",
}


CPU_SAMPLE_S = 10.0       # the CPU oracle leg times at least this long ...
CPU_SAMPLE_MAX = 60       # ... or this many solves


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def blur_flops(n: int, k: int) -> float:
    """Algorithmic flops of one zero-boundary direct convolution: 2 per
    (output, tap) pair that touches the image, t(n,K)^2 pairs with
    t = nK - h(h+1) (one factor per image axis)."""
    h = (k - 1) // 2
    t = n * k - h * (h + 1)
    return 2.0 * float(t) * float(t)


def blur_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    # the sources of the MFMA blur kernel the counters describe
    for f in ("blur_core.h", "blur_mfma.h", "blur_mfma.hip"):
        with open(os.path.join(ROOT, "paper_2311_15393_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def blur_traffic(kernel: str):
    """Counter-measured HBM bytes per forward-blur launch of `kernel`, or None
    when no measurement exists for it and the current blur sources."""
    if (BLUR_TRAFFIC is None or BLUR_TRAFFIC["kernel"] != kernel
            or BLUR_TRAFFIC["sources_sha256"] != blur_sources_sha256()):
        return None
    return BLUR_TRAFFIC["bytes_per_launch"]


def mfma_blur_flops(n: int, k: int, cfg: int = 6) -> float:
    """FP16 MFMA flops the MFMA blur issues per launch.  16x16x32 kernel
    (cfg 6): per 64 x 64 tile, 4 row strips x (chunk MFMAs of the K tap
    rows) x 4 blocks x 3 split products of 16384 flop, where the chunks are
    K x NCH, or with paired rows (NCH = 3) 2 NCH - 1 per pair and NCH for a
    row left without a partner (the second wave group's last row).
    32x32x16 kernel (cfg 7): 2 row halves x K tap rows x NC chunks x 2
    blocks x 3 products of 32768 flop."""
    tiles = ((n + 63) // 64) ** 2
    if cfg == 7:
        nc = (k + 31 + 15) // 16
        return tiles * 2.0 * k * nc * 2 * 3 * 32768
    nch = (k + 15 + 31) // 32
    if nch == 3:
        half = (((k + 1) >> 1) + 1) & ~1
        rows1 = k - half
        chunks = (half // 2 + rows1 // 2) * (2 * nch - 1) + (rows1 % 2) * nch
    else:
        chunks = k * nch
    return tiles * 4.0 * chunks * 4 * 3 * 16384


def settled_x_lambda(SV, prob, lam, kp, nthreads):
    """The oracle's x_lambda for a large problem: FP64 KP-PCG to a true
    residual of 1e-13, accepted only when a run at a 100x looser tolerance
    agrees with it to 1e-7 (check=True), it converged, and its true residual
    is at or below 1e-12."""
    x, info = SV.x_lambda_iterative(prob.psf, prob.b.astype(np.float64), lam, kp=kp,
                                    workers=nthreads, check=True)
    assert info["status"] == "converged" and info["true_relres"] <= 1e-12, info
    return x, info


def cpu_threads() -> int:
    try:
        c = len(os.sched_getaffinity(0))
    except Exception:
        c = os.cpu_count() or 1
    return max(1, min(c, 16))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="skip the oracle parts (for profiler runs)")
    ap.add_argument("--no-periodic", action="store_true",
                    help="skip the periodic- and reflexive-boundary solves (also skipped with "
                         "--profile-only)")
    ap.add_argument("--batch", type=int, default=0, metavar="P",
                    help="also run the uneven batched workload with P problems x 16 lambda")
    ap.add_argument("--instances", type=int, default=0, metavar="S",
                    help="also run the FP16 headline on seeds 0 .. S-1 of the large workload "
                         "(GCV index and 1e-4 parity against the oracle per seed)")
    ap.add_argument("--matvec-sweep", action="store_true",
                    help="only compare the direct blurs with a zero-padded rocFFT H p over K "
                         "(prints its own JSON line)")
    ap.add_argument("--modes", default=",".join(MODES),
                    help="comma list of solver modes to run (the first FP16 one is the headline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the solve of one image fits one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import synthetic as S
    from paper_2311_15393_amd import (KP_CG, KP_EXACT_DIAG, KP_FPCG, KP_OK, KP_P8, KP_P16, KP_P32,
                                      KP_PCG, Plan)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    nthreads = cpu_threads()
    if args.matvec_sweep:
        print(json.dumps(run_matvec_sweep(dev)), flush=True)
        return

    t0 = time.time()
    prob = S.large_moffat(args.seed)
    n, k = prob.n, prob.k
    grid = S.lambda_grid()
    log(f"[bench] problem n={n} k={k} generated in {time.time() - t0:.1f}s")

    b = torch.from_numpy(prob.b).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    plan = Plan(prob.psf, n)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    pinfo = plan.query()
    log(f"[bench] kp_setup {setup_s:.2f}s kp_err={pinfo['kp_rel_error']:.3e} "
        f"blur config {pinfo['blur_config']} times(ms) "
        f"{[round(t, 4) for t in pinfo['blur_config_ms'][:6]]}")

    # lambda by KP-GCV on the GPU
    lam, scores = plan.gcv(b, grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        plan.gcv(b, grid)
    torch.cuda.synchronize()
    gcv_ms = (time.perf_counter() - t0) / 5 * 1e3
    gidx = int(np.argmin(np.abs(grid - lam)))
    log(f"[bench] gcv lambda={lam:.4g} (grid index {gidx}) {gcv_ms:.2f} ms")

    learned = time_learned_lambda(plan, b, grid, dev)
    log(f"[bench] learned lambda: kp_lambda_learned {learned['lambda_learned_ms']:.2f} ms at "
        f"{n}^2; lambda_predict {learned['predict_samples_per_s'] / 1e6:.2f} M rows/s; "
        f"train step (256 rows) {learned['train_step_ms']:.3f} ms")

    oracle = {}
    if not args.profile_only:
        from threadpoolctl import threadpool_limits
        from oracle import kp as KP
        from oracle import lam as L
        from oracle import solvers as SV
        with threadpool_limits(limits=nthreads):
            t0 = time.time()
            kp = KP.kp_svd(prob.psf, n)
            s2, bh2 = L.spectrum(kp, prob.b.astype(np.float64))
            ref_idx = L.grid_argmin(L.gcv(s2, bh2, grid))
            oracle["gcv_index"] = ref_idx
            log(f"[bench] oracle KP-SVD + GCV {time.time() - t0:.1f}s index {ref_idx}")
            assert ref_idx == gidx, f"GPU GCV picked grid index {gidx}, oracle {ref_idx}"
            t0 = time.time()
            xlam, xinfo = settled_x_lambda(SV, prob, lam, kp, nthreads)
            log(f"[bench] oracle x_lambda {time.time() - t0:.1f}s iters={xinfo['iters']} "
                f"relres={xinfo['true_relres']:.1e} loose agreement "
                f"{xinfo['loose_agreement']:.1e}")

    def run(mode, tol, maxit):
        x = torch.empty_like(b)
        x, info = plan.solve(b, lam, tol=tol, maxit=maxit, mode=mode, x=x, raise_on_fail=False)
        return x, info

    # tolerance ladder: 1e-5, 5e-6, 2e-6, 1e-6, 5e-7, ... down to 1e-9
    ladder = [m * 10.0 ** e for e in range(-5, -10, -1) for m in (1.0, 0.5, 0.2)] + [1e-9]

    def pick_tol(name, mode, maxit):
        """Loosest tolerance on the ladder whose solution meets the 1e-4 bar."""
        if args.profile_only:
            tol = PROFILE_TOLS[name]
            _, info = run(mode, tol, maxit)
            return tol, info, float("nan")
        for tol in ladder:
            x, info = run(mode, tol, maxit)
            got = x.cpu().numpy().astype(np.float64)
            err = float(np.linalg.norm(got - xlam) / np.linalg.norm(xlam))
            log(f"[bench]   mode={mode:#x} tol={tol:.0e} iters={info.iters} "
                f"status={info.status} err={err:.2e}")
            if info.status == KP_OK and err <= 1e-4:
                return tol, info, err
        return tol, info, err

    def time_mode(mode, tol, maxit, steps, warmup):
        for _ in range(warmup):
            run(mode, tol, maxit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = []
        for _ in range(steps):
            _, info = run(mode, tol, maxit)
            iters.append(info.iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt / steps * 1e3, iters

    # the paper's one-term S (kp) and the exact KP-basis diagonal (kpdiag)
    mode_bits = {"fp16_kp_fpcg": KP_FPCG | KP_P16, "fp32_kp_pcg": KP_PCG | KP_P32,
                 "fp8_kp_fpcg": KP_FPCG | KP_P8, "none_cg": KP_CG,
                 "fp16_kpdiag_fpcg": KP_FPCG | KP_P16 | KP_EXACT_DIAG,
                 "fp32_kpdiag_pcg": KP_PCG | KP_P32 | KP_EXACT_DIAG}
    chosen = [m for m in args.modes.split(",") if m]
    assert "fp16_kp_fpcg" in chosen and all(m in MODES for m in chosen), args.modes
    modes = {m: (mode_bits[m], MODES[m]) for m in chosen}
    results = {}
    for name, (mode, maxit) in modes.items():
        tol, info, err = pick_tol(name, mode, maxit)
        steps = args.steps if name == "fp16_kp_fpcg" else max(1, min(args.steps, 5))
        warm = args.warmup if name == "fp16_kp_fpcg" else 1
        ms, iters = time_mode(mode, tol, maxit, steps, warm)
        results[name] = {"tol": tol, "iters": info.iters, "rel_err": err,
                         "ms_per_solve": ms, "solves_per_s": 1e3 / ms,
                         "ok": bool(info.status == KP_OK and (err <= 1e-4 or args.profile_only))}
        log(f"[bench] {name}: tol={tol:.0e} iters={info.iters} err={err:.2e} "
            f"{ms:.3f} ms/solve")

    # dominant kernel: the blur matvec (two per iteration), as autotuned
    p = torch.randn((n, n), device=dev, dtype=torch.float32)
    q = torch.empty_like(p)
    plan.time_blur(p, q, reps=3)
    blur_ms = plan.time_blur(p, q, transpose=False, reps=20)
    flops = blur_flops(n, k)
    achieved = flops / (blur_ms * 1e-3)
    prec_ms = plan.time_precond(p, lam, KP_P16, q, reps=20)
    prec_flops = 8.0 * n ** 3
    log(f"[bench] blur kernel {blur_ms * 1e3:.1f} us ({achieved / 1e12:.2f} TFLOP/s); "
        f"FP16 preconditioner chain {prec_ms * 1e3:.1f} us "
        f"({prec_flops / (prec_ms * 1e-3) / 1e12:.1f} TFLOP/s)")

    if args.profile_only:
        # plain copy of known size for the counter calibration
        src = torch.ones(COPY_CALIB_FLOATS, device=dev, dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    if pinfo["blur_config"] in (6, 7):
        if pinfo["blur_config"] == 6:
            kname = f"blur_mfma_kernel<{(k + 46) // 32}, EpiStoreF32>"
        else:
            kname = f"blur_mfma32_kernel<{(k + 46) // 16}, EpiStoreF32>"
        issued = mfma_blur_flops(n, k, pinfo["blur_config"]) / (blur_ms * 1e-3)
        roofline = {
            "bound": "mfma", "achieved": achieved / 1e12, "peak": FP16_MFMA_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": achieved / FP16_MFMA_PEAK,
            "traffic": blur_traffic(kname),
            "kernel": kname + " (A p on FP16-split MFMA; achieved = algorithmic convolution "
                              "flops / time)",
            "avg_us": blur_ms * 1e3,
            "mfma_issued_tflops": issued / 1e12, "mfma_issued_frac": issued / FP16_MFMA_PEAK,
        }
    else:
        kname = "blur_kernel<{}, EpiStoreF32>".format(pinfo["blur_config"])
        roofline = {
            "bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VALU_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": achieved / FP32_VALU_PEAK,
            "traffic": blur_traffic(kname),
            "kernel": kname + " (direct convolution A p, FP32 VALU)",
            "avg_us": blur_ms * 1e3,
        }

    cpu_baseline = None
    if not args.profile_only and not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits
        from oracle import solvers as SV
        with threadpool_limits(limits=nthreads):
            op = SV.NormalOperator(prob.psf, n, lam, workers=nthreads)
            pre = SV.kp_preconditioner(prob.psf, n, lam, kp)
            # repeat the solve for at least CPU_SAMPLE_S (at most CPU_SAMPLE_MAX solves)
            t0 = time.time()
            count = 0
            while True:
                out = SV.solve(op, prob.b.astype(np.float64), mode=SV.FPCG,
                               tol=results["fp16_kp_fpcg"]["tol"], maxit=1000, precond=pre)
                count += 1
                cpu_s = time.time() - t0
                if cpu_s >= CPU_SAMPLE_S or count >= CPU_SAMPLE_MAX:
                    break
        cpu_err = float(np.linalg.norm(out.x - xlam) / np.linalg.norm(xlam))
        cpu_baseline = {
            "value": count / cpu_s, "unit": "solves/s", "cores": nthreads, "kind": "oracle",
            "sample": (f"{count} FP64 KP-preconditioned flexible-PCG solves of the same 1024^2 "
                       f"problem (tol {results['fp16_kp_fpcg']['tol']:.0e}, {out.iters} "
                       f"iterations each, rel err {cpu_err:.1e}; scipy.fft matvecs, numpy BLAS "
                       f"GEMMs, {cpu_s:.1f} s)"),
        }
        log(f"[bench] cpu oracle: {count} solves in {cpu_s:.2f}s iters={out.iters}")

    batch = run_batch(args.batch, dev) if args.batch else None
    lowp = None
    if not args.profile_only:
        lowp = run_lowp_setup(prob, b, lam, results["fp16_kp_fpcg"]["tol"], xlam, setup_s)
    instances = None
    if args.instances and not args.profile_only:
        instances = run_instances(args.instances, grid, ladder, args.steps, args.warmup, dev,
                                  nthreads)
    periodic = reflexive = None
    if not args.profile_only and not args.no_periodic:
        periodic = run_boundary("periodic", args.seed, grid, ladder, dev)
        reflexive = run_boundary("reflexive", args.seed, grid, ladder, dev)

    head = results["fp16_kp_fpcg"]
    line = {
        "metric": METRIC,
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 vectors+matvec, f16 MFMA preconditioner, f64 scalars",
        "data": "synthetic",
        "config": {
            "workload": ("deblur 1024x1024, Moffat(beta=2.5)+motion PSF 63x63, zero BC, "
                         "2% noise, lambda by KP-GCV (32-pt grid), FP16-KP flexible PCG"),
            "n": n, "k": k, "seed": args.seed, "lambda": lam, "gcv_grid_index": gidx,
            "parallelism": "single GPU",
            "modes": results,
            "setup_s": setup_s, "gcv_ms": gcv_ms,
            "kp_rel_error": pinfo["kp_rel_error"],
            "blur_tile_config": pinfo["blur_config"],
            "precond_fp16_chain_us": prec_ms * 1e3,
            "learned_lambda": learned,
            "batched": batch,
            "periodic": periodic,
            "reflexive": reflexive,
            "instances": instances,
            "lowp_setup": lowp,
        },
        "roofline": roofline,
        "cpu_baseline": cpu_baseline,
    }
    print(json.dumps(line), flush=True)
    plan.close()


def time_learned_lambda(plan, b, grid, dev) -> dict:
    """Cost of the learned-lambda path (network kernels with untrained
    weights: the timing does not depend on the weights): features +
    prediction + GCV check for one image, batched inference, and one Adam
    training step on 256 rows."""
    import torch
    from paper_2311_15393_amd import Mlp
    from paper_2311_15393_amd.lambda_net import init_params
    mlp = Mlp(max_batch=4096)
    mlp.set_params(init_params(0))
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    feats = torch.randn((4096, 128), device=dev, generator=g)
    tgt = torch.randn(4096, device=dev, generator=g)
    mlp.fit_normalizer(feats)
    out = torch.empty(4096, device=dev, dtype=torch.float64)
    plan.lambda_learned(mlp, b, grid, tau=0.1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        plan.lambda_learned(mlp, b, grid, tau=0.1)
    ll_ms = (time.perf_counter() - t0) / 5 * 1e3
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    mlp.predict(feats, out=out)
    e0.record(s)
    for _ in range(20):
        mlp.predict(feats, out=out)
    e1.record(s)
    e1.synchronize()
    pred_ms = e0.elapsed_time(e1) / 20
    rows = np.arange(256, dtype=np.int32)
    mlp.train_step(feats, tgt, 1e-4, rows=rows)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(50):
        mlp.train_step(feats, tgt, 1e-4, rows=rows)
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) / 50 * 1e3
    mlp.close()
    return {"lambda_learned_ms": ll_ms, "predict_rows": 4096, "predict_ms": pred_ms,
            "predict_samples_per_s": 4096 / (pred_ms * 1e-3),
            "train_step_ms": step_ms, "train_samples_per_s": 256 / (step_ms * 1e-3)}


def run_lowp_setup(prob, b, lam: float, tol: float, xlam, setup64_s: float):
    """The reduced-precision construction (KP_SETUP_LOWP: factors rounded to
    FP16, FP32 SVDs) on the large workload: kp_setup time against the FP64
    construction's, and the FP16-KP FPCG solve at the headline tolerance
    with it (iterations, error against x_lambda, 5 timed solves)."""
    import torch
    from paper_2311_15393_amd import KP_FPCG, KP_OK, KP_P16, KP_SETUP_LOWP, Plan
    torch.cuda.synchronize()
    t0 = time.time()
    plan = Plan(prob.psf, prob.n, bc=KP_SETUP_LOWP)
    torch.cuda.synchronize()
    setup_s = time.time() - t0

    def run():
        x = torch.empty_like(b)
        return plan.solve(b, lam, tol=tol, maxit=200, mode=KP_FPCG | KP_P16, x=x,
                          raise_on_fail=False)

    x, info = run()
    err = float(np.linalg.norm(x.cpu().numpy().astype(np.float64) - xlam) / np.linalg.norm(xlam))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / 5 * 1e3
    plan.close()
    log(f"[bench] lowp setup: {setup_s:.3f}s (FP64 construction {setup64_s:.3f}s); FP16 solve "
        f"iters={info.iters} err={err:.2e} {ms:.3f} ms/solve")
    return {"setup_s": setup_s, "setup_fp64_s": setup64_s, "tol": tol, "iters": info.iters,
            "rel_err": err, "ok": bool(info.status == KP_OK and err <= 1e-4),
            "ms_per_solve": ms}


def run_boundary(kind: str, seed: int, grid, ladder, dev):
    """The large workload under another boundary: periodic (KP_BC_PERIODIC,
    the same image and PSF draws with periodic data, x_lambda by the 2-D DFT)
    or reflexive (KP_BC_REFLEXIVE, the radial Moffat of the same draw, which
    is symmetric in both axes, with reflexive data, x_lambda by the 2-D DCT).
    Lambda by the device's KP-GCV, FP16-KP flexible PCG at the loosest
    ladder tolerance whose x meets 1e-4 against the FP64 closed form, then 5
    timed solves and the blur's launch time."""
    import torch
    import synthetic as S
    from paper_2311_15393_amd import KP_BC_PERIODIC, KP_BC_REFLEXIVE, KP_FPCG, KP_OK, KP_P16, Plan
    if kind == "periodic":
        from oracle import periodic as ref
        prob, bc = S.large_moffat_periodic(seed), KP_BC_PERIODIC
        what = "Moffat(beta=2.5)+motion PSF 63x63, periodic BC"
    else:
        from oracle import reflexive as ref
        prob, bc = S.large_moffat_reflexive(seed), KP_BC_REFLEXIVE
        what = "radial Moffat(beta=2.5) PSF 63x63, reflexive BC"
    n = prob.n
    b = torch.from_numpy(prob.b).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    plan = Plan(prob.psf, n, bc=bc)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    info0 = plan.query()
    lam, _ = plan.gcv(b, grid)
    gidx = int(np.argmin(np.abs(grid - lam)))
    xlam = ref.x_lambda(prob.psf, prob.b.astype(np.float64), lam)
    mode = KP_FPCG | KP_P16

    def run(tol):
        x = torch.empty_like(b)
        return plan.solve(b, lam, tol=tol, maxit=200, mode=mode, x=x, raise_on_fail=False)

    for tol in ladder:
        x, info = run(tol)
        err = float(np.linalg.norm(x.cpu().numpy().astype(np.float64) - xlam)
                    / np.linalg.norm(xlam))
        if info.status == KP_OK and err <= 1e-4:
            break
    run(tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        run(tol)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / 5 * 1e3
    p = torch.randn((n, n), device=dev, dtype=torch.float32)
    q = torch.empty_like(p)
    plan.time_blur(p, q, reps=3)
    blur_us = plan.time_blur(p, q, reps=20) * 1e3
    plan.close()
    log(f"[bench] {kind}: lambda={lam:.4g} tol={tol:.0e} iters={info.iters} err={err:.2e} "
        f"{ms:.3f} ms/solve; blur {blur_us:.1f} us; setup {setup_s:.2f}s")
    return {"workload": (f"deblur 1024x1024, {what}, 2% noise, lambda by KP-GCV (32-pt grid), "
                         "FP16-KP flexible PCG"),
            "lambda": lam, "gcv_grid_index": gidx, "tol": tol, "iters": info.iters,
            "rel_err": err, "ok": bool(info.status == KP_OK and err <= 1e-4),
            "ms_per_solve": ms, "solves_per_s": 1e3 / ms, "setup_s": setup_s,
            "kp_rel_error": info0["kp_rel_error"], "blur_config": info0["blur_config"],
            "blur_us": blur_us}


def run_instances(count: int, grid, ladder, steps: int, warmup: int, dev, nthreads: int):
    """The headline FP16-KP FPCG solve on seeds 0 .. count-1 of the large
    workload, each with its own image, Moffat + motion PSF and noise: the
    device's KP-GCV grid index must equal the oracle's, the tolerance is the
    loosest ladder value whose x meets 1e-4 against the oracle's x_lambda,
    then `warmup` untimed and `steps` timed solves."""
    import torch
    from threadpoolctl import threadpool_limits
    import synthetic as S
    from oracle import kp as KP
    from oracle import lam as L
    from oracle import solvers as SV
    from paper_2311_15393_amd import KP_FPCG, KP_OK, KP_P16, Plan
    rows = []
    for seed in range(count):
        prob = S.large_moffat(seed)
        n = prob.n
        b = torch.from_numpy(prob.b).to(dev)
        plan = Plan(prob.psf, n)
        lam, _ = plan.gcv(b, grid)
        gidx = int(np.argmin(np.abs(grid - lam)))
        with threadpool_limits(limits=nthreads):
            kp = KP.kp_svd(prob.psf, n)
            s2, bh2 = L.spectrum(kp, prob.b.astype(np.float64))
            ref_idx = L.grid_argmin(L.gcv(s2, bh2, grid))
            xlam, _ = settled_x_lambda(SV, prob, lam, kp, nthreads)
        x = torch.empty_like(b)
        for tol in ladder:
            _, info = plan.solve(b, lam, tol=tol, maxit=200, mode=KP_FPCG | KP_P16, x=x,
                                 raise_on_fail=False)
            err = float(np.linalg.norm(x.cpu().numpy().astype(np.float64) - xlam)
                        / np.linalg.norm(xlam))
            if info.status == KP_OK and err <= 1e-4:
                break
        for _ in range(warmup):
            plan.solve(b, lam, tol=tol, maxit=200, mode=KP_FPCG | KP_P16, x=x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.solve(b, lam, tol=tol, maxit=200, mode=KP_FPCG | KP_P16, x=x)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        plan.close()
        row = {"seed": seed, "lambda": lam, "gcv_grid_index": gidx,
               "oracle_gcv_grid_index": ref_idx, "tol": tol, "iters": info.iters,
               "rel_err": err, "ok": bool(info.status == KP_OK and err <= 1e-4
                                          and gidx == ref_idx),
               "ms_per_solve": ms, "solves_per_s": 1e3 / ms}
        log(f"[bench] instance seed {seed}: lambda={lam:.4g} (index {gidx}, oracle {ref_idx}) "
            f"tol={tol:.0e} iters={info.iters} err={err:.2e} {ms:.3f} ms/solve")
        rows.append(row)
    sps = [r["solves_per_s"] for r in rows]
    return {"rows": rows, "median_solves_per_s": float(np.median(sps)),
            "all_ok": all(r["ok"] for r in rows)}


def psf_spectrum(psf: np.ndarray, L: int, dev):
    """rfft2 of the PSF zero-padded to L x L (FP32, on dev)."""
    import torch
    k = psf.shape[0]
    pt = torch.zeros((L, L), device=dev, dtype=torch.float32)
    pt[:k, :k] = torch.from_numpy(np.ascontiguousarray(psf, dtype=np.float32)).to(dev)
    return torch.fft.rfft2(pt)


def fft_normal(p, pf, pfc, L: int, h: int):
    """A^T A p (zero boundary, centre (h, h)) by zero-padded FFTs of size L:
    entries h .. h + n - 1 of the linear convolution are A p, and the
    circular correlation with the PSF, shifted by h, is A^T y.  Wrapped taps
    land in the zero pad once L >= n + h.  pf, pfc: psf_spectrum and its
    conjugate."""
    import torch
    n = p.shape[0]
    y = torch.fft.irfft2(torch.fft.rfft2(p, s=(L, L)) * pf, s=(L, L))[h:h + n, h:h + n]
    c = torch.fft.irfft2(torch.fft.rfft2(y, s=(L, L)) * pfc, s=(L, L))
    return torch.roll(c, shifts=(h, h), dims=(0, 1))[:n, :n]


def smooth_size(m: int) -> int:
    """Smallest L >= m whose prime factors are all 2, 3, 5 or 7."""
    L = m
    while True:
        r = L
        for f in (2, 3, 5, 7):
            while r % f == 0:
                r //= f
        if r == 1:
            return L
        L += 1


def run_matvec_sweep(dev, n: int = 1024, ks=(15, 23, 31, 47, 63), reps: int = 50):
    """The matvec's two forms at n^2 over the PSF width K (zero boundary):
    the direct blurs the solver runs (A p and A^T y, each on the plan's
    autotuned kernel) against H p = A^T A p by zero-padded FFTs (torch.fft,
    i.e. rocFFT, FP32): p -> A p needs one forward and one inverse
    transform, the crop to n x n, and A^T y two more.  With circular
    indices every wrapped tap lands in the zero pad once L >= n + h, so L is
    the smallest 7-smooth size at or above n + h (a power of two is also
    timed).  The FFT result is checked against the library's FP64 normal
    operator."""
    import torch
    import synthetic as S
    from paper_2311_15393_amd import Plan

    def ev_time(fn, reps):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    p = torch.randn((n, n), device=dev, dtype=torch.float32)
    q = torch.empty_like(p)
    out = []
    for k in ks:
        h = (k - 1) // 2
        psf = S.psf_moffat_motion(k, 5.5, 2.5, 6.0, 0.7)
        plan = Plan(psf, n)
        plan.time_blur(p, q, reps=3)
        fwd_us = plan.time_blur(p, q, reps=reps) * 1e3
        plan.time_blur(p, q, transpose=True, reps=3)
        adj_us = plan.time_blur(p, q, transpose=True, reps=reps) * 1e3
        ref = torch.empty((n, n), device=dev, dtype=torch.float64)
        plan.normal_fp64(p, 0.0, ref)
        torch.cuda.synchronize()
        cfg = plan.query()["blur_config"]
        plan.close()
        row = {"k": k, "blur_config": cfg, "direct_fwd_us": fwd_us, "direct_adj_us": adj_us,
               "direct_hp_us": fwd_us + adj_us}
        for tag, L in (("smooth", smooth_size(n + h)), ("pow2", 1 << (n + h - 1).bit_length())):
            pf = psf_spectrum(psf, L, dev)
            pfc = pf.conj()

            def hp():
                return fft_normal(p, pf, pfc, L, h)

            got = hp().double()
            err = float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref))
            hp_us = ev_time(hp, reps)
            x = torch.randn((n, n), device=dev)
            rfft_us = ev_time(lambda: torch.fft.rfft2(x, s=(L, L)), reps)
            row[f"fft_{tag}"] = {"L": L, "hp_us": hp_us, "rfft2_us": rfft_us, "rel_err": err}
        log(f"[sweep] K={k}: direct A p {fwd_us:.1f} + A^T y {adj_us:.1f} us (cfg {cfg}); "
            f"FFT H p L={row['fft_smooth']['L']} {row['fft_smooth']['hp_us']:.1f} us "
            f"(rfft2 {row['fft_smooth']['rfft2_us']:.1f}, err {row['fft_smooth']['rel_err']:.1e}), "
            f"L={row['fft_pow2']['L']} {row['fft_pow2']['hp_us']:.1f} us")
        out.append(row)
    return {"matvec_sweep": {"n": n, "boundary": "zero", "rows": out}}


def run_batch(nprob: int, dev):
    """Uneven batch: problems of sizes {128,...,1024}, supports 15..63, each
    with 16 lambda values log-spaced over lambda_gcv * 10^[-1.5, 1.5] (KP-GCV
    on the 32-point grid picks lambda_gcv), all solved by one batched FP16
    FPCG call; the sweep is scored by KP-GCV and by the discrepancy principle
    on the solves' actual misfits."""
    import torch
    import synthetic as S
    from paper_2311_15393_amd import KP_EXACT_DIAG, KP_FPCG, KP_OK, KP_P16, Plan, solve_batched

    t0 = time.time()
    probs = [S.batch_problem(i) for i in range(nprob)]
    gen_s = time.time() - t0
    t0 = time.time()
    plans = [Plan(p.psf, p.n) for p in probs]
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    grid = S.lambda_grid()
    bs_dev = [torch.from_numpy(p.b).to(dev) for p in probs]
    items, sweeps = [], []
    for pi, (p, plan) in enumerate(zip(probs, plans)):
        lam_g, _ = plan.gcv(bs_dev[pi], grid)
        sweep = np.clip(lam_g * 10.0 ** np.linspace(-1.5, 1.5, 16), 1e-4, 1.0)
        sweeps.append(sweep)
        items += [(pi, float(l)) for l in sweep]
    bs = [bs_dev[pi] for pi, _ in items]
    lams = [l for _, l in items]
    poi = [pi for pi, _ in items]
    log(f"[bench] batch: {nprob} problems x 16 lambda = {len(items)} solves, "
        f"{sum(p.n * p.n for p in probs) * 16 / 1e6:.1f} Mpx; setup {setup_s:.1f}s")
    xs = [torch.empty_like(b) for b in bs]
    solve_batched(plans, bs, lams, poi, tol=1e-6, maxit=1000, mode=KP_FPCG | KP_P16, xs=xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, infos, st = solve_batched(plans, bs, lams, poi, tol=1e-6, maxit=1000,
                                  mode=KP_FPCG | KP_P16, xs=xs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iters = np.array([i.iters for i in infos])
    ok = sum(i.status == KP_OK for i in infos)
    # score each problem's sweep: KP-GCV (16 points) and discrepancy on misfits
    errs_gcv, errs_dp = [], []
    for pi, (p, plan) in enumerate(zip(probs, plans)):
        sweep = sweeps[pi]
        _, g = plan.gcv(bs_dev[pi], sweep)
        idx = [k for k, (q, _) in enumerate(items) if q == pi]
        mis = np.array([infos[k].misfit for k in idx])
        d = mis ** 2 - p.noise_norm ** 2
        below = np.nonzero(d <= 0)[0]
        k_dp = int(below[-1]) if below.size else 0
        k_gcv = int(np.argmin(g))
        xt = p.x_true
        for kk, store in ((k_gcv, errs_gcv), (k_dp, errs_dp)):
            x = xs[idx[kk]].cpu().numpy().astype(np.float64)
            store.append(float(np.linalg.norm(x - xt) / np.linalg.norm(xt)))
    # the same batch with the exact KP-basis diagonal in the preconditioner
    xs2 = [torch.empty_like(b) for b in bs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, infos2, _ = solve_batched(plans, bs, lams, poi, tol=1e-6, maxit=1000,
                                 mode=KP_FPCG | KP_P16 | KP_EXACT_DIAG, xs=xs2)
    torch.cuda.synchronize()
    wall2 = time.perf_counter() - t0
    iters2 = np.array([i.iters for i in infos2])
    ok2 = sum(i.status == KP_OK for i in infos2)
    log(f"[bench] batch, exact diagonal: {wall2:.3f}s ({len(items) / wall2:.1f}/s), converged "
        f"{ok2}, iters mean {iters2.mean():.1f} max {iters2.max()}")
    out = {
        "problems": nprob, "solves": len(items), "wall_s": wall,
        "solves_per_s": len(items) / wall, "converged": ok,
        "iters_mean": float(iters.mean()), "iters_max": int(iters.max()),
        "setup_s_total": setup_s, "tol": 1e-6, "mode": "fp16_kp_fpcg",
        "err_vs_true_gcv_pick_mean": float(np.mean(errs_gcv)),
        "err_vs_true_dp_pick_mean": float(np.mean(errs_dp)),
        "exact_diag": {"wall_s": wall2, "solves_per_s": len(items) / wall2, "converged": ok2,
                       "iters_mean": float(iters2.mean()), "iters_max": int(iters2.max())},
    }
    log(f"[bench] batch: {wall:.3f}s for {len(items)} solves ({len(items) / wall:.1f}/s), "
        f"converged {ok}, iters mean {iters.mean():.1f} max {iters.max()}; "
        f"error vs x_true at GCV pick {np.mean(errs_gcv):.3f}, DP pick {np.mean(errs_dp):.3f}")
    for pl in plans:
        pl.close()
    return out


if __name__ == "__main__":
    main()
