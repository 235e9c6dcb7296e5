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


# HBM bandwidth of the two vector steps of an iteration on a working set far
# above the 256 MB Infinity Cache: the batched update (x += alpha p in FP64,
# r -= alpha w, ||r||^2 partials: 32 B per element) and direction update
# (p = z + beta p: 12 B per element) over 16 items of 1024^2 (one lambda sweep
# of the large workload; ~1 GiB of item vectors), from
# `rocprofv3 --kernel-trace --stats -- python3 bench.py --vector-batch` (mean
# duration of the launches over all 16 items) and two --pmc runs of the same
# command (FETCH_SIZE, WRITE_SIZE, scaled by the calibration copy it
# launches).  Null when the batched kernels' source differs from the one
# measured (sha256 of batch.hip).
VECTOR_KERNELS = {
    "workload": "16 items of 1024^2 (~1 GiB of item vectors), profiles/vector_kernels_batch16_1024_hbm.md",
    "update": {"kernel": "vec_batched_kernel<0>", "avg_us": 83.24, "bytes_per_launch": 536870912,
               "achieved_TBps": 6.450, "frac_of_8TBps": 0.806,
               "traffic": {"fetch_bytes": 336246474, "write_bytes": 202213344}},
    "pupdate": {"kernel": "vec_batched_kernel<1>", "avg_us": 35.75, "bytes_per_launch": 201326592,
                "achieved_TBps": 5.632, "frac_of_8TBps": 0.704,
                "traffic": {"fetch_bytes": 134845617, "write_bytes": 67108864}},
    "sources_sha256": "d8fca763271cf33e80eff01f5104fb099d6a1429e3f0db134c5cf7e616a19724",
}


# HBM traffic of one H p by FFTs (the five passes: rows_fwd, cols, rows_mid,
# cols, rows_out) at the 1024^2, K=63 workload, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE) of `python bench.py --profile-only --modes
# fp16_kp_fpcg --steps 2 --warmup 1`, the mean per launch of each pass scaled
# by the calibration copy, summed over the passes of one H p.  The unit is
# the plain H p that kp_time_normal times (in that run's solves the profiler's
# per-launch cost makes the setup pick the direct form, so the FFT launches
# counted are the timing and autotuning ones).  Null when the FFT source
# differs from the one measured (sha256 of fft.hip) or the plan's transform
# length differs.
FFT_TRAFFIC = {
    "fft_length": 1080,
    # per launch of each pass, as counted
    "fetch_kib_raw": {"rows_fwd": 2147.6, "cols": 4611.4, "rows_mid": 2279.0, "rows_out": 4323.5},
    "write_kib_raw": {"rows_fwd": 4395.5, "cols": 4328.0, "rows_mid": 4395.5, "rows_out": 4098.0},
    "fetch_scale": 1.99980, "write_scale": 1.0,              # copy bytes / counter
    "bytes_per_unit": 58866873,                               # one H p (two column passes)
    "sources_sha256": "ff14c3948e211595118c07693ceac7577a3244fc8d8f3c9b2b04bcdf794797ae",
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


def batch_sources_sha256() -> str:
    import hashlib
    with open(os.path.join(ROOT, "paper_2311_15393_amd", "csrc", "batch.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def vector_kernels():
    """The recorded bandwidth of the batched vector steps, or None when the
    batched kernels' source has changed since it was measured."""
    if VECTOR_KERNELS is None or VECTOR_KERNELS["sources_sha256"] != batch_sources_sha256():
        return None
    return {k: v for k, v in VECTOR_KERNELS.items() if k != "sources_sha256"}


def blur_traffic(kernel: str):
    """Counter-measured HBM bytes per forward-blur launch of `kernel`, or None
    when no measurement exists for it and the current blur sources."""
    if (BLUR_TRAFFIC is None or BLUR_TRAFFIC["kernel"] != kernel
            or BLUR_TRAFFIC["sources_sha256"] != blur_sources_sha256()):
        return None
    return BLUR_TRAFFIC["bytes_per_launch"]


def fft_sources_sha256() -> str:
    import hashlib
    with open(os.path.join(ROOT, "paper_2311_15393_amd", "csrc", "fft.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def fft_normal_bytes(n: int, L: int) -> int:
    """Algorithmic HBM bytes of one H p by the five FFT passes: p read twice
    and w written (FP32 n x n), the half spectra (F = L/2 + 1 frequencies of
    n rows, FP32 complex) written by four passes and read by four, and the
    PSF spectrum (F x L complex) read by both column passes."""
    F = L // 2 + 1
    return 3 * 4 * n * n + 8 * 8 * F * n + 2 * 8 * F * L


def fft_traffic(L: int):
    """Counter-measured HBM bytes per H p by FFTs at this length, or None."""
    if (FFT_TRAFFIC is None or FFT_TRAFFIC["fft_length"] != L
            or FFT_TRAFFIC["sources_sha256"] != fft_sources_sha256()):
        return None
    return FFT_TRAFFIC["bytes_per_unit"]


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


MODE_LABELS = {"fp16_kp_fpcg": "FP16-KP flexible PCG", "fp32_kp_pcg": "FP32-KP PCG",
               "fp8_kp_fpcg": "FP8-KP flexible PCG", "none_cg": "CG (no preconditioner)",
               "fp16_kpdiag_fpcg": "FP16-KP flexible PCG, exact KP-basis diagonal",
               "fp32_kpdiag_pcg": "FP32-KP PCG, exact KP-basis diagonal"}


def mode_bits_table():
    from paper_2311_15393_amd import KP_CG, KP_EXACT_DIAG, KP_FPCG, KP_P8, KP_P16, KP_P32, KP_PCG
    return {"fp16_kp_fpcg": KP_FPCG | KP_P16, "fp32_kp_pcg": KP_PCG | KP_P32,
            "fp8_kp_fpcg": KP_FPCG | KP_P8, "none_cg": KP_CG,
            "fp16_kpdiag_fpcg": KP_FPCG | KP_P16 | KP_EXACT_DIAG,
            "fp32_kpdiag_pcg": KP_PCG | KP_P32 | KP_EXACT_DIAG}


# tolerance ladder: 1e-5, 5e-6, 2e-6, 1e-6, 5e-7, ... down to 1e-9
LADDER = [m * 10.0 ** e for e in range(-5, -10, -1) for m in (1.0, 0.5, 0.2)] + [1e-9]


def time_solves(run, steps: int, warmup: int):
    """`warmup` untimed solves, then exactly `steps` timed ones, each from b
    resident in HBM to x resident in HBM (pcg_solve returns after its stream
    has drained); the device is synchronised on both sides of the timed
    region.  Returns the per-solve wall times (ms) and the last info."""
    import torch
    info = None
    for _ in range(warmup):
        _, info = run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        _, info = run()
        ts.append((time.perf_counter() - t0) * 1e3)
    torch.cuda.synchronize()
    return ts, info


def run_instance(seed: int, modes, args, grid, dev, nthreads: int, keep: bool):
    """One instance of the large workload (its own image, Moffat + motion
    PSF and noise): lambda by the device's KP-GCV (its grid index must equal
    the oracle's), the oracle's settled x_lambda, then per mode the loosest
    ladder tolerance whose x is within 1e-4 of x_lambda and `steps` timed
    solves (per-solve median)."""
    import torch
    import synthetic as S
    from paper_2311_15393_amd import KP_NORMAL_DIRECT, KP_NORMAL_FFT, KP_OK, Plan
    t0 = time.time()
    prob = S.large_moffat(seed)
    n = prob.n
    b = torch.from_numpy(prob.b).to(dev)
    torch.cuda.synchronize()
    t1 = time.time()
    plan = Plan(prob.psf, n)
    torch.cuda.synchronize()
    setup_s = time.time() - t1
    if args.normal_op != "auto":
        # a profiler's per-launch overhead can tip the setup's choice between
        # the two forms: profiling runs name the one the plain run picks
        plan.set_normal_op(KP_NORMAL_FFT if args.normal_op == "fft" else KP_NORMAL_DIRECT)
    pinfo = plan.query()
    lam, _ = plan.gcv(b, grid)
    gidx = int(np.argmin(np.abs(grid - lam)))
    out = {"seed": seed, "lambda": lam, "gcv_grid_index": gidx, "setup_s": setup_s,
           "kp_rel_error": pinfo["kp_rel_error"], "blur_config": pinfo["blur_config"],
           "normal_op": pinfo["normal_op"], "modes": {}}
    xlam = kp = None
    if not args.profile_only:
        from threadpoolctl import threadpool_limits
        from oracle import kp as KP
        from oracle import lam as L
        from oracle import solvers as SV
        with threadpool_limits(limits=nthreads):
            kp = KP.kp_svd(prob.psf, n)
            s2, bh2 = L.spectrum(kp, prob.b.astype(np.float64))
            ref_idx = L.grid_argmin(L.gcv(s2, bh2, grid))
            xlam, xinfo = settled_x_lambda(SV, prob, lam, kp, nthreads)
        out["oracle_gcv_grid_index"] = ref_idx
        out["x_lambda_oracle"] = {"iters": xinfo["iters"], "true_relres": xinfo["true_relres"],
                                  "loose_agreement": xinfo["loose_agreement"]}
    log(f"[bench] seed {seed}: setup {setup_s:.2f}s lambda={lam:.4g} (index {gidx}, oracle "
        f"{out.get('oracle_gcv_grid_index')}) normal op {pinfo['normal_op']} "
        f"({time.time() - t0:.1f}s with the oracle)")
    bits = mode_bits_table()

    def run(mode, tol, maxit):
        x = torch.empty_like(b)
        return plan.solve(b, lam, tol=tol, maxit=maxit, mode=mode, x=x, raise_on_fail=False)

    for name in modes:
        mode, maxit = bits[name], MODES[name]
        if args.profile_only:
            tol = PROFILE_TOLS[name]
            _, info = run(mode, tol, maxit)
            err = float("nan")
        else:
            for tol in LADDER:
                x, info = run(mode, tol, maxit)
                err = float(np.linalg.norm(x.cpu().numpy().astype(np.float64) - xlam)
                            / np.linalg.norm(xlam))
                if info.status == KP_OK and err <= 1e-4:
                    break
        steps = args.steps if name == "fp16_kp_fpcg" else max(1, min(args.steps, 5))
        warm = args.warmup if name == "fp16_kp_fpcg" else 1
        ts, info2 = time_solves(lambda: run(mode, tol, maxit), steps, warm)
        ok = bool(info.status == KP_OK and (args.profile_only or err <= 1e-4)
                  and (args.profile_only or gidx == out["oracle_gcv_grid_index"]))
        out["modes"][name] = {"tol": tol, "iters": info.iters, "rel_err": err,
                              "ms_median": float(np.median(ts)), "ms_mean": float(np.mean(ts)),
                              "ms_min": float(np.min(ts)), "ok": ok}
        log(f"[bench]   {name}: tol={tol:.0e} iters={info.iters} err={err:.2e} "
            f"median {np.median(ts):.3f} ms/solve (min {np.min(ts):.3f})")
    if keep:
        return out, {"prob": prob, "b": b, "plan": plan, "lam": lam, "xlam": xlam, "kp": kp,
                     "pinfo": pinfo, "gidx": gidx, "setup_s": setup_s}
    plan.close()
    return out, None


def cpu_description() -> dict:
    """The host the CPU baseline ran on: core counts, CPU model, the BLAS
    numpy uses (threadpoolctl) and the thread variables."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        info["blas"] = [{k: d.get(k) for k in ("internal_api", "version", "num_threads",
                                                 "threading_layer")}
                        for d in threadpool_info() if d.get("user_api") == "blas"]
    except Exception:
        pass
    info["thread_env"] = {k: os.environ[k] for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                                      "MKL_NUM_THREADS") if k in os.environ}
    return info


def matvec_label(pinfo) -> str:
    if pinfo.get("normal_op") == 1:
        return ("A^T A p by FP32 zero-padded FFTs (A^T b and the true residuals on the "
                + ("MFMA blur, FP16 hi/lo split" if pinfo["blur_config"] in (6, 7)
                   else "FP32 VALU blur") + ")")
    if pinfo["blur_config"] in (6, 7):
        return "A p and A^T q on MFMA, FP16 hi/lo split (3 products, ~22-bit)"
    return "A p and A^T q on FP32 VALU"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0, help="first seed of the instances")
    ap.add_argument("--instances", type=int, default=8, metavar="S",
                    help="seeds seed .. seed+S-1 of the large workload; the headline is the "
                         "median over them")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--normal-op", choices=("auto", "direct", "fft"), default="auto",
                    help="form of H p in the solves (default: the setup's autotuned choice)")
    ap.add_argument("--profile-only", action="store_true",
                    help="skip the oracle parts (for profiler runs)")
    ap.add_argument("--no-periodic", action="store_true",
                    help="skip the periodic- and reflexive-boundary solves (also skipped with "
                         "--profile-only)")
    ap.add_argument("--batch", type=int, default=64, metavar="P",
                    help="the uneven batched workload with P problems x 16 lambda (0: skip)")
    ap.add_argument("--vector-batch", action="store_true",
                    help="only run one 16-lambda batch of the 1024^2 workload for 40 iterations "
                         "(and the counter calibration copy), for profiling the batched vector "
                         "kernels on a working set above the Infinity Cache")
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
    from paper_2311_15393_amd import KP_P16

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    nthreads = cpu_threads()
    if args.matvec_sweep:
        print(json.dumps(run_matvec_sweep(dev)), flush=True)
        return
    if args.vector_batch:
        print(json.dumps(run_vector_batch(dev)), flush=True)
        return
    grid = S.lambda_grid()
    chosen = [m for m in args.modes.split(",") if m]
    assert "fp16_kp_fpcg" in chosen and all(m in MODES for m in chosen), args.modes

    # ---- the headline: every mode on each instance, median over instances
    rows, first = [], None
    for i in range(max(1, args.instances)):
        row, kept = run_instance(args.seed + i, chosen, args, grid, dev, nthreads, keep=(i == 0))
        rows.append(row)
        if kept is not None:
            first = kept
    summary = {}
    for name in chosen:
        ms = [r["modes"][name]["ms_median"] for r in rows]
        summary[name] = {
            "label": MODE_LABELS[name],
            "ms_median_over_instances": float(np.median(ms)),
            "solves_per_s": 1e3 / float(np.median(ms)),
            "ms_per_instance": ms,
            "iters_per_instance": [r["modes"][name]["iters"] for r in rows],
            "tol_per_instance": [r["modes"][name]["tol"] for r in rows],
            "rel_err_per_instance": [r["modes"][name]["rel_err"] for r in rows],
            "all_ok": all(r["modes"][name]["ok"] for r in rows),
        }
        log(f"[bench] {name}: median {np.median(ms):.3f} ms over {len(rows)} instances "
            f"({1e3 / np.median(ms):.1f} solves/s), all ok {summary[name]['all_ok']}")
    head = summary["fp16_kp_fpcg"]

    # ---- the paper's break-even (Section 5.2): preconditioning pays iff
    # m_P t_P < m_N t_N, i.e. m_P / m_N < t_N / t_P with t the time of one
    # iteration of each method, here measured per instance
    break_even = None
    if "none_cg" in chosen:
        per = []
        for r in rows:
            mp, mn = r["modes"]["fp16_kp_fpcg"]["iters"], r["modes"]["none_cg"]["iters"]
            tp = r["modes"]["fp16_kp_fpcg"]["ms_median"] / max(mp, 1)
            tn = r["modes"]["none_cg"]["ms_median"] / max(mn, 1)
            per.append({"seed": r["seed"], "m_P": mp, "m_N": mn, "mP_over_mN": mp / max(mn, 1),
                        "t_P_ms": tp, "t_N_ms": tn, "tN_over_tP": tn / tp,
                        "pays": bool(mp * tp < mn * tn)})
        break_even = {"preconditioner": "FP16-KP", "rows": per,
                      "paper_model_bound": 8.0 / 9.0,
                      "note": "m_P/m_N against the measured per-iteration cost ratio t_N/t_P "
                              "(solve time / iterations, including true-residual work)"}

    # ---- seed 0 extras: GCV timing, learned lambda, kernels, CPU baseline
    prob, b, plan, lam = first["prob"], first["b"], first["plan"], first["lam"]
    xlam, kp, pinfo = first["xlam"], first["kp"], first["pinfo"]
    n, k = prob.n, prob.k
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        plan.gcv(b, grid)
    torch.cuda.synchronize()
    gcv_ms = (time.perf_counter() - t0) / 5 * 1e3
    learned = time_learned_lambda(plan, b, grid, dev)
    log(f"[bench] learned lambda: kp_lambda_learned {learned['lambda_learned_ms']:.2f} ms at "
        f"{n}^2; lambda_predict {learned['predict_samples_per_s'] / 1e6:.2f} M rows/s; "
        f"train step (256 rows) {learned['train_step_ms']:.3f} ms")

    # dominant kernel: the blur matvec (two per iteration), as autotuned
    p = torch.randn((n, n), device=dev, dtype=torch.float32)
    q = torch.empty_like(p)
    plan.time_blur(p, q, reps=3)
    blur_ms = plan.time_blur(p, q, transpose=False, reps=20)
    flops = blur_flops(n, k)
    achieved = flops / (blur_ms * 1e-3)
    prec_ms = plan.time_precond(p, lam, KP_P16, q, reps=20)
    prec_flops = 8.0 * n ** 3
    normal_ms = {op: plan.time_normal(p, q, op, reps=20) for op in (0, 1)}
    log(f"[bench] blur kernel {blur_ms * 1e3:.1f} us ({achieved / 1e12:.2f} TFLOP/s); "
        f"FP16 preconditioner chain {prec_ms * 1e3:.1f} us "
        f"({prec_flops / (prec_ms * 1e-3) / 1e12:.1f} TFLOP/s); H p direct "
        f"{normal_ms[0] * 1e3:.1f} us, FFT {normal_ms[1] * 1e3:.1f} us")

    if args.profile_only:
        # plain copy of known size for the counter calibration
        src = torch.ones(COPY_CALIB_FLOATS, device=dev, dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    blur_entry = None
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
    if pinfo["normal_op"] == 1:
        # the iterations' H p runs as the five FFT passes: that unit is the
        # dominant work of an iteration; the blur (right-hand side and true
        # residuals) is kept beside it
        blur_entry = roofline
        L = pinfo["fft_length"]
        fft_s = normal_ms[1] * 1e-3
        fbytes = fft_normal_bytes(n, L)
        roofline = {
            "bound": "hbm", "achieved": fbytes / fft_s / 1e9, "peak": HBM_PEAK / 1e9,
            "unit": "GB/s", "frac": fbytes / fft_s / HBM_PEAK,
            "traffic": fft_traffic(L),
            "kernel": (f"H p by FFTs, L = {L}: fft_rows_fwd, fft_cols, fft_rows_mid, fft_cols, "
                       "fft_rows_out (one unit of five launches; achieved = algorithmic bytes "
                       f"{fbytes} / time)"),
            "avg_us": normal_ms[1] * 1e3,
            "blur": blur_entry,
        }

    cpu_baseline = None
    if not args.profile_only and not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits
        from oracle import solvers as SV
        tol0 = rows[0]["modes"]["fp16_kp_fpcg"]["tol"]
        with threadpool_limits(limits=nthreads):
            op = SV.NormalOperator(prob.psf, n, lam, workers=nthreads)
            pre = SV.kp_preconditioner(prob.psf, n, lam, kp)
            # repeat the solve for at least CPU_SAMPLE_S (at most CPU_SAMPLE_MAX solves)
            t0 = time.time()
            count = 0
            while True:
                out = SV.solve(op, prob.b.astype(np.float64), mode=SV.FPCG, tol=tol0,
                               maxit=1000, precond=pre)
                count += 1
                cpu_s = time.time() - t0
                if cpu_s >= CPU_SAMPLE_S or count >= CPU_SAMPLE_MAX:
                    break
        cpu_err = float(np.linalg.norm(out.x - xlam) / np.linalg.norm(xlam))
        cpu_baseline = {
            "value": count / cpu_s, "unit": "solves/s", "cores": nthreads, "kind": "oracle",
            "sample": (f"{count} FP64 KP-preconditioned flexible-PCG solves of the seed-{args.seed} "
                       f"1024^2 problem (tol {tol0:.0e}, {out.iters} iterations each, rel err "
                       f"{cpu_err:.1e}; scipy.fft matvecs with {nthreads} workers, numpy BLAS "
                       f"GEMMs with {nthreads} threads, {cpu_s:.1f} s)"),
            "host": cpu_description(),
        }
        log(f"[bench] cpu oracle: {count} solves in {cpu_s:.2f}s iters={out.iters}")

    batch = run_batch(args.batch, dev, nthreads, parity=not args.profile_only) \
        if args.batch else None
    lowp = None
    if not args.profile_only:
        lowp = run_lowp_setup(prob, b, lam, rows[0]["modes"]["fp16_kp_fpcg"]["tol"], xlam,
                              first["setup_s"])
    periodic = reflexive = reflexive_motion = None
    if not args.profile_only and not args.no_periodic:
        periodic = run_boundary("periodic", args.seed, grid, LADDER, dev)
        reflexive = run_boundary("reflexive", args.seed, grid, LADDER, dev)
        reflexive_motion = run_boundary("reflexive-motion", args.seed, grid, LADDER, dev)

    seeds = f"seeds {args.seed}-{args.seed + len(rows) - 1}" if len(rows) > 1 \
        else f"seed {args.seed}"
    line = {
        "metric": METRIC,
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_median_over_instances"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": (f"FP32 vectors with x accumulated in FP64; {matvec_label(pinfo)}; "
                  "FP16 MFMA preconditioner with FP32 accumulation; FP64 scalars"),
        "data": "synthetic",
        "config": {
            "workload": (f"deblur 1024x1024, Moffat(beta=2.5)+motion PSF 63x63 ({seeds}), zero "
                         "BC, 2% noise, lambda by KP-GCV (32-pt grid), FP16-KP flexible PCG; "
                         "value = 1 / (median over the instances of each instance's median "
                         "solve time)"),
            "n": n, "k": k, "instances": len(rows),
            "parallelism": "single GPU",
            "modes": summary,
            "per_instance": rows,
            "break_even": break_even,
            "gcv_ms": gcv_ms,
            "blur_tile_config": pinfo["blur_config"],
            "normal_op": pinfo["normal_op"],
            "normal_op_us": {"direct": normal_ms[0] * 1e3, "fft": normal_ms[1] * 1e3},
            "precond_fp16_chain_us": prec_ms * 1e3,
            "learned_lambda": learned,
            "batched": batch,
            "periodic": periodic,
            "reflexive": reflexive,
            "reflexive_motion": reflexive_motion,
            "lowp_setup": lowp,
        },
        "roofline": roofline,
        "vector_kernels": vector_kernels(),
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
    the same image and PSF draws with periodic data, x_lambda by the 2-D DFT),
    reflexive (KP_BC_REFLEXIVE, the radial Moffat of the same draw, which
    is symmetric in both axes, with reflexive data, x_lambda by the 2-D DCT)
    or reflexive-motion (the Moffat + motion PSF itself, not symmetric, with
    reflexive data: A^T and H p by the folded FFT passes, x_lambda by the
    oracle's settled FP64 PCG, tolerances from 1e-7 up).
    Lambda by the device's KP-GCV, FP16-KP flexible PCG at the loosest
    ladder tolerance whose x meets 1e-4 against the FP64 x_lambda, then 5
    timed solves and the blur's launch time."""
    import torch
    import synthetic as S
    from paper_2311_15393_amd import KP_BC_PERIODIC, KP_BC_REFLEXIVE, KP_FPCG, KP_OK, KP_P16, Plan
    from oracle import reflexive as RB
    if kind == "periodic":
        from oracle import periodic as ref
        prob, bc = S.large_moffat_periodic(seed), KP_BC_PERIODIC
        what = "Moffat(beta=2.5)+motion PSF 63x63, periodic BC"
        x_lambda = ref.x_lambda
    elif kind == "reflexive":
        prob, bc = S.large_moffat_reflexive(seed), KP_BC_REFLEXIVE
        what = "radial Moffat(beta=2.5) PSF 63x63, reflexive BC"
        x_lambda = RB.x_lambda
    else:
        prob, bc = S.large_moffat_motion_reflexive(seed), KP_BC_REFLEXIVE
        what = "Moffat(beta=2.5)+motion PSF 63x63 (not symmetric), reflexive BC"
        x_lambda = lambda psf, b64, lam: RB.x_lambda_general(psf, b64, lam, tol=1e-12)[0]
        ladder = [t for t in ladder if t >= 1e-7]
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
    xlam = x_lambda(prob.psf, prob.b.astype(np.float64), lam)
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
    plan.time_normal(p, q, reps=3)
    normal_us = plan.time_normal(p, q, reps=20) * 1e3
    plan.close()
    log(f"[bench] {kind}: lambda={lam:.4g} tol={tol:.0e} iters={info.iters} err={err:.2e} "
        f"{ms:.3f} ms/solve; blur {blur_us:.1f} us; H p ({info0['normal_op']}) "
        f"{normal_us:.1f} us; setup {setup_s:.2f}s")
    return {"workload": (f"deblur 1024x1024, {what}, 2% noise, lambda by KP-GCV (32-pt grid), "
                         "FP16-KP flexible PCG"),
            "lambda": lam, "gcv_grid_index": gidx, "tol": tol, "iters": info.iters,
            "rel_err": err, "ok": bool(info.status == KP_OK and err <= 1e-4),
            "ms_per_solve": ms, "solves_per_s": 1e3 / ms, "setup_s": setup_s,
            "kp_rel_error": info0["kp_rel_error"], "blur_config": info0["blur_config"],
            "blur_us": blur_us, "normal_op": info0["normal_op"], "normal_op_us": normal_us}


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


def run_vector_batch(dev, items: int = 16, iters: int = 40) -> dict:
    """One lambda sweep of the seed-0 1024^2 problem as a batch of `items`
    FP16-KP FPCG solves, run for `iters` iterations (a tolerance no item
    reaches), after one warm-up batch; then the plain copy that calibrates
    the HBM counters.  The item vectors (r, p, q, w, z in FP32; x, y and the
    anchor in FP64; the GEMM intermediates) take ~64 MiB per item."""
    import torch
    import synthetic as S
    from paper_2311_15393_amd import KP_FPCG, KP_P16, Plan, solve_batched
    prob = S.large_moffat(0)
    b = torch.from_numpy(prob.b).to(dev)
    plan = Plan(prob.psf, prob.n)
    lam_g, _ = plan.gcv(b, S.lambda_grid())
    lams = [float(v) for v in np.clip(lam_g * 10.0 ** np.linspace(-1.5, 1.5, items), 1e-4, 1.0)]
    xs = [torch.empty_like(b) for _ in range(items)]

    def run():
        return solve_batched([plan], [b] * items, lams, [0] * items, tol=1e-12, maxit=iters,
                             mode=KP_FPCG | KP_P16, xs=xs)
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, infos, _ = run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    src = torch.ones(COPY_CALIB_FLOATS, device=dev, dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    plan.close()
    n2 = prob.n * prob.n
    return {"vector_batch": {"items": items, "n": prob.n, "iterations": [i.iters for i in infos],
                             "wall_s": wall,
                             "update_bytes_per_launch": 32 * n2 * items,
                             "pupdate_bytes_per_launch": 12 * n2 * items}}


def run_batch(nprob: int, dev, nthreads: int = 16, parity: bool = True):
    """Uneven batch: problems of sizes {128,...,1024}, supports 15..63, each
    with 16 lambda values log-spaced over lambda_gcv * 10^[-1.5, 1.5] (KP-GCV
    on the 32-point grid picks lambda_gcv), all solved by one batched FP16
    FPCG call; the sweep is scored by KP-GCV and by the discrepancy principle
    on the solves' actual misfits.  With `parity`, one item for each of the
    image sizes 128, 768 and 1024 (the first problem of that size, at the
    middle of its sweep) is compared with the oracle's settled x_lambda."""
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
    # parity sample: one item per image size against the oracle's x_lambda
    samples = []
    if parity:
        from threadpoolctl import threadpool_limits
        from oracle import solvers as SV
        seen = set()
        for pi, p in enumerate(probs):
            # the smallest and the two largest image sizes (the oracle's
            # settled x_lambda at 1024^2 takes tens of seconds on the host)
            if p.n in seen or p.n not in (128, 768, 1024):
                continue
            seen.add(p.n)
            idx = [kk for kk, (q, _) in enumerate(items) if q == pi]
            it = idx[len(idx) // 2]
            lam_it = items[it][1]
            with threadpool_limits(limits=nthreads):
                xl, xi = SV.x_lambda_iterative(p.psf, p.b.astype(np.float64), lam_it,
                                               workers=nthreads, check=True)
            got = xs[it].cpu().numpy().astype(np.float64)
            err = float(np.linalg.norm(got - xl) / np.linalg.norm(xl))
            samples.append({"problem": pi, "n": p.n, "k": p.k, "lambda": lam_it,
                            "status": int(infos[it].status), "iters": int(infos[it].iters),
                            "rel_err": err, "ok": bool(infos[it].status == KP_OK and err <= 1e-4
                                                       and xi["status"] == "converged"),
                            "_xl": xl})
            log(f"[bench] batch parity: problem {pi} n={p.n} K={p.k} lambda={lam_it:.3g} "
                f"iters={infos[it].iters} err={err:.2e}")
    # the same sweep by continuation: 16 batched calls, largest lambda first,
    # each item warm-started (KP_WARM) from its problem's solution at the
    # previous lambda of the sweep
    from paper_2311_15393_amd import KP_WARM
    order = [[k for k, (q, _) in enumerate(items) if q == pi] for pi in range(nprob)]
    nl = len(order[0])
    xs_c = [torch.empty_like(b) for b in bs]
    infos_c = [None] * len(items)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for stage in range(nl):
        sel = [order[pi][nl - 1 - stage] for pi in range(nprob)]
        if stage > 0:
            prev = [order[pi][nl - stage] for pi in range(nprob)]
            for k, kp_ in zip(sel, prev):
                xs_c[k].copy_(xs_c[kp_])
        out_x, out_i, _ = solve_batched(plans, [bs[k] for k in sel], [lams[k] for k in sel],
                                        [poi[k] for k in sel], tol=1e-6, maxit=1000,
                                        mode=KP_FPCG | KP_P16 | (KP_WARM if stage else 0),
                                        xs=[xs_c[k] for k in sel])
        for k, inf in zip(sel, out_i):
            infos_c[k] = inf
    torch.cuda.synchronize()
    wall_c = time.perf_counter() - t0
    iters_c = np.array([i.iters for i in infos_c])
    ok_c = sum(i.status == KP_OK for i in infos_c)
    cont_samples = []
    for smp in samples:
        k = next(kk for kk, (q, lam_k) in enumerate(items)
                 if q == smp["problem"] and lam_k == smp["lambda"])
        got = xs_c[k].cpu().numpy().astype(np.float64)
        err = float(np.linalg.norm(got - smp["_xl"]) / np.linalg.norm(smp["_xl"]))
        cont_samples.append({"problem": smp["problem"], "n": smp["n"], "rel_err": err,
                             "iters": int(infos_c[k].iters),
                             "ok": bool(infos_c[k].status == KP_OK and err <= 1e-4)})
    log(f"[bench] batch by continuation: {wall_c:.3f}s ({len(items) / wall_c:.1f}/s), converged "
        f"{ok_c}, iters mean {iters_c.mean():.1f} max {iters_c.max()}")
    for smp in samples:
        smp.pop("_xl", None)
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
        "parity_samples": samples,
        "parity_ok": all(x["ok"] for x in samples) if samples else None,
        "exact_diag": {"wall_s": wall2, "solves_per_s": len(items) / wall2, "converged": ok2,
                       "iters_mean": float(iters2.mean()), "iters_max": int(iters2.max())},
        "continuation": {"what": "16 batched calls over the sweep, largest lambda first, each "
                                 "item warm-started from its problem's previous solution",
                         "wall_s": wall_c, "solves_per_s": len(items) / wall_c,
                         "converged": ok_c, "iters_mean": float(iters_c.mean()),
                         "iters_max": int(iters_c.max()), "parity_samples": cont_samples},
    }
    log(f"[bench] batch: {wall:.3f}s for {len(items)} solves ({len(items) / wall:.1f}/s), "
        f"converged {ok}, iters mean {iters.mean():.1f} max {iters.max()}; "
        f"error vs x_true at GCV pick {np.mean(errs_gcv):.3f}, DP pick {np.mean(errs_dp):.3f}")
    for pl in plans:
        pl.close()
    return out


if __name__ == "__main__":
    main()
