"""KP-SVD-preconditioned (flexible) CG for Tikhonov image deblurring on
MI355X (gfx950): HIP kernels behind the C ABI in include/kpcg.h, with a thin
ctypes binding (kpcg.py)."""
from .kpcg import (KP_BLUR_MFMA, KP_BLUR_MFMA32, KP_NORMAL_PLAN, KP_NORMAL_DIRECT, KP_NORMAL_FFT, KP_OK_FALLBACK, KP_NO_FALLBACK, KP_EXACT_DIAG, KP_HIST, KP_HIST_MAX, KP_BC_ZERO, KP_BC_PERIODIC, KP_BC_REFLEXIVE, KP_SETUP_LOWP, KP_CG, KP_PCG, KP_FPCG, KP_P32, KP_P16, KP_P8, KP_WARM, KP_OK, KP_MAXIT,
                   KP_BREAKDOWN, KP_ERR_ARG, KP_ERR_UNSUPPORTED, KP_ERR_HIP, KP_ERR_SOLVER,
                   KP_ERR_WORKSPACE, KP_MAX_PSF, KPError, Plan, SolveInfo, load, strerror,
                   workspace_size, exported_symbols, LIB_PATH, KP_BATCH_EAGER,
                   solve_batched, batched_workspace_size, Mlp, KP_MLP_NFEAT, KP_MLP_HIDDEN, KP_MLP_NPARAM,
                   KP_PREDICT_NOALLOC_MAX_ROWS)

__all__ = ["KP_BLUR_MFMA", "KP_BLUR_MFMA32", "KP_NORMAL_PLAN", "KP_NORMAL_DIRECT", "KP_NORMAL_FFT", "KP_OK_FALLBACK", "KP_NO_FALLBACK", "KP_EXACT_DIAG", "KP_HIST", "KP_HIST_MAX", "KP_BC_ZERO", "KP_BC_PERIODIC", "KP_BC_REFLEXIVE", "KP_SETUP_LOWP", "KP_CG", "KP_PCG", "KP_FPCG", "KP_P32", "KP_P16", "KP_P8", "KP_WARM", "KP_OK",
           "KP_MAXIT", "KP_BREAKDOWN", "KP_ERR_ARG", "KP_ERR_UNSUPPORTED", "KP_ERR_HIP",
           "KP_ERR_SOLVER", "KP_ERR_WORKSPACE", "KP_MAX_PSF", "KPError", "Plan", "SolveInfo",
           "load", "strerror", "workspace_size", "exported_symbols", "LIB_PATH",
           "KP_BATCH_EAGER", "solve_batched", "batched_workspace_size", "Mlp", "KP_MLP_NFEAT", "KP_MLP_HIDDEN",
           "KP_MLP_NPARAM", "KP_PREDICT_NOALLOC_MAX_ROWS"]
