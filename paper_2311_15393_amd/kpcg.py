"""Thin ctypes binding of libkpcg (the C ABI declared in include/kpcg.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch CUDA tensors (float32, contiguous, n x n);
torch supplies all device memory (the plan, model and batch workspaces are
torch uint8 tensors the library only takes views into) and the stream.  The
binding fails loudly if the shared library has not been built.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libkpcg.so")

# status codes and mode bits (mirror include/kpcg.h)
KP_OK, KP_MAXIT, KP_BREAKDOWN, KP_OK_FALLBACK = 0, 1, 2, 3
KP_ERR_ARG, KP_ERR_UNSUPPORTED, KP_ERR_HIP, KP_ERR_WORKSPACE, KP_ERR_SOLVER = -1, -2, -3, -4, -5
KP_CG, KP_PCG, KP_FPCG = 0x000, 0x001, 0x002
KP_P32, KP_P16, KP_P8 = 0x000, 0x010, 0x020
KP_WARM = 0x100
KP_BATCH_EAGER = 0x200
KP_NO_FALLBACK = 0x400
KP_EXACT_DIAG = 0x800
KP_HIST = 0x1000
KP_HIST_MAX = 16384
KP_PREDICT_NOALLOC_MAX_ROWS = 2048
KP_MAX_PSF = 63
KP_BC_ZERO = 0
KP_BC_PERIODIC = 1
KP_BC_REFLEXIVE = 2
KP_SETUP_LOWP = 0x100
KP_BLUR_MFMA = 6
KP_BLUR_MFMA32 = 7
KP_NORMAL_PLAN, KP_NORMAL_DIRECT, KP_NORMAL_FFT = -1, 0, 1
KP_MLP_NFEAT, KP_MLP_HIDDEN, KP_MLP_NPARAM = 128, 256, 164865


class KPError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {strerror(status)} (status {status})")
        self.status = status


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("replacements", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("relres_rec", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("rhs_norm", ctypes.c_double),
                ("misfit", ctypes.c_double), ("ms", ctypes.c_float),
                ("reserved", ctypes.c_int32)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("kron_terms", ctypes.c_int32), ("normal_op", ctypes.c_int32),
                ("kp_rel_error", ctypes.c_double),
                ("sigma_c_max", ctypes.c_double), ("sigma_c_min", ctypes.c_double),
                ("sigma_r_max", ctypes.c_double), ("sigma_r_min", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t), ("blur_config", ctypes.c_int32),
                ("blur_config_ms", ctypes.c_float * 8), ("fft_length", ctypes.c_int32),
                ("normal_op_ms", ctypes.c_float * 2)]


class _LambdaInfo(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("lambda_pred", ctypes.c_double),
                ("lambda_gcv", ctypes.c_double), ("gcv_ratio", ctypes.c_double),
                ("fell_back", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None

_VP = ctypes.c_void_p
_SIGS = {
    "kp_workspace_size": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "kp_setup": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP,
                                ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "kp_plan_query": (ctypes.c_int, [_VP, ctypes.POINTER(_PlanInfo)]),
    "pcg_solve": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int, _VP, ctypes.POINTER(_Info), _VP]),
    "gcv_lambda": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, ctypes.c_double, _VP, _VP,
                                  _VP]),
    "discrepancy_lambda": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, _VP, _VP, _VP]),
    "kp_destroy": (ctypes.c_int, [_VP]),
    "pcg_solve_batched": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int, _VP,
                                         _VP, _VP, ctypes.c_size_t, _VP]),
    "pcg_solve_batched_workspace_size": (ctypes.c_size_t, [_VP, ctypes.c_int, _VP, ctypes.c_int,
                                                           ctypes.c_int]),
    "kp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "kp_blur": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, _VP]),
    "kp_normal_fp64": (ctypes.c_int, [_VP, _VP, ctypes.c_double, _VP, _VP]),
    "kp_precond": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_int, _VP, _VP]),
    "kp_get_factors": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "kp_get_diag": (ctypes.c_int, [_VP, _VP]),
    "kp_get_history": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                      _VP]),
    "kp_time_blur": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_float), _VP]),
    "kp_time_precond": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_int, _VP,
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_float), _VP]),
    "kp_set_blur_config": (ctypes.c_int, [_VP, ctypes.c_int, _VP]),
    "kp_set_normal_op": (ctypes.c_int, [_VP, ctypes.c_int, _VP]),
    "kp_normal": (ctypes.c_int, [_VP, _VP, ctypes.c_double, _VP, ctypes.c_int, _VP]),
    "kp_time_normal": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_float), _VP]),
    "opt_lambda": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int, _VP, _VP, _VP]),
    "kp_features": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "mlp_workspace_size": (ctypes.c_size_t, [ctypes.c_int]),
    "mlp_create": (ctypes.c_int, [ctypes.c_int, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "mlp_set_params": (ctypes.c_int, [_VP, _VP, _VP]),
    "mlp_get_params": (ctypes.c_int, [_VP, _VP, _VP]),
    "mlp_set_normalizer": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "mlp_get_normalizer": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "mlp_fit_normalizer": (ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP]),
    "lambda_predict": (ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP, _VP]),
    "lambda_predict_noalloc": (ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP, _VP]),
    "mlp_train_step": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, _VP, ctypes.c_int,
                                      ctypes.c_float, _VP, _VP]),
    "mlp_gradients": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, _VP, _VP, _VP]),
    "mlp_destroy": (ctypes.c_int, [_VP]),
    "kp_lambda_learned": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int, ctypes.c_double,
                                         ctypes.POINTER(_LambdaInfo), _VP]),
}


def exported_symbols():
    return sorted(_SIGS)


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libkpcg not built: {path} is missing "
                          "(run python -m paper_2311_15393_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().kp_strerror(int(status)).decode()


def _check(status: int, what: str, ok=(KP_OK,)):
    if status not in ok:
        raise KPError(status, what)
    return status


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _dev_image(t, n, name, dtype=None):
    import torch
    dtype = dtype or torch.float32
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or tuple(t.shape) != (n, n) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {n}x{n} {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class SolveInfo:
    iters: int
    status: int
    replacements: int
    relres_rec: float
    relres_true: float
    lam: float
    rhs_norm: float
    misfit: float = 0.0
    fallback: int = 0
    ms: float = 0.0             # device time of the solve (pcg_solve)
    # with history=True: ||r_k|| / ||A^T b|| of the recurrence after
    # iteration k, and of the true residual where one was formed (else NaN)
    history_rec: np.ndarray | None = None
    history_true: np.ndarray | None = None


def workspace_size(n: int, k: int) -> int:
    """kp_workspace_size: device bytes of a plan (0 for invalid sizes)."""
    return int(load().kp_workspace_size(n, k, 0))


def _workspace(nbytes: int, what: str):
    """A torch-owned device buffer of nbytes (uint8, 256-byte aligned by the
    caching allocator) for the library to take views into."""
    import torch
    if nbytes <= 0:
        raise KPError(KP_ERR_ARG, what)
    return torch.empty(int(nbytes), dtype=torch.uint8, device=torch.cuda.current_device())


def _ws_ptr(workspace):
    if workspace is None:
        return None, 0
    return (ctypes.c_void_p(workspace.data_ptr()),
            workspace.numel() * workspace.element_size())


class Plan:
    """kp_setup / kp_destroy around one PSF and image size.  The plan lives
    in `workspace` (a CUDA tensor of at least workspace_size(n, k) bytes);
    by default the binding allocates one with torch."""

    def __init__(self, psf: np.ndarray, n: int, bc: int = 0, stream=None, workspace=None):
        lib = load()
        psf = np.ascontiguousarray(psf, dtype=np.float64)
        if psf.ndim != 2 or psf.shape[0] != psf.shape[1]:
            raise ValueError("psf must be a square 2-D array")
        self.n, self.k = int(n), int(psf.shape[0])
        self.bc = int(bc)
        if workspace is None and 1 <= self.k <= 2 * self.n - 1 and self.k % 2 == 1:
            nbytes = lib.kp_workspace_size(self.n, self.k, 0)
            if nbytes:
                workspace = _workspace(nbytes, "kp_workspace_size")
        self._ws = workspace
        wptr, wbytes = _ws_ptr(workspace)
        h = ctypes.c_void_p()
        st = lib.kp_setup(psf.ctypes.data_as(ctypes.c_void_p), self.k, self.n, int(bc), wptr,
                          wbytes, _stream(stream), ctypes.byref(h))
        _check(st, "kp_setup")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().kp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- properties -------------------------------------------------------
    def query(self) -> dict:
        pi = _PlanInfo()
        _check(load().kp_plan_query(self._h, ctypes.byref(pi)), "kp_plan_query")
        out = {f: getattr(pi, f) for f, _ in _PlanInfo._fields_}
        out["blur_config_ms"] = list(out["blur_config_ms"])
        out["normal_op_ms"] = list(out["normal_op_ms"])
        return out

    def factors(self, with_v: bool = True):
        n = self.n
        sc, sr = np.empty(n), np.empty(n)
        vc = np.empty((n, n)) if with_v else None
        vr = np.empty((n, n)) if with_v else None
        p = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        _check(load().kp_get_factors(self._h, p(sc), p(sr), p(vc), p(vr)), "kp_get_factors")
        return sc, sr, vc, vr

    def exact_diag(self):
        """kp_get_diag: D0[i, j] = ||A (v_c,i v_r,j^T)||_F^2 (n x n float32)."""
        d0 = np.empty((self.n, self.n), dtype=np.float32)
        _check(load().kp_get_diag(self._h, d0.ctypes.data_as(ctypes.c_void_p)), "kp_get_diag")
        return d0

    # -- the hot path -----------------------------------------------------
    def solve(self, b, lam: float, tol: float = 1e-6, maxit: int = 1000,
              mode: int = KP_FPCG | KP_P16, x=None, stream=None, raise_on_fail=True,
              history: bool = False):
        import torch
        bp = _dev_image(b, self.n, "b")
        if x is None:
            x = torch.empty_like(b)
        xp = _dev_image(x, self.n, "x")
        info = _Info()
        if history:
            mode |= KP_HIST
        st = load().pcg_solve(self._h, bp, float(lam), float(tol), int(maxit), int(mode), xp,
                              ctypes.byref(info), _stream(stream))
        if st < 0 or (raise_on_fail and st not in (KP_OK, KP_OK_FALLBACK, KP_MAXIT)):
            raise KPError(st, "pcg_solve")
        out = SolveInfo(info.iters, st, info.replacements, info.relres_rec, info.relres_true,
                        info.lambda_, info.rhs_norm, info.misfit, info.fallback, info.ms)
        if mode & KP_HIST:
            out.history_rec, out.history_true = self.history(stream=stream)
        return x, out

    def history(self, stream=None):
        """kp_get_history: (relres_rec, relres_true) of the last solve run
        with KP_HIST (empty arrays if it ran without)."""
        count = ctypes.c_int()
        _check(load().kp_get_history(self._h, None, None, 0, ctypes.byref(count),
                                     _stream(stream)), "kp_get_history")
        m = count.value
        rec, tru = np.empty(m), np.empty(m)
        if m:
            _check(load().kp_get_history(self._h, rec.ctypes.data_as(ctypes.c_void_p),
                                         tru.ctypes.data_as(ctypes.c_void_p), m,
                                         ctypes.byref(count), _stream(stream)),
                   "kp_get_history")
        return rec, tru

    def gcv(self, b, grid, omega: float = 1.0, stream=None):
        bp = _dev_image(b, self.n, "b")
        grid = np.ascontiguousarray(grid, dtype=np.float64)
        out = ctypes.c_double()
        scores = np.empty(grid.size)
        _check(load().gcv_lambda(self._h, bp, grid.ctypes.data_as(ctypes.c_void_p), grid.size,
                                 float(omega), ctypes.byref(out),
                                 scores.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
               "gcv_lambda")
        return out.value, scores

    def discrepancy(self, b, grid, noise_norm: float, eta: float = 1.0, stream=None):
        bp = _dev_image(b, self.n, "b")
        grid = np.ascontiguousarray(grid, dtype=np.float64)
        out = ctypes.c_double()
        vals = np.empty(grid.size)
        _check(load().discrepancy_lambda(self._h, bp, grid.ctypes.data_as(ctypes.c_void_p),
                                         grid.size, float(noise_norm), float(eta),
                                         ctypes.byref(out),
                                         vals.ctypes.data_as(ctypes.c_void_p),
                                         _stream(stream)), "discrepancy_lambda")
        return out.value, vals

    def opt(self, b, x_true, grid, stream=None):
        """opt_lambda: optimal-error rule in the KP basis (needs the true image)."""
        grid = np.ascontiguousarray(grid, dtype=np.float64)
        out = ctypes.c_double()
        scores = np.empty(grid.size)
        _check(load().opt_lambda(self._h, _dev_image(b, self.n, "b"),
                                 _dev_image(x_true, self.n, "x_true"),
                                 grid.ctypes.data_as(ctypes.c_void_p), grid.size,
                                 ctypes.byref(out), scores.ctypes.data_as(ctypes.c_void_p),
                                 _stream(stream)), "opt_lambda")
        return out.value, scores

    def features(self, b, out=None, stream=None):
        """kp_features: the 128 spectral features of b into out (CUDA float32, 128)."""
        import torch
        if out is None:
            out = torch.empty(KP_MLP_NFEAT, device=b.device, dtype=torch.float32)
        _check_vec(out, KP_MLP_NFEAT, "out")
        _check(load().kp_features(self._h, _dev_image(b, self.n, "b"),
                                  ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "kp_features")
        return out

    def lambda_learned(self, mlp, b, grid, tau: float, stream=None) -> dict:
        """kp_lambda_learned: the network's lambda, judged by GCV (fallback)."""
        grid = np.ascontiguousarray(grid, dtype=np.float64)
        info = _LambdaInfo()
        _check(load().kp_lambda_learned(self._h, mlp._h, _dev_image(b, self.n, "b"),
                                        grid.ctypes.data_as(ctypes.c_void_p), grid.size,
                                        float(tau), ctypes.byref(info), _stream(stream)),
               "kp_lambda_learned")
        return {"lambda": info.lambda_, "lambda_pred": info.lambda_pred,
                "lambda_gcv": info.lambda_gcv, "gcv_ratio": info.gcv_ratio,
                "fell_back": bool(info.fell_back)}

    # -- operator-level entry points -------------------------------------
    def blur(self, x, y, transpose: bool = False, stream=None):
        _check(load().kp_blur(self._h, _dev_image(x, self.n, "x"), _dev_image(y, self.n, "y"),
                              int(bool(transpose)), _stream(stream)), "kp_blur")
        return y

    def normal_fp64(self, x, lam: float, y, stream=None):
        import torch
        _check(load().kp_normal_fp64(self._h, _dev_image(x, self.n, "x"), float(lam),
                                     _dev_image(y, self.n, "y", torch.float64),
                                     _stream(stream)), "kp_normal_fp64")
        return y

    def time_blur(self, x, y, transpose: bool = False, reps: int = 20, stream=None) -> float:
        ms = ctypes.c_float()
        _check(load().kp_time_blur(self._h, _dev_image(x, self.n, "x"),
                                   _dev_image(y, self.n, "y"), int(bool(transpose)), int(reps),
                                   ctypes.byref(ms), _stream(stream)), "kp_time_blur")
        return float(ms.value)

    def time_precond(self, r, lam: float, mode: int, z, reps: int = 20, stream=None) -> float:
        ms = ctypes.c_float()
        _check(load().kp_time_precond(self._h, _dev_image(r, self.n, "r"), float(lam), int(mode),
                                      _dev_image(z, self.n, "z"), int(reps), ctypes.byref(ms),
                                      _stream(stream)), "kp_time_precond")
        return float(ms.value)

    def set_normal_op(self, op: int) -> int:
        """kp_set_normal_op: H p for the solver's iterations by the direct
        blurs (KP_NORMAL_DIRECT) or the FFTs (KP_NORMAL_FFT); returns the
        previous choice."""
        prev = ctypes.c_int()
        _check(load().kp_set_normal_op(self._h, int(op), ctypes.byref(prev)), "kp_set_normal_op")
        return prev.value

    def normal(self, x, lam: float, y, op: int = KP_NORMAL_PLAN, stream=None):
        """kp_normal: y = (A^T A + lam^2 I) x in FP32 by the given form."""
        _check(load().kp_normal(self._h, _dev_image(x, self.n, "x"), float(lam),
                                _dev_image(y, self.n, "y"), int(op), _stream(stream)),
               "kp_normal")
        return y

    def time_normal(self, x, y, op: int = KP_NORMAL_PLAN, reps: int = 20, stream=None) -> float:
        ms = ctypes.c_float()
        _check(load().kp_time_normal(self._h, _dev_image(x, self.n, "x"),
                                     _dev_image(y, self.n, "y"), int(op), int(reps),
                                     ctypes.byref(ms), _stream(stream)), "kp_time_normal")
        return float(ms.value)

    def set_blur_config(self, cfg: int) -> int:
        """kp_set_blur_config: force the blur kernel (0..5 VALU shapes, 6 MFMA);
        returns the previous choice."""
        prev = ctypes.c_int()
        _check(load().kp_set_blur_config(self._h, int(cfg), ctypes.byref(prev)),
               "kp_set_blur_config")
        return prev.value

    def precond(self, r, lam: float, mode: int, z, stream=None):
        _check(load().kp_precond(self._h, _dev_image(r, self.n, "r"), float(lam), int(mode),
                                 _dev_image(z, self.n, "z"), _stream(stream)), "kp_precond")
        return z


def _check_vec(t, count, name, dtype=None):
    import torch
    dtype = dtype or torch.float32
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or t.numel() != count or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of {count} elements")
    return ctypes.c_void_p(t.data_ptr())


class Mlp:
    """mlp_create / mlp_destroy: the lambda-predicting network (include/kpcg.h)."""

    def __init__(self, max_batch: int = 1024, stream=None, workspace=None):
        lib = load()
        self.max_batch = int(max_batch)
        if workspace is None:
            nbytes = lib.mlp_workspace_size(self.max_batch)
            if nbytes:
                workspace = _workspace(nbytes, "mlp_workspace_size")
        self._ws = workspace
        wptr, wbytes = _ws_ptr(workspace)
        h = ctypes.c_void_p()
        _check(lib.mlp_create(self.max_batch, wptr, wbytes, _stream(stream), ctypes.byref(h)),
               "mlp_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, stream=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != KP_MLP_NPARAM:
            raise ValueError(f"expected {KP_MLP_NPARAM} parameters")
        _check(load().mlp_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p),
                                     _stream(stream)), "mlp_set_params")

    def get_params(self, stream=None) -> np.ndarray:
        p = np.empty(KP_MLP_NPARAM, dtype=np.float32)
        _check(load().mlp_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p),
                                     _stream(stream)), "mlp_get_params")
        return p

    def set_normalizer(self, mean, scale, stream=None):
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(scale, dtype=np.float32)
        if m.size != KP_MLP_NFEAT or s.size != KP_MLP_NFEAT:
            raise ValueError("normaliser needs 128 means and 128 scales")
        _check(load().mlp_set_normalizer(self._h, m.ctypes.data_as(ctypes.c_void_p),
                                         s.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
               "mlp_set_normalizer")

    def get_normalizer(self, stream=None):
        m = np.empty(KP_MLP_NFEAT, dtype=np.float32)
        s = np.empty(KP_MLP_NFEAT, dtype=np.float32)
        _check(load().mlp_get_normalizer(self._h, m.ctypes.data_as(ctypes.c_void_p),
                                         s.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
               "mlp_get_normalizer")
        return m, s

    def fit_normalizer(self, features, stream=None):
        nb = _feature_rows(features)
        _check(load().mlp_fit_normalizer(self._h, ctypes.c_void_p(features.data_ptr()), nb,
                                         _stream(stream)), "mlp_fit_normalizer")

    def predict(self, features, out=None, stream=None):
        """lambda_predict: log10(lambda) for each feature row (CUDA float64 out)."""
        import torch
        nb = _feature_rows(features)
        if out is None:
            out = torch.empty(nb, device=features.device, dtype=torch.float64)
        _check_vec(out, nb, "out", torch.float64)
        _check(load().lambda_predict(self._h, ctypes.c_void_p(features.data_ptr()), nb,
                                     ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "lambda_predict")
        return out

    def predict_noalloc(self, features, out, stream=None):
        """lambda_predict_noalloc: as predict, with the activations in the
        library's static device array (at most KP_PREDICT_NOALLOC_MAX_ROWS
        rows; `out` is required, so nothing is allocated)."""
        import torch
        nb = _feature_rows(features)
        _check_vec(out, nb, "out", torch.float64)
        _check(load().lambda_predict_noalloc(self._h, ctypes.c_void_p(features.data_ptr()), nb,
                                             ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "lambda_predict_noalloc")
        return out

    def train_step(self, features, targets, lr: float, rows=None, want_loss: bool = False,
                   stream=None):
        """mlp_train_step on rows (host int array or None = all rows)."""
        import torch
        nrows = _feature_rows(features)
        _check_vec(targets, nrows, "targets")
        if rows is None:
            rp, nb = None, nrows
        else:
            rows = np.ascontiguousarray(rows, dtype=np.int32)
            rp, nb = rows.ctypes.data_as(ctypes.c_void_p), rows.size
        loss = ctypes.c_double()
        _check(load().mlp_train_step(self._h, ctypes.c_void_p(features.data_ptr()),
                                     ctypes.c_void_p(targets.data_ptr()), nrows, rp, nb,
                                     float(lr), ctypes.byref(loss) if want_loss else None,
                                     _stream(stream)), "mlp_train_step")
        return loss.value if want_loss else None

    def gradients(self, features, targets, stream=None):
        """mlp_gradients: (loss, flat FP32 gradient) on all rows, no update."""
        nb = _feature_rows(features)
        _check_vec(targets, nb, "targets")
        g = np.empty(KP_MLP_NPARAM, dtype=np.float32)
        loss = ctypes.c_double()
        _check(load().mlp_gradients(self._h, ctypes.c_void_p(features.data_ptr()),
                                    ctypes.c_void_p(targets.data_ptr()), nb,
                                    g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss),
                                    _stream(stream)), "mlp_gradients")
        return loss.value, g


def _feature_rows(features) -> int:
    import torch
    if (not isinstance(features, torch.Tensor) or not features.is_cuda
            or features.dtype != torch.float32 or features.dim() != 2
            or features.shape[1] != KP_MLP_NFEAT or not features.is_contiguous()):
        raise ValueError("features must be a contiguous CUDA float32 (rows, 128) tensor")
    return int(features.shape[0])


def batched_workspace_size(plans, plan_of_item, mode: int = KP_FPCG | KP_P16) -> int:
    """pcg_solve_batched_workspace_size: device bytes of one batched call."""
    hp = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    poi = np.ascontiguousarray(plan_of_item, dtype=np.int32)
    return int(load().pcg_solve_batched_workspace_size(hp, len(plans),
                                                       poi.ctypes.data_as(ctypes.c_void_p),
                                                       poi.size, int(mode)))


def solve_batched(plans, bs, lambdas, plan_of_item, tol: float = 1e-6, maxit: int = 1000,
                  mode: int = KP_FPCG | KP_P16, xs=None, stream=None, workspace=None):
    """pcg_solve_batched: item i solves with plans[plan_of_item[i]], data bs[i]
    (CUDA float32 n_i x n_i), parameter lambdas[i].  The batch runs in
    `workspace` (CUDA tensor of at least batched_workspace_size bytes; by
    default allocated with torch for the call).  Returns (xs, infos, status)."""
    import torch
    lib = load()
    nitems = len(bs)
    if not (len(lambdas) == nitems == len(plan_of_item)):
        raise ValueError("bs, lambdas and plan_of_item must have the same length")
    if xs is None:
        xs = [torch.empty_like(b) for b in bs]
    if workspace is None:
        nbytes = batched_workspace_size(plans, plan_of_item, mode)
        if nbytes == 0:
            # the size query cannot say why: the solve itself names the
            # refusal (it validates everything before it needs a workspace)
            hp = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
            poi = np.ascontiguousarray(plan_of_item, dtype=np.int32)
            st = lib.pcg_solve_batched(hp, len(plans), None, None,
                                       poi.ctypes.data_as(ctypes.c_void_p), nitems, 1.0, 1,
                                       int(mode), None, None, None, 0, _stream(stream))
            raise KPError(st if st < 0 else KP_ERR_ARG, "pcg_solve_batched_workspace_size")
        workspace = _workspace(nbytes, "pcg_solve_batched_workspace_size")
    wptr, wbytes = _ws_ptr(workspace)
    hp = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    bp = (ctypes.c_void_p * nitems)(*[_dev_image(b, plans[plan_of_item[i]].n, "b").value
                                      for i, b in enumerate(bs)])
    xp = (ctypes.c_void_p * nitems)(*[_dev_image(x, plans[plan_of_item[i]].n, "x").value
                                      for i, x in enumerate(xs)])
    lam = np.ascontiguousarray(lambdas, dtype=np.float64)
    poi = np.ascontiguousarray(plan_of_item, dtype=np.int32)
    infos = (_Info * nitems)()
    st = lib.pcg_solve_batched(hp, len(plans), bp, lam.ctypes.data_as(ctypes.c_void_p),
                               poi.ctypes.data_as(ctypes.c_void_p), nitems, float(tol),
                               int(maxit), int(mode), xp, infos, wptr, wbytes, _stream(stream))
    if st < 0:
        raise KPError(st, "pcg_solve_batched")
    out = [SolveInfo(i.iters, i.status, i.replacements, i.relres_rec, i.relres_true, i.lambda_,
                     i.rhs_norm, i.misfit) for i in infos]
    return xs, out, st
