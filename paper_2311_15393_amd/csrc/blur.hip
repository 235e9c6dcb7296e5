// Direct-convolution matvecs with the blur A and its transpose.
//
// The paper applies A and A^T through structured matvecs and names them the
// most expensive part of an iteration (Section 5.2, work-unit model).  Here
// they are 2-D correlations computed directly:
//     out[i][j] = sum_{a,b < K} Q[a][b] in[i + a - h][j + b - h]
// with Q = P for A^T and Q = P rotated by 180 degrees for A, and the input
// zero outside the image (KP_BC_ZERO) or extended periodically
// (KP_BC_PERIODIC, indices taken mod n).
//
// Design (gfx950): one workgroup per TH x TW output tile stages the
// (TH+K-1) x (TW+KQ) input halo tile in LDS with coalesced global loads and
// zero fill outside the image.  Each thread owns RY rows x RX consecutive
// columns.  The tap loop walks input rows once ("row sweep"): a window of
// RX+BC-1 inputs is read from LDS with 16-byte loads and reused by RX*BC
// FMAs for each of the RY output rows it feeds, with taps read as
// wave-uniform values.  Taps are padded to KQ = ceil(K/BC)*BC columns with
// zeros.  The work is FP32-VALU bound (K^2/4 flop per byte moved).
#include "blur_core.h"

namespace kpcg {

template <int TX, int TY, int RX, int RY, int BC, typename In, typename Acc, typename Tap,
          class Epi>
__global__ __launch_bounds__(TX* TY) void blur_kernel(
    const In* __restrict__ src, const Tap* __restrict__ taps, int n, int K, int KQ, int LDW,
    Epi epi, Ctrl* ctrl, int skip_if_done, double* partials, int bc) {
  if (skip_if_done && ctrl->done != RUNNING) return;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  blur_tile<TX, TY, RX, RY, BC, In, Acc, Tap, Epi>(
      src, taps, n, K, KQ, LDW, blockIdx.y * (TY * RY), blockIdx.x * (TX * RX), epi,
      partials + Epi::kSlot * MAX_PARTIALS + bid, bc);
}

// ---------------------------------------------------------------------------
// launch configurations
// ---------------------------------------------------------------------------

template <int TX, int TY, int RX, int RY, typename In, typename Acc, typename Tap, class Epi>
static hipError_t run_blur(const Plan& P, const In* src, const Tap* taps, Epi epi,
                           Ctrl* ctrl, int skip, hipStream_t s) {
  constexpr int TW = TX * RX, TH = TY * RY;
  const int n = P.n, K = P.k, KQ = P.kq;
  const int ldw = lds_width<TX, TY, RX, RY, In>(KQ);
  const size_t lds = (size_t)(TH + K - 1) * ldw * sizeof(In);
  dim3 grid((n + TW - 1) / TW, (n + TH - 1) / TH);
  if ((long)grid.x * grid.y > MAX_PARTIALS) return hipErrorInvalidValue;
  auto kern = blur_kernel<TX, TY, RX, RY, BC, In, Acc, Tap, Epi>;
  if (lds > 65536) {
    // beyond 64 KB the kernel must opt in to the larger dynamic LDS size
    static size_t granted = 65536;
    if (lds > granted) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      granted = lds;
    }
  }
  hipLaunchKernelGGL(kern, grid, dim3(TX * TY), lds, s, src, taps, n, K, KQ, ldw, epi, ctrl,
                     skip, P.partials, P.bc);
  return hipGetLastError();
}

template <int TX, int TY, int RX, int RY>
static int blur_blocks(int n) {
  return ((n + TX * RX - 1) / (TX * RX)) * ((n + TY * RY - 1) / (TY * RY));
}

template <class Epi>
static hipError_t blur_dispatch(int cfg, const Plan& P, const float* src, const float* taps,
                                Epi epi, Ctrl* ctrl, int skip, hipStream_t s, int* nb) {
  const int n = P.n;
  switch (cfg) {
    case BLUR_CFG_MFMA: *nb = mfma_blocks(n);
      return launch_blur_mfma(P, src, taps == P.taps32, epi, ctrl, skip, s);
    case BLUR_CFG_MFMA32: *nb = mfma_blocks(n);
      return launch_blur_mfma32(P, src, taps == P.taps32, epi, ctrl, skip, s);
    case 1: *nb = blur_blocks<KP_CFG1>(n);
      return run_blur<KP_CFG1, float, float, float>(P, src, taps, epi, ctrl, skip, s);
    case 2: *nb = blur_blocks<KP_CFG2>(n);
      return run_blur<KP_CFG2, float, float, float>(P, src, taps, epi, ctrl, skip, s);
    case 3: *nb = blur_blocks<KP_CFG3>(n);
      return run_blur<KP_CFG3, float, float, float>(P, src, taps, epi, ctrl, skip, s);
    case 4: *nb = blur_blocks<KP_CFG4>(n);
      return run_blur<KP_CFG4, float, float, float>(P, src, taps, epi, ctrl, skip, s);
    case 5: *nb = blur_blocks<KP_CFG5>(n);
      return run_blur<KP_CFG5, float, float, float>(P, src, taps, epi, ctrl, skip, s);
    default: *nb = blur_blocks<KP_CFG0>(n);
      return run_blur<KP_CFG0, float, float, float>(P, src, taps, epi, ctrl, skip, s);
  }
}

hipError_t launch_blur_f32(const Plan& P, const float* src, float* dst, bool transpose,
                           hipStream_t s, const Ctrl* ctrl) {
  if (transpose && P.refl_general) {
    // the reflexive A^T of a PSF that is not symmetric is no blur: the
    // folded correlation by FFTs (no control-block test)
    if (ctrl) return hipErrorInvalidValue;
    return launch_fft_at(P, src, dst, s);
  }
  EpiStoreF32 e{dst, P.n};
  int nb;
  return blur_dispatch(P.blur_cfg, P, src, transpose ? P.taps32 : P.taps32_flip, e,
                       const_cast<Ctrl*>(ctrl), ctrl != nullptr, s, &nb);
}

hipError_t launch_blur_normal(const Plan& P, const float* q, const float* p, float* w,
                              float lam2, hipStream_t s, int* nb) {
  EpiNormalW e{p, w, lam2, P.n};
  return blur_dispatch(P.blur_cfg, P, q, P.taps32, e, P.ctrl, 1, s, nb);
}

// Autotuner: time every FP32-VALU tile shape and the MFMA kernel on this
// plan's (n, K) and keep the fastest (3 timed launches each after one
// warm-up; scratch vectors p, q); the batched path uses the fastest VALU shape.
hipError_t autotune_blur(Plan& P, hipStream_t s, float* times_ms) {
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return err;
  err = hipEventCreate(&e1);
  if (err != hipSuccess) return err;
  err = hipMemsetAsync(P.p, 0, sizeof(float) * (size_t)P.n * P.n, s);
  int best = 0, best_valu = 0;
  float best_ms = 1e30f, best_valu_ms = 1e30f;
  for (int c = 0; c <= BLUR_CFG_MFMA32 && err == hipSuccess; ++c) {
    EpiStoreF32 e{P.q, P.n};
    int nb;
    err = blur_dispatch(c, P, P.p, P.taps32_flip, e, nullptr, 0, s, &nb);
    if (err != hipSuccess) break;
    err = hipEventRecord(e0, s);
    for (int it = 0; it < 3 && err == hipSuccess; ++it)
      err = blur_dispatch(c, P, P.p, P.taps32_flip, e, nullptr, 0, s, &nb);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    ms /= 3.f;
    if (times_ms) times_ms[c] = ms;
    if (err == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = c;
    }
    if (err == hipSuccess && c < NUM_BLUR_CFG && ms < best_valu_ms) {
      best_valu_ms = ms;
      best_valu = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  P.blur_cfg = best;
  P.blur_cfg_valu = best_valu;
  return err;
}

// The two forms of w = A^T A p + lam2 p (p . w partials included): the
// direct blurs (A p into q, then the normal epilogue) and the FFT passes.
// Each is timed over 3 launches after one warm-up on the scratch vector p
// (zeros) and the faster is kept; kp_set_normal_op overrides the choice.
hipError_t launch_normal_direct(const Plan& P, const float* p, float* w, float lam2,
                                hipStream_t s, int* nb) {
  hipError_t e = launch_blur_f32(P, p, P.q, false, s, nullptr);
  if (e != hipSuccess) return e;
  EpiNormalW en{p, w, lam2, P.n};
  return blur_dispatch(P.blur_cfg, P, P.q, P.taps32, en, nullptr, 0, s, nb);
}

hipError_t autotune_normal(Plan& P, hipStream_t s) {
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return err;
  err = hipEventCreate(&e1);
  if (err != hipSuccess) {
    hipEventDestroy(e0);
    return err;
  }
  const float lam2 = 1e-4f;
  // the FFT form covers the zero and reflexive boundaries; with a PSF that
  // is not symmetric the reflexive A^T is no blur and the FFT form is the
  // only one
  const int op0 = P.refl_general ? 1 : 0;
  const int nops = (P.fft_L > 0 && (P.bc == KP_BC_ZERO || P.bc == KP_BC_REFLEXIVE)) ? 2 : 1;
  P.normal_times[0] = P.normal_times[1] = 0.f;
  for (int op = op0; op < nops && err == hipSuccess; ++op) {
    auto run = [&]() {
      int nb;
      return op == 0 ? launch_normal_direct(P, P.p, P.w, lam2, s, &nb)
                     : launch_fft_normal(P, P.p, P.w, lam2, s, &nb, nullptr);
    };
    err = run();
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int it = 0; it < 3 && err == hipSuccess; ++it) err = run();
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    P.normal_times[op] = ms / 3.f;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  P.normal_op = P.refl_general ? 1
                : (err == hipSuccess && nops == 2 && P.normal_times[1] < P.normal_times[0]) ? 1
                                                                                          : 0;
  return err;
}

hipError_t launch_rhs(const Plan& P, const float* b, bool zero_x, hipStream_t s) {
  if (P.refl_general) return launch_fft_rhs(P, b, zero_x, s);
  EpiRhs e{P.r, P.n, P.p, P.w, zero_x ? P.x64 : nullptr};
  int nb;
  hipError_t err = blur_dispatch(P.blur_cfg, P, b, P.taps32, e, P.ctrl, 0, s, &nb);
  if (err != hipSuccess) return err;
  return launch_scalar(P, SC_RHS, nb, s);
}

hipError_t launch_true_residual(const Plan& P, const float* b, const double* x, double lam2,
                                bool fin, int trmode, hipStream_t s) {
  const bool fast = trmode != TR_FP64;
  hipError_t err;
  if (trmode == TR_FAST_ALL) {
    // u = b - A fp32(x) on the plan's blur, into q (z holds fp32(x))
    err = launch_convert_x(P, P.z, true, s);
    if (err != hipSuccess) return err;
    EpiResid e1{b, P.q, nullptr, P.n};
    int nb1;
    err = blur_dispatch(P.blur_cfg, P, P.z, P.taps32_flip, e1, P.ctrl, 0, s, &nb1);
  } else {
    // u = b - A x (FP64 accumulation) into q (FP32) or y64 (FP64)
    EpiResid e1{b, fast ? P.q : nullptr, fast ? nullptr : P.y64, P.n};
    err = run_blur<KP_F64IN_CFG, double, double, double>(P, x, P.taps64_flip, e1, P.ctrl, 0, s);
  }
  if (err != hipSuccess) return err;
  if (P.refl_general) {
    // A^T of the reflexive boundary with a PSF that is not symmetric: the
    // folded correlation by FFTs, on u in q (the solver refuses TR_FP64)
    if (!fast) return hipErrorInvalidValue;
    return launch_fft_true_res(P, lam2, fin, s);
  }
  EpiTrueRes e2{x, P.r, lam2, P.n, P.xa64, P.ra64};
  int nb;
  if (fast) {
    err = blur_dispatch(P.blur_cfg, P, P.q, P.taps32, e2, P.ctrl, 0, s, &nb);
  } else {
    nb = blur_blocks<KP_F64IN_CFG>(P.n);
    err = run_blur<KP_F64IN_CFG, double, double, double>(P, P.y64, P.taps64, e2, P.ctrl, 0, s);
  }
  if (err != hipSuccess) return err;
  return launch_scalar(P, fin ? SC_TRUE : SC_TRUE_INFO, nb, s);
}

hipError_t launch_anchor_residual(const Plan& P, double lam2, bool fin, hipStream_t s) {
  // H (x - x_a) in the form the iterations use (the FFT passes: one H p
  // instead of the two blurs)
  if (P.refl_general || P.normal_op == KP_NORMAL_FFT)
    return launch_fft_anchor_residual(P, lam2, fin, s);
  // q = fp32(x - x_a), z = A q, r = r_a - A^T z - lam2 (x - x_a)
  hipError_t err = launch_diff32(P, P.q, s);
  if (err != hipSuccess) return err;
  err = launch_blur_f32(P, P.q, P.z, false, s, nullptr);
  if (err != hipSuccess) return err;
  EpiAnchorRes e{P.x64, P.xa64, P.ra64, P.r, lam2, P.n};
  int nb;
  err = blur_dispatch(P.blur_cfg, P, P.z, P.taps32, e, P.ctrl, 0, s, &nb);
  if (err != hipSuccess) return err;
  return launch_scalar(P, fin ? SC_TRUE : SC_TRUE_INFO, nb, s);
}

// y = (A^T A + lam2 I) x with FP64 accumulation (test entry point)
struct EpiNormal64 {
  const float* x; double* y; double lam2; int n;
  static constexpr bool kReduce = false;
  static constexpr int kSlot = SLOT_NORM;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double&) const {
    const size_t o = (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) y[o + c] = (double)v[c] + lam2 * (double)x[o + c];
  }
};

hipError_t launch_normal_fp64(const Plan& P, const float* x, double lam2, double* y,
                              hipStream_t s) {
  EpiStoreF64 e1{P.y64, P.n};
  hipError_t err =
      run_blur<KP_F32_CFG, float, double, double>(P, x, P.taps64_flip, e1, P.ctrl, 0, s);
  if (err != hipSuccess) return err;
  EpiNormal64 e2{x, y, lam2, P.n};
  return run_blur<KP_F64IN_CFG, double, double, double>(P, P.y64, P.taps64, e2, P.ctrl, 0, s);
}

}  // namespace kpcg
