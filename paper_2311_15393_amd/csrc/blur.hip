// Direct-convolution matvecs with the blur A and its transpose.
//
// The paper applies A and A^T through structured matvecs and names them the
// most expensive part of an iteration (Section 5.2, work-unit model).  Here
// they are zero-boundary 2-D correlations computed directly:
//     out[i][j] = sum_{a,b < K} Q[a][b] in[i + a - h][j + b - h]
// with Q = P for A^T and Q = P rotated by 180 degrees for A.
//
// Design (gfx950): one workgroup per TH x TW output tile stages the
// (TH+K-1) x (TW+KQ) input halo tile in LDS with coalesced global loads and
// zero fill outside the image.  Each thread owns RY rows x RX consecutive
// columns.  The tap loop walks input rows once ("row sweep"): a window of
// RX+BC-1 inputs is read from LDS with 16-byte loads and reused by RX*BC
// FMAs for each of the RY output rows it feeds, with taps read as
// wave-uniform values.  Taps are padded to KQ = ceil(K/BC)*BC columns with
// zeros.  The work is FP32-VALU bound (K^2/4 flop per byte moved).
#include "common.h"

namespace kpcg {

template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int N = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int N = 2; };

template <typename Acc, typename In, int W>
__device__ inline void load_window(const In* __restrict__ sp, Acc (&win)[W]) {
  using V = typename Vec16<In>::type;
  constexpr int NV = Vec16<In>::N;
  static_assert(W % NV == 0, "window must be a whole number of 16-byte loads");
#pragma unroll
  for (int m = 0; m < W / NV; ++m) {
    const V v = *reinterpret_cast<const V*>(sp + m * NV);
    if constexpr (NV == 4) {
      win[4 * m + 0] = (Acc)v.x; win[4 * m + 1] = (Acc)v.y;
      win[4 * m + 2] = (Acc)v.z; win[4 * m + 3] = (Acc)v.w;
    } else {
      win[2 * m + 0] = (Acc)v.x; win[2 * m + 1] = (Acc)v.y;
    }
  }
}

// ---------------------------------------------------------------------------
// epilogues
// ---------------------------------------------------------------------------
struct EpiStoreF32 {
  float* dst; int n;
  static constexpr bool kReduce = false;
  static constexpr int kSlot = SLOT_NORM;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double&) const {
    float* o = dst + (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) o[c] = (float)v[c];
  }
};

struct EpiStoreF64 {
  double* dst; int n;
  static constexpr bool kReduce = false;
  static constexpr int kSlot = SLOT_NORM;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double&) const {
    double* o = dst + (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) o[c] = (double)v[c];
  }
};

// w = A^T q + lambda^2 p and delta = p . w  (the H p product of CG)
struct EpiNormalW {
  const float* p; float* w; float lam2; int n;
  static constexpr bool kReduce = true;
  static constexpr int kSlot = SLOT_DELTA;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double& d) const {
    const size_t o = (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) {
      const float pv = p[o + c];
      const float wv = fmaf(lam2, pv, (float)v[c]);
      w[o + c] = wv;
      d += (double)pv * (double)wv;
    }
  }
};

// c = A^T b in FP64, r_0 = (float) c, ||c||^2
struct EpiRhs {
  double* c64; float* r; int n;
  static constexpr bool kReduce = true;
  static constexpr int kSlot = SLOT_RHS;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double& d) const {
    const size_t o = (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) {
      const double cv = (double)v[c];
      c64[o + c] = cv;
      r[o + c] = (float)cv;
      d += cv * cv;
    }
  }
};

// r = c - A^T y - lambda^2 x with y = A x in FP64: the true residual
struct EpiTrueRes {
  const double* c64; const double* x; float* r; double lam2; int n;
  static constexpr bool kReduce = true;
  static constexpr int kSlot = SLOT_TRUE;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double& d) const {
    const size_t o = (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) {
      const double rv = c64[o + c] - (double)v[c] - lam2 * x[o + c];
      r[o + c] = (float)rv;
      d += rv * rv;
    }
  }
};

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <int TX, int TY, int RX, int RY, int BC, typename In, typename Acc, typename Tap,
          class Epi>
__global__ __launch_bounds__(TX* TY) void blur_kernel(
    const In* __restrict__ src, const Tap* __restrict__ taps, int n, int K, int KQ, int LDW,
    Epi epi, Ctrl* ctrl, int skip_if_done, double* partials) {
  constexpr int NT = TX * TY;
  constexpr int TW = TX * RX, TH = TY * RY;
  constexpr int WIN = RX + BC;   // RX + BC - 1 inputs used, one pad entry
  if (skip_if_done && ctrl->done != RUNNING) return;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  In* s = reinterpret_cast<In*>(smem_raw);
  const int h = (K - 1) >> 1;
  const int ti0 = blockIdx.y * TH, tj0 = blockIdx.x * TW;
  const int rows = TH + K - 1;
  const int cvalid = TW + K - 1;

  for (int idx = threadIdx.x; idx < rows * LDW; idx += NT) {
    const int r = idx / LDW, c = idx - r * LDW;
    const int gi = ti0 - h + r, gj = tj0 - h + c;
    In v = In(0);
    if (c < cvalid && (unsigned)gi < (unsigned)n && (unsigned)gj < (unsigned)n)
      v = src[(size_t)gi * n + gj];
    s[idx] = v;
  }
  __syncthreads();

  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  Acc acc[RY][RX];
#pragma unroll
  for (int ry = 0; ry < RY; ++ry)
#pragma unroll
    for (int rx = 0; rx < RX; ++rx) acc[ry][rx] = Acc(0);

  const In* sbase = s + (ty * RY) * LDW + tx * RX;
  for (int t = 0; t < K + RY - 1; ++t) {
    const In* srow = sbase + t * LDW;
    for (int b0 = 0; b0 < KQ; b0 += BC) {
      Acc win[WIN];
      load_window<Acc, In, WIN>(srow + b0, win);
#pragma unroll
      for (int ry = 0; ry < RY; ++ry) {
        const int a = t - ry;
        if (a < 0 || a >= K) continue;
        const Tap* q = taps + a * KQ + b0;
#pragma unroll
        for (int b = 0; b < BC; ++b) {
          const Acc tb = (Acc)q[b];
#pragma unroll
          for (int rx = 0; rx < RX; ++rx) acc[ry][rx] = fma(tb, win[rx + b], acc[ry][rx]);
        }
      }
    }
  }

  double d = 0.0;
#pragma unroll
  for (int ry = 0; ry < RY; ++ry) {
    const int i = ti0 + ty * RY + ry;
    const int j0 = tj0 + tx * RX;
    if (i < n && j0 < n) epi.row(i, j0, min(RX, n - j0), acc[ry], d);
  }
  if constexpr (Epi::kReduce) {
    __shared__ double sh[NT / 64];
    const double v1[1] = {block_sum<NT>(d, sh)};
    write_partials<1>(v1, partials, Epi::kSlot, blockIdx.y * gridDim.x + blockIdx.x);
  }
}

// ---------------------------------------------------------------------------
// launch configurations
// ---------------------------------------------------------------------------
constexpr int BC = 16;

template <int TX, int TY, int RX, int RY, typename In>
static int lds_width(int kq) {
  constexpr int TW = TX * RX;
  int w = TW + kq;                    // window reads reach column TW + kq - 1
  constexpr int NV = 16 / (int)sizeof(In);
  w = (w + NV - 1) / NV * NV;
  return w;
}

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
                     skip, P.partials);
  return hipGetLastError();
}

template <int TX, int TY, int RX, int RY>
static int blur_blocks(int n) {
  return ((n + TX * RX - 1) / (TX * RX)) * ((n + TY * RY - 1) / (TY * RY));
}

// FP32 tile shapes (TX threads across x RX columns each, TY threads down x
// RY rows each); the plan picks the fastest for its (n, K) at setup.
#define KP_CFG0 8, 32, 8, 1     // 64 x 32 tile, 256 threads
#define KP_CFG1 8, 16, 8, 1     // 64 x 16 tile, 128 threads
#define KP_CFG2 8, 32, 8, 2     // 64 x 64 tile, 256 threads, 2 rows / thread
#define KP_CFG3 16, 16, 8, 1    // 128 x 16 tile, 256 threads
#define KP_CFG4 8, 64, 8, 1     // 64 x 64 tile, 512 threads
#define KP_CFG5 16, 16, 4, 2    // 64 x 32 tile, 256 threads, 4 x 2 per thread
constexpr int NUM_BLUR_CFG = 6;
// FP32 input, FP64 accumulation (right-hand side)
#define KP_F32_CFG KP_CFG0
// FP64-input tiles (true residual): 64 x 64 outputs, 512 threads, 129 KB LDS at K = 63
#define KP_F64IN_CFG 8, 64, 8, 1

template <class Epi>
static hipError_t blur_dispatch(int cfg, const Plan& P, const float* src, const float* taps,
                                Epi epi, Ctrl* ctrl, int skip, hipStream_t s, int* nb) {
  const int n = P.n;
  switch (cfg) {
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
  EpiStoreF32 e{dst, P.n};
  int nb;
  return blur_dispatch(P.blur_cfg, P, src, transpose ? P.taps32 : P.taps32_flip, e,
                       const_cast<Ctrl*>(ctrl), ctrl != nullptr, s, &nb);
}

hipError_t launch_blur_normal(const Plan& P, const float* q, const float* p, float* w,
                              float lam2, hipStream_t s) {
  EpiNormalW e{p, w, lam2, P.n};
  int nb;
  hipError_t err = blur_dispatch(P.blur_cfg, P, q, P.taps32, e, P.ctrl, 1, s, &nb);
  if (err != hipSuccess) return err;
  return launch_scalar(P, SC_ALPHA, nb, s);
}

// Autotuner: time every FP32 tile shape on this plan's (n, K) and keep the
// fastest (3 timed launches each after one warm-up; scratch vectors p, q).
hipError_t autotune_blur(Plan& P, hipStream_t s, float* times_ms) {
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return err;
  err = hipEventCreate(&e1);
  if (err != hipSuccess) return err;
  err = hipMemsetAsync(P.p, 0, sizeof(float) * (size_t)P.n * P.n, s);
  int best = 0;
  float best_ms = 1e30f;
  for (int c = 0; c < NUM_BLUR_CFG && err == hipSuccess; ++c) {
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
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  P.blur_cfg = best;
  return err;
}

hipError_t launch_rhs(const Plan& P, const float* b, hipStream_t s) {
  EpiRhs e{P.c64, P.r, P.n};
  hipError_t err = run_blur<KP_F32_CFG, float, double, double>(P, b, P.taps64, e, P.ctrl, 0, s);
  if (err != hipSuccess) return err;
  return launch_scalar(P, SC_RHS, blur_blocks<KP_F32_CFG>(P.n), s);
}

hipError_t launch_true_residual(const Plan& P, const double* x, double lam2, bool fin,
                                hipStream_t s) {
  EpiStoreF64 e1{P.y64, P.n};
  hipError_t err =
      run_blur<KP_F64IN_CFG, double, double, double>(P, x, P.taps64_flip, e1, P.ctrl, 0, s);
  if (err != hipSuccess) return err;
  EpiTrueRes e2{P.c64, x, P.r, lam2, P.n};
  err = run_blur<KP_F64IN_CFG, double, double, double>(P, P.y64, P.taps64, e2, P.ctrl, 0, s);
  if (err != hipSuccess) return err;
  return launch_scalar(P, fin ? SC_TRUE : SC_TRUE_INFO, blur_blocks<KP_F64IN_CFG>(P.n), s);
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
