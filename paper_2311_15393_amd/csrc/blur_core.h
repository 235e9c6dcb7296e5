// Shared body of the direct-convolution blur kernels (single-problem and
// batched launches): one workgroup computes one TH x TW output tile.
//
//     out[i][j] = sum_{a,b < K} Q[a][b] in[i + a - h][j + b - h]
//
// with Q = P for A^T and Q = P rotated by 180 degrees for A (zero boundary).
// The (TH+K-1) x (TW+KQ) input halo tile is staged in LDS with coalesced
// global loads and zero fill outside the image.  Each thread owns RY rows x
// RX consecutive columns; the tap loop walks input rows once, reading a
// window of RX+BC-1 inputs with 16-byte LDS loads and reusing it for RX*BC
// FMAs per output row it feeds, with taps read as wave-uniform (scalar)
// values.  Taps are padded to KQ = ceil(K/BC)*BC columns with zeros.
#pragma once

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

// r_0 = c = A^T b and ||c||^2.  c only seeds the recursion: every true
// residual is formed from b directly (EpiResid, EpiTrueRes), so an FP32-class
// blur suffices here.
// Optionally it also clears the solver's p, w and x (x_0 = 0) at the same
// positions, saving separate fills.
struct EpiRhs {
  float* r; int n;
  float* p0 = nullptr; float* w0 = nullptr; double* x0 = nullptr;
  static constexpr bool kReduce = true;
  static constexpr int kSlot = SLOT_RHS;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double& d) const {
    const size_t o = (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) {
      const double cv = (double)v[c];
      r[o + c] = (float)cv;
      d += cv * cv;
      if (p0) {
        p0[o + c] = 0.0f;
        w0[o + c] = 0.0f;
      }
      if (x0) x0[o + c] = 0.0;
    }
  }
};

// u = b - A x with A x accumulated in FP64: the data residual, stored as FP32
// (input of the FP32-class A^T) and/or FP64 (input of the FP64 A^T)
struct EpiResid {
  const float* b; float* u32; double* u64; int n;
  static constexpr bool kReduce = false;
  static constexpr int kSlot = SLOT_NORM;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double&) const {
    const size_t o = (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) {
      const double uv = (double)b[o + c] - (double)v[c];
      if (u32) u32[o + c] = (float)uv;
      if (u64) u64[o + c] = uv;
    }
  }
};

// r = A^T u - lambda^2 x with u = b - A x (EpiResid): the true residual of the
// normal equations, A^T(b - A x) - lambda^2 x = c - H x, without forming the
// difference of the two large terms c and H x.  The epilogue is FP64; v comes
// from either blur.  Also records (x, r) in FP64 as the anchor of later
// residuals (EpiAnchorRes).
struct EpiTrueRes {
  const double* x; float* r; double lam2; int n;
  double* xa = nullptr; double* ra = nullptr;
  static constexpr bool kReduce = true;
  static constexpr int kSlot = SLOT_TRUE;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double& d) const {
    const size_t o = (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) {
      const double xv = x[o + c];
      const double rv = (double)v[c] - lam2 * xv;
      r[o + c] = (float)rv;
      if (xa) {                        // anchor recorded unless not asked for
        xa[o + c] = xv;
        ra[o + c] = rv;
      }
      d += rv * rv;
    }
  }
};

// r = r_a - (A^T A dx + lambda^2 dx), dx = x - x_a: the true residual from
// the anchor, with v = A^T A fp32(dx) from the FP32 blur and the rest in
// FP64; the anchor moves to (x, r).  Pointwise in ra / xa, so the in-place
// update is safe.
struct EpiAnchorRes {
  const double* x; double* xa; double* ra; float* r; double lam2; int n;
  static constexpr bool kReduce = true;
  static constexpr int kSlot = SLOT_TRUE;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double& d) const {
    const size_t o = (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) {
      const double xv = x[o + c];
      const double rv = ra[o + c] - ((double)v[c] + lam2 * (xv - xa[o + c]));
      r[o + c] = (float)rv;
      xa[o + c] = xv;
      ra[o + c] = rv;
      d += rv * rv;
    }
  }
};

// Source row or column of a staged tile entry.  The zero boundary keeps the
// index (out-of-range entries are zero-filled by the caller); the periodic
// boundary (KP_BC_PERIODIC) wraps it by one period and the reflexive one
// (KP_BC_REFLEXIVE) reflects it once about the half-sample edge (-1 -> 0,
// n -> n - 1), which covers every entry that feeds an output inside the
// image (|index - [0, n)| <= h < n); entries further out only feed the
// discarded outputs of edge tiles and are clamped.
template <int BCV>
__device__ inline int bc_index_c(int g, int n) {
  if constexpr (BCV == KP_BC_ZERO) return g;
  if constexpr (BCV == KP_BC_PERIODIC) g = g < 0 ? g + n : (g >= n ? g - n : g);
  else g = g < 0 ? -g - 1 : (g >= n ? 2 * n - 1 - g : g);
  return g < 0 ? 0 : (g >= n ? n - 1 : g);
}
__device__ inline int bc_index(int g, int n, int bc) {
  if (bc == KP_BC_ZERO) return bc_index_c<KP_BC_ZERO>(g, n);
  if (bc == KP_BC_PERIODIC) return bc_index_c<KP_BC_PERIODIC>(g, n);
  return bc_index_c<KP_BC_REFLEXIVE>(g, n);
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <int TX, int TY, int RX, int RY, int BC, typename In, typename Acc, typename Tap,
          class Epi>
__device__ inline void blur_tile(const In* __restrict__ src, const Tap* __restrict__ taps,
                                 int n, int K, int KQ, int LDW, int ti0, int tj0, Epi epi,
                                 double* partial_out, int bc = 0) {
  constexpr int NT = TX * TY;
  constexpr int TW = TX * RX, TH = TY * RY;
  constexpr int WIN = RX + BC;   // RX + BC - 1 inputs used, one pad entry
  extern __shared__ __align__(16) unsigned char smem_raw[];
  In* s = reinterpret_cast<In*>(smem_raw);
  const int h = (K - 1) >> 1;
  const int rows = TH + K - 1;
  const int cvalid = TW + K - 1;

  for (int idx = threadIdx.x; idx < rows * LDW; idx += NT) {
    const int r = idx / LDW, c = idx - r * LDW;
    const int gi = bc_index(ti0 - h + r, n, bc), gj = bc_index(tj0 - h + c, n, bc);
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
    if (threadIdx.x == 0) *partial_out = v1[0];
  }
}

// FP32 tile shapes (TX threads across x RX columns each, TY threads down x
// RY rows each); the plan picks the fastest for its (n, K) at setup.
#define KP_CFG0 8, 32, 8, 1     // 64 x 32 tile, 256 threads
#define KP_CFG1 8, 16, 8, 1     // 64 x 16 tile, 128 threads
#define KP_CFG2 8, 32, 8, 2     // 64 x 64 tile, 256 threads, 2 rows / thread
#define KP_CFG3 16, 16, 8, 1    // 128 x 16 tile, 256 threads
#define KP_CFG4 8, 64, 8, 1     // 64 x 64 tile, 512 threads
#define KP_CFG5 16, 16, 4, 2    // 64 x 32 tile, 256 threads, 4 x 2 per thread
constexpr int NUM_BLUR_CFG = 6;        // FP32-VALU tile shapes
constexpr int BLUR_CFG_MFMA = 6;       // the MFMA kernel (blur_mfma.hip), 16 x 16 x 32
constexpr int BLUR_CFG_MFMA32 = 7;     // the MFMA kernel on 32 x 32 x 16
__host__ __device__ constexpr bool blur_cfg_is_mfma(int cfg) { return cfg >= BLUR_CFG_MFMA; }
constexpr int BC = 16;
// FP32 input, FP64 accumulation (right-hand side)
#define KP_F32_CFG KP_CFG0
// FP64-input tiles (true residual): 64 x 64 outputs, 512 threads, 129 KB LDS at K = 63
#define KP_F64IN_CFG 8, 64, 8, 1


template <int TX, int TY, int RX, int RY, typename In>
__host__ __device__ inline int lds_width(int kq) {
  constexpr int TW = TX * RX;
  int w = TW + kq;                    // window reads reach column TW + kq - 1
  constexpr int NV = 16 / (int)sizeof(In);
  w = (w + NV - 1) / NV * NV;
  return w;
}

// the MFMA blur (blur_mfma.hip): A^T if transpose, else A
template <class Epi>
hipError_t launch_blur_mfma(const Plan& P, const float* src, bool transpose, Epi epi,
                            Ctrl* ctrl, int skip, hipStream_t s);
template <class Epi>
hipError_t launch_blur_mfma32(const Plan& P, const float* src, bool transpose, Epi epi,
                              Ctrl* ctrl, int skip, hipStream_t s);

}  // namespace kpcg
