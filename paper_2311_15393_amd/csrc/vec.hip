// Fused vector kernels of the (P)CG iteration.
//
// The paper keeps everything outside the preconditioner solve in double
// precision (Section 1, mixed-precision paragraph).  Here the vectors are
// FP32 in HBM and every scalar that steers the iteration (||r||^2, alpha,
// beta, the convergence test) is accumulated and kept in FP64 on the device.
// These kernels are HBM-bound: 16-byte accesses, grid-stride loops with a
// fixed grid so the FP64 reductions are deterministic.
#include "common.h"

namespace kpcg {

constexpr int VT = 256;          // threads per block
constexpr int VMAXB = 512;       // blocks per vector kernel

static inline int vec_blocks(int n4) {
  int b = (n4 + VT - 1) / VT;
  return b < 1 ? 1 : (b > VMAXB ? VMAXB : b);
}

// x += alpha p (FP64 accumulator) ; r -= alpha w ; ||r||^2 (partials)
__device__ inline void update_body(double* __restrict__ x, float* __restrict__ r,
                                   const float* __restrict__ p, const float* __restrict__ w,
                                   int N, double ad, double* partials) {
  const float a = (float)ad;
  const int n4 = N >> 2;
  double d = 0.0;
  double2* x2 = reinterpret_cast<double2*>(x);
  float4* r4 = reinterpret_cast<float4*>(r);
  const float4* p4 = reinterpret_cast<const float4*>(p);
  const float4* w4 = reinterpret_cast<const float4*>(w);
  for (int i = blockIdx.x * VT + threadIdx.x; i < n4; i += gridDim.x * VT) {
    double2 xa = x2[2 * i], xb = x2[2 * i + 1];
    float4 rv = r4[i];
    const float4 pv = p4[i], wv = w4[i];
    xa.x = fma(ad, (double)pv.x, xa.x); xa.y = fma(ad, (double)pv.y, xa.y);
    xb.x = fma(ad, (double)pv.z, xb.x); xb.y = fma(ad, (double)pv.w, xb.y);
    rv.x = fmaf(-a, wv.x, rv.x); rv.y = fmaf(-a, wv.y, rv.y);
    rv.z = fmaf(-a, wv.z, rv.z); rv.w = fmaf(-a, wv.w, rv.w);
    x2[2 * i] = xa;
    x2[2 * i + 1] = xb;
    r4[i] = rv;
    d += (double)rv.x * rv.x + (double)rv.y * rv.y + (double)rv.z * rv.z +
         (double)rv.w * rv.w;
  }
  if (blockIdx.x == 0) {
    for (int i = 4 * n4 + threadIdx.x; i < N; i += VT) {
      x[i] = fma(ad, (double)p[i], x[i]);
      const float rv = fmaf(-a, w[i], r[i]);
      r[i] = rv;
      d += (double)rv * rv;
    }
  }
  __shared__ double sh[VT / 64];
  const double v1[1] = {block_sum<VT>(d, sh)};
  write_partials<1>(v1, partials, SLOT_RR, blockIdx.x);
}

__global__ __launch_bounds__(VT) void update_kernel(double* __restrict__ x,
                                                    float* __restrict__ r,
                                                    const float* __restrict__ p,
                                                    const float* __restrict__ w, int N,
                                                    Ctrl* ctrl, double* partials) {
  if (ctrl->done != RUNNING) return;
  update_body(x, r, p, w, N, ctrl->alpha, partials);
}

// p = z + beta p
__global__ __launch_bounds__(VT) void pupdate_kernel(float* __restrict__ p,
                                                     const float* __restrict__ z, int N,
                                                     const Ctrl* __restrict__ ctrl) {
  if (ctrl->done != RUNNING) return;
  const float b = (float)ctrl->beta;
  const int n4 = N >> 2;
  float4* p4 = reinterpret_cast<float4*>(p);
  const float4* z4 = reinterpret_cast<const float4*>(z);
  for (int i = blockIdx.x * VT + threadIdx.x; i < n4; i += gridDim.x * VT) {
    float4 pv = p4[i];
    const float4 zv = z4[i];
    pv.x = fmaf(b, pv.x, zv.x); pv.y = fmaf(b, pv.y, zv.y);
    pv.z = fmaf(b, pv.z, zv.z); pv.w = fmaf(b, pv.w, zv.w);
    p4[i] = pv;
  }
  if (blockIdx.x == 0)
    for (int i = 4 * n4 + threadIdx.x; i < N; i += VT) p[i] = fmaf(b, p[i], z[i]);
}

// The direction step folded into p = z + beta p: every block sums the nbz
// partials of r.z and z.Hp of the preconditioner's last GEMM (in the scalar
// step's order) and takes beta from them; block 0 stores r.z, z.Hp, beta
// (or the breakdown) and publishes.  The fields beta_of reads (first,
// fr_next, rho, delta) are written only by the step length that follows.
__global__ __launch_bounds__(VT) void pupdate_fold_kernel(float* __restrict__ p,
                                                          const float* __restrict__ z, int N,
                                                          Ctrl* ctrl,
                                                          const double* __restrict__ partials,
                                                          int nbz,
                                                          CtrlMirror* __restrict__ mirror) {
  if (ctrl->done != RUNNING) return;
  const StepIn kin = step_in(ctrl);
  __shared__ double sh[2 * fold_sh<VT>()];
  const double2 f = fold_slot2<VT>(partials, SLOT_RZ, SLOT_ZW, nbz, sh);
  const double rz = f.x, zw = f.y;
  bool ok;
  const double beta = beta_of(kin, rz, zw, &ok);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->rz = rz;
    ctrl->zw = zw;
    if (ok) ctrl->beta = beta;
    else ctrl->done = BREAKDOWN;
    if (mirror != nullptr) publish_mirror(ctrl, mirror);
  }
  if (!ok) return;
  const float b = (float)beta;
  const int n4 = N >> 2;
  float4* p4 = reinterpret_cast<float4*>(p);
  const float4* z4 = reinterpret_cast<const float4*>(z);
  for (int i = blockIdx.x * VT + threadIdx.x; i < n4; i += gridDim.x * VT) {
    float4 pv = p4[i];
    const float4 zv = z4[i];
    pv.x = fmaf(b, pv.x, zv.x); pv.y = fmaf(b, pv.y, zv.y);
    pv.z = fmaf(b, pv.z, zv.z); pv.w = fmaf(b, pv.w, zv.w);
    p4[i] = pv;
  }
  if (blockIdx.x == 0)
    for (int i = 4 * n4 + threadIdx.x; i < N; i += VT) p[i] = fmaf(b, p[i], z[i]);
}

// ||v||^2 -> rr and the preconditioner scales (standalone preconditioner use)
__global__ __launch_bounds__(VT) void norm_scale_kernel(const float* __restrict__ v, int N,
                                                        Ctrl* ctrl, double* partials) {
  double d = 0.0;
  for (int i = blockIdx.x * VT + threadIdx.x; i < N; i += gridDim.x * VT)
    d += (double)v[i] * v[i];
  __shared__ double sh[VT / 64];
  const double v1[1] = {block_sum<VT>(d, sh)};
  write_partials<1>(v1, partials, SLOT_NORM, blockIdx.x);
}

hipError_t launch_update(const Plan& P, bool rr_step, hipStream_t s) {
  const int N = P.n * P.n;
  const int nb = vec_blocks(N >> 2);
  hipLaunchKernelGGL(update_kernel, dim3(nb), dim3(VT), 0, s, P.x64, P.r, P.p, P.w, N, P.ctrl,
                     P.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !rr_step) return e;
  return launch_scalar(P, SC_RR, nb, s);
}

__global__ __launch_bounds__(VT) void convert_x_kernel(double* __restrict__ x64,
                                                       float* __restrict__ x, int N,
                                                       int to_f32) {
  for (int i = blockIdx.x * VT + threadIdx.x; i < N; i += gridDim.x * VT) {
    if (to_f32) x[i] = (float)x64[i];
    else x64[i] = (double)x[i];
  }
}

hipError_t launch_convert_x(const Plan& P, float* x, bool to_f32, hipStream_t s) {
  const int N = P.n * P.n;
  hipLaunchKernelGGL(convert_x_kernel, dim3(vec_blocks(N >> 2)), dim3(VT), 0, s, P.x64, x, N,
                     to_f32 ? 1 : 0);
  return hipGetLastError();
}

__global__ void init_ctrl_kernel(Ctrl* __restrict__ c, Ctrl v) {
  if (threadIdx.x == 0) *c = v;
}

hipError_t launch_init_ctrl(const Plan& P, const Ctrl& c, hipStream_t s) {
  hipLaunchKernelGGL(init_ctrl_kernel, dim3(1), dim3(64), 0, s, P.ctrl, c);
  return hipGetLastError();
}

// d = fp32(x - x_a): the step since the anchor
__global__ __launch_bounds__(VT) void diff32_kernel(const double* __restrict__ x64,
                                                    const double* __restrict__ xa64,
                                                    float* __restrict__ d, int N) {
  for (int i = blockIdx.x * VT + threadIdx.x; i < N; i += gridDim.x * VT)
    d[i] = (float)(x64[i] - xa64[i]);
}

hipError_t launch_diff32(const Plan& P, float* d, hipStream_t s) {
  const int N = P.n * P.n;
  hipLaunchKernelGGL(diff32_kernel, dim3(vec_blocks(N >> 2)), dim3(VT), 0, s, P.x64, P.xa64, d,
                     N);
  return hipGetLastError();
}

hipError_t launch_pupdate_from(const Plan& P, const float* z, hipStream_t s) {
  const int N = P.n * P.n;
  hipLaunchKernelGGL(pupdate_kernel, dim3(vec_blocks(N >> 2)), dim3(VT), 0, s, P.p, z, N,
                     P.ctrl);
  return hipGetLastError();
}

hipError_t launch_pupdate_fold(const Plan& P, const float* z, int nbz, hipStream_t s) {
  if (nbz > MAX_PARTIALS) return hipErrorInvalidValue;
  const int N = P.n * P.n;
  hipLaunchKernelGGL(pupdate_fold_kernel, dim3(vec_blocks(N >> 2)), dim3(VT), 0, s, P.p, z, N,
                     P.ctrl, P.partials, nbz, P.mirror_dev);
  return hipGetLastError();
}

hipError_t launch_pupdate(const Plan& P, hipStream_t s) {
  return launch_pupdate_from(P, P.z, s);
}

hipError_t launch_norm_scale(const Plan& P, const float* v, hipStream_t s) {
  const int N = P.n * P.n;
  const int nb = vec_blocks(N >> 2);
  hipLaunchKernelGGL(norm_scale_kernel, dim3(nb), dim3(VT), 0, s, v, N, P.ctrl, P.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_scalar(P, SC_NORM, nb, s);
}

// ---------------------------------------------------------------------------
// scalar kernel: one block sums the partials of the kernel before it in a
// fixed order and applies the (P)CG scalar logic; thread 0 updates Ctrl
// ---------------------------------------------------------------------------
constexpr int ST = 256;

__device__ inline double sum_slot(const double* partials, int slot, int nb, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += ST) s += partials[slot * MAX_PARTIALS + i];
  return block_sum<ST>(s, sh);
}

// Every step that the host follows (the residual norm after an update, the
// direction step, the right-hand side, true residuals, and a breakdown found
// by the step length) publishes the new state to the host mirror.
__global__ __launch_bounds__(ST) void scalar_kernel(Ctrl* __restrict__ c,
                                                    const double* __restrict__ partials,
                                                    int kind, int nb,
                                                    CtrlMirror* __restrict__ mirror) {
  __shared__ double sh[ST / 64];
  const int done = c->done;
  if ((kind == SC_ALPHA || kind == SC_RR) && done != RUNNING) return;
  const int slot = kind == SC_ALPHA ? SLOT_DELTA
                 : kind == SC_RR ? SLOT_RR
                 : kind == SC_RHS ? SLOT_RHS
                 : kind == SC_NORM ? SLOT_NORM : SLOT_TRUE;
  const double S = sum_slot(partials, slot, nb, sh);
  if (threadIdx.x != 0) return;
  switch (kind) {
    case SC_ALPHA:                          // delta = p . Hp
      c->delta = S;
      if (!(S > 0.0) || !isfinite(S)) {
        c->done = BREAKDOWN;
      } else {
        c->alpha = step_rho(c) / S;
        commit_direction(c);
      }
      break;
    case SC_RR:                             // after x += alpha p, r -= alpha w
      apply_rr(c, S);                       // (records the history itself)
      break;
    case SC_RHS:                            // c = A^T b
      c->gamma0sq = S;
      c->rr = S;
      c->rho = S;
      c->tol2 = c->tol_rel2 * S;
      c->repl2 = REPLACE_DROP * REPLACE_DROP * S;
      set_scales(c, S);
      // zero data: x = 0 is the solution; non-finite data: nothing to do
      if (!(S > 0.0)) c->done = S == 0.0 ? CONVERGED : BREAKDOWN;
      else if (!isfinite(S)) c->done = BREAKDOWN;
      break;
    case SC_TRUE:                           // r = c - H x replaced the recurrence
      c->true_rr = S;
      c->rr = S;
      c->repl2 = REPLACE_DROP * REPLACE_DROP * S;
      set_scales(c, S);
      if (c->solver == KP_CG) {
        if (done == PENDING) c->beta = S / c->rho_prev;
        c->rho = S;
      } else {
        c->fr_next = 1;
      }
      if (!isfinite(S)) c->done = BREAKDOWN;
      else if (S <= c->tol2) c->done = CONVERGED;
      else if (done == PENDING) c->done = RUNNING;
      c->repl += 1;
      break;
    case SC_TRUE_INFO:
      c->true_rr = S;
      break;
    case SC_NORM:
      c->rr = S;
      set_scales(c, S);
      break;
  }
  // KP_HIST: r_0 = c (the recurrence norms after each iteration are
  // recorded by apply_rr), and every true residual at the iteration it was
  // formed
  double* hist = c->hist;
  const int it = c->iter;
  if (hist != nullptr && it >= 0 && it < KP_HIST_MAX) {
    if (kind == SC_RHS) hist[it] = S;
    else if (kind == SC_TRUE || kind == SC_TRUE_INFO) hist[KP_HIST_MAX + it] = S;
  }
  const bool publish = kind == SC_RR || kind == SC_RHS || kind == SC_TRUE ||
                       kind == SC_TRUE_INFO || (kind == SC_ALPHA && c->done != RUNNING);
  if (mirror != nullptr && publish) publish_mirror(c, mirror);
}

__global__ __launch_bounds__(VT) void fill_f64_kernel(double* __restrict__ a, int count,
                                                      double v) {
  for (int i = blockIdx.x * VT + threadIdx.x; i < count; i += gridDim.x * VT) a[i] = v;
}

hipError_t launch_fill_f64(double* a, int count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(vec_blocks(count)), dim3(VT), 0, s, a, count, v);
  return hipGetLastError();
}

// The step length fused into the update: every block sums the nbd
// partials of p.Hp in the scalar step's order (ST == VT threads, the same
// block_sum), so all blocks hold the same delta and alpha = rho / delta;
// block 0 stores them (and a breakdown, which it publishes).  No block
// reads a control-block field that block 0 writes here.
static_assert(ST == VT, "the fused step must reduce in the scalar step's order");
__global__ __launch_bounds__(VT) void update_alpha_kernel(double* __restrict__ x,
                                                          float* __restrict__ r,
                                                          const float* __restrict__ p,
                                                          const float* __restrict__ w, int N,
                                                          Ctrl* ctrl, double* partials, int nbd,
                                                          CtrlMirror* __restrict__ mirror) {
  if (ctrl->done != RUNNING) return;
  const StepIn kin = step_in(ctrl);
  __shared__ double shd[VT / 64];
  __shared__ double s_delta;
  const double S0 = sum_slot(partials, SLOT_DELTA, nbd, shd);     // valid in thread 0
  if (threadIdx.x == 0) s_delta = S0;
  __syncthreads();
  const double S = s_delta;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (!(S > 0.0) || !isfinite(S)) {
    if (lead) {
      ctrl->delta = S;
      ctrl->done = BREAKDOWN;
      if (mirror != nullptr) publish_mirror(ctrl, mirror);
    }
    return;
  }
  const double ad = step_rho(kin) / S;
  if (lead) {
    ctrl->delta = S;
    ctrl->alpha = ad;
    commit_direction(ctrl);                 // no block here reads rho, first, fr_next
  }
  update_body(x, r, p, w, N, ad, partials);
}

// alpha from the nbd partials of the normal-equations blur, then the update
// and ||r||^2; one launch when the partials are few enough for every block
// to sum them
constexpr int FUSED_ALPHA_MAX = 1024;

int update_partials(const Plan& P) { return vec_blocks((P.n * P.n) >> 2); }

hipError_t launch_update_alpha(const Plan& P, int nbd, bool rr_step, hipStream_t s) {
  if (nbd > FUSED_ALPHA_MAX) {
    hipError_t e = launch_scalar(P, SC_ALPHA, nbd, s);
    if (e != hipSuccess) return e;
    return launch_update(P, rr_step, s);
  }
  const int N = P.n * P.n;
  const int nb = vec_blocks(N >> 2);
  hipLaunchKernelGGL(update_alpha_kernel, dim3(nb), dim3(VT), 0, s, P.x64, P.r, P.p, P.w, N,
                     P.ctrl, P.partials, nbd, P.mirror_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !rr_step) return e;
  return launch_scalar(P, SC_RR, nb, s);
}

hipError_t launch_scalar(const Plan& P, int kind, int nb, hipStream_t s) {
  if (nb > MAX_PARTIALS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scalar_kernel, dim3(1), dim3(ST), 0, s, P.ctrl, P.partials, kind, nb,
                     P.mirror_dev);
  return hipGetLastError();
}

}  // namespace kpcg
