// FP8 (e4m3) preconditioner chain with block scaling: the four GEMMs of
// Section 3, eq. (PreconSolve), on the tiles of gemm_fp8.h.
#include "gemm_fp8.h"

namespace kpcg {

// The residual-norm step of the update before, folded in while the first
// operand loads are in flight (the FP8 chain does not scale the residual, so
// only the state is needed here).
struct Fp8RrFold {
  Ctrl* ctrl;
  const double* partials;
  int nb;
  CtrlMirror* mirror;
  StepIn kin;             // taken at the kernel's start
  __device__ bool operator()() const {
    __shared__ double fsh[fold_sh<G8T>()];
    const double S = fold_slot<G8T>(partials, SLOT_RR, nb, fsh);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
      apply_rr(ctrl, S);
      if (mirror != nullptr) publish_mirror(ctrl, mirror);
    }
    return rr_state(kin, S) == RUNNING;                 // the same decision in every block
  }
};

template <bool B_F32, int EPI>
__global__ __launch_bounds__(G8T) void gemm8_kernel(Gemm8Args g, Ctrl* ctrl, int skip,
                                                    double* partials, int fold_rr,
                                                    CtrlMirror* __restrict__ mirror) {
  if (skip && ctrl->done != RUNNING) return;
  const int m0 = blockIdx.y * B8M, n0 = blockIdx.x * B8N;
  double* pout = partials + SLOT_RZ * MAX_PARTIALS + blockIdx.y * gridDim.x + blockIdx.x;
  if (fold_rr > 0)
    gemm8_tile<B_F32, EPI>(g, m0, n0, ctrl, pout, MAX_PARTIALS,
                           Fp8RrFold{ctrl, partials, fold_rr, mirror, step_in(ctrl)});
  else
    gemm8_tile<B_F32, EPI>(g, m0, n0, ctrl, pout, MAX_PARTIALS, NoFold8{});
}

template <bool BF, int EPI>
static hipError_t run8(const Plan& P, const Gemm8Args& a, int skip, hipStream_t s,
                       int fold_rr = 0) {
  dim3 grid(P.n / B8N, P.n / B8M);
  hipLaunchKernelGGL((gemm8_kernel<BF, EPI>), grid, dim3(G8T), 0, s, a, P.ctrl, skip,
                     P.partials, fold_rr, P.mirror_dev);
  return hipGetLastError();
}

bool fp8_supported_size(int n) { return n % B8K == 0; }

int precond_partials_fp8(const Plan& P) { return (P.n / B8N) * (P.n / B8M); }

hipError_t launch_precond_fp8(const Plan& P, const float* r, float* z, const float* w,
                              bool finalize, float lam2, hipStream_t s, int fold_rr) {
  if (r == nullptr) return hipSuccess;                 // capability probe
  if (!fp8_supported_size(P.n)) return hipErrorNotSupported;
  const int n = P.n, skip = finalize ? 1 : 0;
  uint8_t* t1 = reinterpret_cast<uint8_t*>(P.t1);
  uint8_t* t2 = reinterpret_cast<uint8_t*>(P.t2);
  uint8_t* t3 = reinterpret_cast<uint8_t*>(P.t3);
  Gemm8Args a{};
  a.n = n;
  a.sc2 = P.sc2;
  a.sr2 = P.sr2;
  a.d0 = P.sprime_d0;
  a.lam2 = lam2;
  // 1. T1 = Vc^T R (R quantised per (column, 32 rows) while staged)
  a.A = P.VcT8; a.As = P.VcT8s; a.Bf32 = r; a.C = t1; a.Cs = P.t1s;
  hipError_t e = run8<true, E8_ROWS>(P, a, skip, s, fold_rr);
  if (e != hipSuccess) return e;
  // 2. T2^T = (S' .* (T1 Vr))^T
  a.A = t1; a.As = P.t1s; a.B = P.VrT8; a.Bs = P.VrT8s; a.C = t2; a.Cs = P.t2s;
  e = run8<false, E8_SPRIME_T>(P, a, skip, s);
  if (e != hipSuccess) return e;
  // 3. T3 = Vc T2
  a.A = P.Vc8; a.As = P.Vc8s; a.B = t2; a.Bs = P.t2s; a.C = t3; a.Cs = P.t3s;
  e = run8<false, E8_ROWS>(P, a, skip, s);
  if (e != hipSuccess) return e;
  // 4. z = T3 Vr^T / lambda^2
  a.A = t3; a.As = P.t3s; a.B = P.Vr8; a.Bs = P.Vr8s; a.z = z; a.r = r; a.w = w;
  if (!finalize) return run8<false, E8_FINAL_NR>(P, a, skip, s);
  // the partials of r.z and z.w go to the direction step (launch_pupdate_fold)
  return run8<false, E8_FINAL>(P, a, skip, s);
}

}  // namespace kpcg
