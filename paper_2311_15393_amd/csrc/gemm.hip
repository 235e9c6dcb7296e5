// Preconditioner solve z = M^{-1} r on MFMA.
//
// Section 3, eq. (PreconSolve): Z = V_c (S .* (V_c^T R V_r)) V_r^T, with
// vec(S) = diag(D^{-1}), S[i][j] = 1/(s_c[i]^2 s_r[j]^2 + lambda^2), and the
// factors stored -- and the products computed -- in reduced precision.
//
// Four n x n x n GEMMs, each written as C = A * Bt^T with both operands
// K-contiguous in memory (so every operand feeds the MFMA straight from LDS):
//   1. T1  = Vc^T  * R      A = VcT (stored), B = R read row-major from the
//                            FP32 residual, scaled and rounded while staged
//   2. T   = T1    * Vr     A = T1, Bt = VrT (stored); epilogue T2 = S' .* T,
//                            written transposed for stage 3
//   3. T3  = Vc    * T2     A = Vc (stored), Bt = T2^T
//   4. Z   = T3    * Vr^T   A = T3, Bt = Vr (stored); epilogue z = Z * zscale,
//                            with the FP64 dots r.z and z.(Hp) of the iteration
// S' = lambda^2 S lies in (0, 1] (lambda^2 folded out, restored by zscale =
// 1/(pscale lambda^2)); for FP16 the residual is scaled by a power of two
// pscale so that ||pscale r|| < 2^14, which keeps every FP16 intermediate
// below 65504 (V orthogonal).  This replaces the paper's literal "S in
// half precision", which overflows FP16 for lambda < 3.9e-3.
//
// Tiles: 64 x 64 per workgroup, 4 waves in 2 x 2, each wave 32 x 32 as 2 x 2
// MFMA 16x16 blocks; FP32 uses v_mfma_f32_16x16x4_f32, FP16
// v_mfma_f32_16x16x32_f16, both accumulating in FP32.  The contraction is
// split over four such wave groups per workgroup, reduced in LDS.
#include "gemm_core.h"

namespace kpcg {

// contraction split over GEMM_KS wave groups per workgroup (see
// gemm_tile_splitk): at n = 1024 a 64 x 64 tile grid is only 256
// workgroups, one per CU, so the k-loop's global latency is otherwise exposed
constexpr int GEMM_KS = 4;

// The residual-norm step of the update before the preconditioner, folded
// into its first GEMM while the first operand loads are in flight: every
// workgroup sums the update's partials of ||r||^2 (LDS scratch at the start
// of the stage buffers, free until the first stage is staged), block 0
// records the step and publishes, and the FP16 residual scale follows from
// the sum.
struct RrFold {
  Ctrl* ctrl;
  const double* partials;
  int nb;
  CtrlMirror* mirror;
  bool scale;
  StepIn kin;             // taken at the kernel's start
  __device__ bool operator()(float& bscale, char* lds) const {
    double* sh = reinterpret_cast<double*>(lds);
    const double S = fold_slot<GT * GEMM_KS>(partials, SLOT_RR, nb, sh);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
      apply_rr(ctrl, S);
      if (mirror != nullptr) publish_mirror(ctrl, mirror);
    }
    if (rr_state(kin, S) != RUNNING) return false;     // the same decision in every block
    if (scale) bscale = kin.prec == KP_P16 ? fp16_residual_scale(S) : 1.0f;
    return true;
  }
};

template <typename T, bool B_FROM_F32, class Epi>
__global__ __launch_bounds__(GT * GEMM_KS) void gemm_kernel(const T* __restrict__ A,
                                                            const void* __restrict__ Bsrc, int n,
                                                            Epi epi, Ctrl* ctrl, int skip_if_done,
                                                            int scale_mode, double* partials,
                                                            int fold_rr,
                                                            CtrlMirror* __restrict__ mirror) {
  extern __shared__ __align__(16) char gemm_lds[];
  if (skip_if_done && ctrl->done != RUNNING) return;
  // scale_mode bit 0: scale the FP32 B source by pscale; bit 1: scale the
  // output by zscale (both set on the device from ||r||)
  const float bscale = (scale_mode & 1) ? ctrl->pscale : 1.0f;
  const float oscale = (scale_mode & 2) ? ctrl->zscale : 1.0f;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (fold_rr > 0) {
    RrFold f{ctrl, partials, fold_rr, mirror, (scale_mode & 1) != 0, step_in(ctrl)};
    gemm_tile_splitk<T, B_FROM_F32, Epi, GEMM_KS, RrFold>(
        A, Bsrc, n, blockIdx.y * BM, blockIdx.x * BN, epi, bscale, oscale,
        partials + SLOT_RZ * MAX_PARTIALS + bid, MAX_PARTIALS, gemm_lds, f);
    return;
  }
  gemm_tile_splitk<T, B_FROM_F32, Epi, GEMM_KS>(A, Bsrc, n, blockIdx.y * BM, blockIdx.x * BN,
                                                epi, bscale, oscale,
                                                partials + SLOT_RZ * MAX_PARTIALS + bid,
                                                MAX_PARTIALS, gemm_lds);
}

template <typename T, bool BF, class Epi>
static hipError_t run_gemm(const Plan& P, const T* A, const void* B, Epi epi, int skip,
                           int scale_mode, hipStream_t s, int fold_rr = 0) {
  const int n = P.n;
  dim3 grid((n + BN - 1) / BN, (n + BM - 1) / BM);
  if ((long)grid.x * grid.y > MAX_PARTIALS) return hipErrorInvalidValue;
  constexpr size_t lds = gemm_splitk_lds<T>(GEMM_KS);
  auto kern = gemm_kernel<T, BF, Epi>;
  static bool granted = false;          // once per instantiation
  if (!granted) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    granted = true;
  }
  hipLaunchKernelGGL(kern, grid, dim3(GT * GEMM_KS), lds, s, A, B, n, epi, P.ctrl, skip,
                     scale_mode, P.partials, fold_rr, P.mirror_dev);
  return hipGetLastError();
}

template <typename T>
static hipError_t precond_chain(const Plan& P, const T* VcT, const T* Vc, const T* Vr,
                                const T* VrT, const float* r, float* z, const float* w,
                                bool finalize, float lam2, hipStream_t s, int fold_rr) {
  const int n = P.n;
  const int skip = finalize ? 1 : 0;
  T* t1 = reinterpret_cast<T*>(P.t1);
  T* t2 = reinterpret_cast<T*>(P.t2);
  T* t3 = reinterpret_cast<T*>(P.t3);
  hipError_t e;
  e = run_gemm<T, true>(P, VcT, r, GEpiStore<T>{t1, n}, skip, 1, s, fold_rr);
  if (e != hipSuccess) return e;
  e = run_gemm<T, false>(P, t1, VrT, GEpiSPrimeT<T>{t2, P.sc2, P.sr2, lam2, n, nullptr, P.sprime_d0 ? P.d0t : nullptr}, skip, 0, s);
  if (e != hipSuccess) return e;
  e = run_gemm<T, false>(P, Vc, t2, GEpiStore<T>{t3, n}, skip, 0, s);
  if (e != hipSuccess) return e;
  if (!finalize) return run_gemm<T, false>(P, t3, Vr, GEpiFinal<false>{z, r, w, n}, skip, 2, s);
  // the partials of r.z and z.w go to the direction step (launch_pupdate_fold)
  return run_gemm<T, false>(P, t3, Vr, GEpiFinal<true>{z, r, w, n}, skip, 2, s);
}

int precond_partials(const Plan& P, int prec) {
  if (prec == KP_P8) return precond_partials_fp8(P);
  return ((P.n + BN - 1) / BN) * ((P.n + BM - 1) / BM);
}

hipError_t launch_precond(const Plan& P, const float* r, float* z, const float* w, int prec,
                          bool finalize, float lam2, hipStream_t s, int fold_rr) {
  if (fold_rr > MAX_PARTIALS) return hipErrorInvalidValue;
  if (prec == KP_P16)
    return precond_chain<_Float16>(P, reinterpret_cast<const _Float16*>(P.VcT16),
                                   reinterpret_cast<const _Float16*>(P.Vc16),
                                   reinterpret_cast<const _Float16*>(P.Vr16),
                                   reinterpret_cast<const _Float16*>(P.VrT16), r, z, w,
                                   finalize, lam2, s, fold_rr);
  if (prec == KP_P32)
    return precond_chain<float>(P, P.VcT32, P.Vc32, P.Vr32, P.VrT32, r, z, w, finalize, lam2,
                                s, fold_rr);
  return launch_precond_fp8(P, r, z, w, finalize, lam2, s, fold_rr);
}

// plain FP32 GEMM C = A * B (B from FP32 rows) then C2 = C * Bt^T, used for the
// spectral coefficients b_hat = Uc^T B Ur of the parameter-choice rules
hipError_t launch_spectral_gemms(const Plan& P, const float* b, float* out, hipStream_t s) {
  const int n = P.n;
  float* t1 = reinterpret_cast<float*>(P.t1);
  hipError_t e = run_gemm<float, true>(P, P.UcT32, b, GEpiStore<float>{t1, n}, 0, 0, s);
  if (e != hipSuccess) return e;
  return run_gemm<float, false>(P, t1, P.UrT32, GEpiStore<float>{out, n}, 0, 0, s);
}

// the same two GEMMs in the right singular bases: out = Vc^T B Vr (features
// of the data, and x_hat of the optimal-error score)
hipError_t launch_vbasis_gemms(const Plan& P, const float* b, float* out, hipStream_t s) {
  const int n = P.n;
  float* t1 = reinterpret_cast<float*>(P.t1);
  hipError_t e = run_gemm<float, true>(P, P.VcT32, b, GEpiStore<float>{t1, n}, 0, 0, s);
  if (e != hipSuccess) return e;
  return run_gemm<float, false>(P, t1, P.VrT32, GEpiStore<float>{out, n}, 0, 0, s);
}

}  // namespace kpcg
