// Regularisation-parameter rules in the KP-SVD basis (Section 2.2, used with
// the Kronecker approximation's SVD as in Section 5.1).
//
//   b_hat = U_c^T B U_r (two FP32 MFMA GEMMs), s_ij = s_c[i] s_r[j] (FP64),
//   GCV / wGCV, eq. (wGCVTikSVD):
//     G_w(l) = N sum (l^2 b_hat/(s^2+l^2))^2 / (sum ((1-w) s^2 + l^2)/(s^2+l^2))^2
//   discrepancy, eq. (DSCTikSVD):
//     D(l) = sum (l^2 b_hat/(s^2+l^2))^2 - eps^2
// Sums over the N = n^2 spectral entries are FP64, deterministic (per-block
// partials in a fixed order).  The paper minimises / roots these with MATLAB
// fminbnd / fzero; here they are evaluated on a grid and the host picks the
// grid point.
#include "common.h"

namespace kpcg {

constexpr int ST = 256;
constexpr int SMAXB = 256;

// partial sums per (grid point, block): num[g][blk], tr[g][blk]
__global__ __launch_bounds__(ST) void spectral_partials_kernel(
    const float* __restrict__ bhat, const double* __restrict__ sc, const double* __restrict__ sr,
    int n, const double* __restrict__ grid, int ngrid, double omega, double* __restrict__ out) {
  __shared__ double sh[ST / 64];
  const size_t N = (size_t)n * n;
  const size_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const size_t e0 = (size_t)blockIdx.x * chunk;
  const size_t e1 = e0 + chunk < N ? e0 + chunk : N;
  for (int g = 0; g < ngrid; ++g) {
    const double l2 = grid[g] * grid[g];
    double num = 0.0, tr = 0.0;
    for (size_t e = e0 + threadIdx.x; e < e1; e += ST) {
      const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
      const double s = sc[i] * sr[j];
      const double s2 = s * s;
      const double b = (double)bhat[e];
      const double den = s2 + l2;
      const double f = l2 * b / den;
      num += f * f;
      tr += ((1.0 - omega) * s2 + l2) / den;
    }
    const double a = block_sum<ST>(num, sh);
    const double t = block_sum<ST>(tr, sh);
    if (threadIdx.x == 0) {
      out[(size_t)(2 * g) * gridDim.x + blockIdx.x] = a;
      out[(size_t)(2 * g + 1) * gridDim.x + blockIdx.x] = t;
    }
  }
}

// kind 0: (weighted) GCV score; kind 1: discrepancy value (noise2 = eps^2)
__global__ __launch_bounds__(64) void spectral_final_kernel(const double* __restrict__ part,
                                                            int nb, int ngrid, int kind, double N,
                                                            double noise2,
                                                            double* __restrict__ scores) {
  const int g = blockIdx.x;
  if (g >= ngrid || threadIdx.x != 0) return;
  double num = 0.0, tr = 0.0;
  for (int b = 0; b < nb; ++b) {
    num += part[(size_t)(2 * g) * nb + b];
    tr += part[(size_t)(2 * g + 1) * nb + b];
  }
  scores[g] = kind == 0 ? N * num / (tr * tr) : num - noise2;
}

hipError_t launch_spectrum(const Plan& P, const float* b, hipStream_t s) {
  return launch_spectral_gemms(P, b, reinterpret_cast<float*>(P.spec), s);
}

// spec layout: [bhat: n*n floats][grid: 64 doubles][scores: 64 doubles][partials]
hipError_t launch_spectral_scores(const Plan& P, const double* grid_dev, int ngrid,
                                  double omega, double noise2, int kind, double* out_dev,
                                  hipStream_t s) {
  const int n = P.n;
  const size_t N = (size_t)n * n;
  int nb = (int)((N + ST * 8 - 1) / (ST * 8));
  nb = nb < 1 ? 1 : (nb > SMAXB ? SMAXB : nb);
  double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(P.spec) +
                                           ((N * sizeof(float) + 255) / 256) * 256 +
                                           128 * sizeof(double));
  hipLaunchKernelGGL(spectral_partials_kernel, dim3(nb), dim3(ST), 0, s,
                     reinterpret_cast<const float*>(P.spec), P.sc, P.sr, n, grid_dev, ngrid,
                     omega, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(spectral_final_kernel, dim3(ngrid), dim3(64), 0, s, part, nb, ngrid, kind,
                     (double)N, noise2, out_dev);
  return hipGetLastError();
}

}  // namespace kpcg
