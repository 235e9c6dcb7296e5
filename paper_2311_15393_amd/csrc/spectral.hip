// Regularisation-parameter rules in the KP-SVD basis (Section 2.2, used with
// the Kronecker approximation's SVD as in Section 5.1).
//
//   b_hat = U_c^T B U_r (two FP32 MFMA GEMMs), s_ij = s_c[i] s_r[j] (FP64),
//   GCV / wGCV, eq. (wGCVTikSVD):
//     G_w(l) = N sum (l^2 b_hat/(s^2+l^2))^2 / (sum ((1-w) s^2 + l^2)/(s^2+l^2))^2
//   discrepancy, eq. (DSCTikSVD):
//     D(l) = sum (l^2 b_hat/(s^2+l^2))^2 - eps^2
//   optimal error, eq. (OptTikSVD), with x_hat = V_c^T X_true V_r:
//     O(l) = sum (s b_hat/(s^2+l^2) - x_hat)^2
// Sums over the N = n^2 spectral entries are FP64, deterministic (per-block
// partials in a fixed order).  The paper minimises / roots these with MATLAB
// fminbnd / fzero; here they are evaluated on a grid and the host picks the
// grid point.
#include "common.h"

namespace kpcg {

constexpr int ST = 256;
constexpr int SMAXB = 256;

// partial sums per (grid point, block): num[g][blk], tr[g][blk]; with xhat
// (the optimal-error kind) num is the squared error and tr is unused
__global__ __launch_bounds__(ST) void spectral_partials_kernel(
    const float* __restrict__ bhat, const float* __restrict__ xhat,
    const double* __restrict__ sc, const double* __restrict__ sr, int n,
    const double* __restrict__ grid, int ngrid, double omega, double* __restrict__ out) {
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
      if (xhat) {
        const double d = s * b / den - (double)xhat[e];
        num += d * d;
      } else {
        const double f = l2 * b / den;
        num += f * f;
        tr += ((1.0 - omega) * s2 + l2) / den;
      }
    }
    const double a = block_sum<ST>(num, sh);
    const double t = block_sum<ST>(tr, sh);
    if (threadIdx.x == 0) {
      out[(size_t)(2 * g) * gridDim.x + blockIdx.x] = a;
      out[(size_t)(2 * g + 1) * gridDim.x + blockIdx.x] = t;
    }
  }
}

// kind 0: (weighted) GCV score; kind 1: discrepancy value (noise2 = eps^2);
// kind 2: optimal error.  The weighted GCV trace term increases with lambda;
// for omega > 1 it is negative below some lambda_0, where the score would
// fall back towards 0: only the branch with a positive trace (continuous
// with large lambda) is admissible, the others score +inf.
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
  scores[g] = kind == 0 ? (tr > 0.0 ? N * num / (tr * tr) : INFINITY)
                       : (kind == 1 ? num - noise2 : num);
}

hipError_t launch_spectrum(const Plan& P, const float* b, hipStream_t s) {
  return launch_spectral_gemms(P, b, reinterpret_cast<float*>(P.spec), s);
}

// spec layout: [bhat: n*n floats][grid: 64 doubles][scores: 64 doubles][partials]
hipError_t launch_spectral_scores(const Plan& P, const double* grid_dev, int ngrid,
                                  double omega, double noise2, int kind, double* out_dev,
                                  hipStream_t s, const float* xhat) {
  const int n = P.n;
  const size_t N = (size_t)n * n;
  int nb = (int)((N + ST * 8 - 1) / (ST * 8));
  nb = nb < 1 ? 1 : (nb > SMAXB ? SMAXB : nb);
  double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(P.spec) +
                                           ((N * sizeof(float) + 255) / 256) * 256 +
                                           128 * sizeof(double));
  hipLaunchKernelGGL(spectral_partials_kernel, dim3(nb), dim3(ST), 0, s,
                     reinterpret_cast<const float*>(P.spec), kind == 2 ? xhat : nullptr, P.sc,
                     P.sr, n, grid_dev, ngrid, omega, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(spectral_final_kernel, dim3(ngrid), dim3(64), 0, s, part, nb, ngrid, kind,
                     (double)N, noise2, out_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// features of the data for the lambda-predicting network: with c = V_c^T B V_r
// and s_ij = s_c[i] s_r[j], 64 bins of log10(s) over [-8, 0) (s below 1e-8 in
// bin 0, s >= 1 in bin 63); feature k = log10(max(mean c^2 over bin k, 1e-30))
// (empty bin: 1e-30), feature 64 + k = log10(count_k / N + 1e-12).
// Per-thread private histograms in LDS, summed in a fixed order.
// ---------------------------------------------------------------------------
constexpr int FT = 64, NBIN = 64, FMAXB = 256;

__device__ inline int spectral_bin(double s) {
  if (!(s > 0.0)) return 0;
  const double b = floor((log10(s) + 8.0) / 8.0 * 64.0);
  return b < 0.0 ? 0 : (b > 63.0 ? 63 : (int)b);
}

__global__ __launch_bounds__(FT) void feature_partials_kernel(const float* __restrict__ c,
                                                              const double* __restrict__ sc,
                                                              const double* __restrict__ sr,
                                                              int n, double* __restrict__ part) {
  __shared__ double hs[NBIN][FT + 1];
  __shared__ int hc[NBIN][FT + 1];
  const int t = threadIdx.x;
  for (int k = 0; k < NBIN; ++k) {
    hs[k][t] = 0.0;
    hc[k][t] = 0;
  }
  const size_t N = (size_t)n * n;
  const size_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const size_t e0 = (size_t)blockIdx.x * chunk;
  const size_t e1 = e0 + chunk < N ? e0 + chunk : N;
  for (size_t e = e0 + t; e < e1; e += FT) {
    const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
    const int k = spectral_bin(sc[i] * sr[j]);
    const double v = (double)c[e];
    hs[k][t] += v * v;
    hc[k][t] += 1;
  }
  __syncthreads();
  double s = 0.0;
  long cnt = 0;
  for (int u = 0; u < FT; ++u) {
    s += hs[t][u];
    cnt += hc[t][u];
  }
  part[(size_t)blockIdx.x * 2 * NBIN + t] = s;
  part[(size_t)blockIdx.x * 2 * NBIN + NBIN + t] = (double)cnt;
}

__global__ __launch_bounds__(FT) void feature_final_kernel(const double* __restrict__ part,
                                                           int nb, double N,
                                                           float* __restrict__ out) {
  const int k = threadIdx.x;
  double s = 0.0, cnt = 0.0;
  for (int b = 0; b < nb; ++b) {
    s += part[(size_t)b * 2 * NBIN + k];
    cnt += part[(size_t)b * 2 * NBIN + NBIN + k];
  }
  const double mean = cnt > 0.0 ? s / cnt : 0.0;
  out[k] = (float)log10(mean > 1e-30 ? mean : 1e-30);
  out[NBIN + k] = (float)log10(cnt / N + 1e-12);
}

hipError_t launch_features(const Plan& P, const float* b, float* out, hipStream_t s) {
  const int n = P.n;
  const size_t N = (size_t)n * n;
  float* c = reinterpret_cast<float*>(P.t2);
  hipError_t e = launch_vbasis_gemms(P, b, c, s);
  if (e != hipSuccess) return e;
  int nb = (int)((N + 4095) / 4096);
  nb = nb < 1 ? 1 : (nb > FMAXB ? FMAXB : nb);
  double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(P.spec) +
                                           ((N * sizeof(float) + 255) / 256) * 256 +
                                           128 * sizeof(double));
  hipLaunchKernelGGL(feature_partials_kernel, dim3(nb), dim3(FT), 0, s, c, P.sc, P.sr, n, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(feature_final_kernel, dim3(1), dim3(FT), 0, s, part, nb, (double)N, out);
  return hipGetLastError();
}

}  // namespace kpcg
