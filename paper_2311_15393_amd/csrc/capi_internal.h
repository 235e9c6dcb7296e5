// Pieces shared by the C ABI translation units (capi.hip, capi_lambda.hip).
#pragma once

#include <cstdint>

#include "common.h"

struct kp_plan_s {
  kpcg::Plan P;
};

#define HIP_OR(x, code)                   \
  do {                                    \
    if ((x) != hipSuccess) return (code); \
  } while (0)
#define HIPCHK(x) HIP_OR(x, KP_ERR_HIP)

namespace kpcg {

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }


// grid of ngrid in [1, max_points] finite positive values
bool valid_grid(const double* grid, int ngrid, int max_points = 64);

// b_hat of b, then the kind's score on each grid value (kind 0: weighted
// GCV with omega, 1: discrepancy with noise2, 2: optimal error against
// x_hat = V_c^T X_true V_r of x_true); scores copied to the host.
// Synchronises.
int spectral_call(kp_plan_t plan, const float* b, const double* grid, int ngrid, double omega,
                  double noise2, int kind, double* scores_host, void* stream,
                  const float* x_true = nullptr);

}  // namespace kpcg
