// Learned choice of the regularisation parameter: a small MLP mapping 128
// spectral features of the data (in the KP-SVD basis) to log10(lambda).
//
// The paper selects lambda with GCV, weighted GCV or the discrepancy principle
// evaluated with the Kronecker approximation's SVD (Section 2.2, Section 5.1)
// and leaves a more systematic choice of these parameters open (Section 5.1,
// Section 6).  This network is this library's extension for that open point;
// GCV stays the judge of its answer (kp_lambda_learned falls back to the GCV
// grid choice when the predicted lambda scores too far above the GCV minimum).
//
// Network: 128 -> 256 -> 256 -> 256 -> 1, exact GELU g(z) = z Phi(z) after each
// hidden layer, linear output; loss mean((y - t)^2); Adam with bias correction.
// Hidden layers run on FP16 MFMA (FP16 weights and activations, FP32
// accumulation), the output layer and the whole backward pass in FP32, the
// optimiser on FP32 master weights.
#pragma once

#include "common.h"

namespace kpcg {

constexpr int MLP_NF = 128;   // input features
constexpr int MLP_NH = 256;   // hidden width

// flat FP32 parameter layout, weights [out][in] row-major
constexpr size_t MLP_OFF_W1 = 0;
constexpr size_t MLP_OFF_B1 = MLP_OFF_W1 + (size_t)MLP_NH * MLP_NF;
constexpr size_t MLP_OFF_W2 = MLP_OFF_B1 + MLP_NH;
constexpr size_t MLP_OFF_B2 = MLP_OFF_W2 + (size_t)MLP_NH * MLP_NH;
constexpr size_t MLP_OFF_W3 = MLP_OFF_B2 + MLP_NH;
constexpr size_t MLP_OFF_B3 = MLP_OFF_W3 + (size_t)MLP_NH * MLP_NH;
constexpr size_t MLP_OFF_W4 = MLP_OFF_B3 + MLP_NH;
constexpr size_t MLP_OFF_B4 = MLP_OFF_W4 + MLP_NH;
constexpr size_t MLP_NPARAM = MLP_OFF_B4 + 1;

// FP16 copies of the three hidden-layer weight matrices, back to back
constexpr size_t MLP_H16_W1 = 0;
constexpr size_t MLP_H16_W2 = MLP_H16_W1 + (size_t)MLP_NH * MLP_NF;
constexpr size_t MLP_H16_W3 = MLP_H16_W2 + (size_t)MLP_NH * MLP_NH;
constexpr size_t MLP_H16_N = MLP_H16_W3 + (size_t)MLP_NH * MLP_NH;

// contraction slices of the backward GEMMs and their partial-sum buffer
constexpr int MLP_KSPLIT_MAX = 16;
constexpr size_t MLP_PART_FLOATS = (size_t)1 << 20;

struct Mlp {
  int max_batch = 0;
  bool owns = false;
  char* base = nullptr;
  size_t bytes = 0;
  long step = 0;                 // Adam steps taken
  float* params = nullptr;       // FP32 master weights
  float* grads = nullptr;
  float* m = nullptr;            // Adam first moment
  float* v = nullptr;            // Adam second moment
  _Float16* w16 = nullptr;       // FP16 hidden-layer weights
  float* mu = nullptr;           // feature normaliser
  float* scale = nullptr;
  int* rows = nullptr;           // minibatch row indices (max_batch)
  _Float16* h0 = nullptr;        // [B][128] normalised input
  float* z1 = nullptr;           // [B][256] pre-activations
  _Float16* h1 = nullptr;
  float* z2 = nullptr;
  _Float16* h2 = nullptr;
  float* z3 = nullptr;
  float* h3 = nullptr;           // [B][256] FP32 (input of the output layer)
  float* y = nullptr;            // [B] outputs
  float* dz4 = nullptr;          // [B] dL/dy
  float* dza = nullptr;          // [B][256] dL/dz ping-pong
  float* dzb = nullptr;
  double* loss = nullptr;        // [1]
  float* gpart = nullptr;        // [MLP_PART_FLOATS] sliced backward GEMM partials
  double* host_loss = nullptr;   // pinned
};

size_t mlp_layout(int max_batch, char* base, Mlp* M);

// bytes of the forward activations (h0, z1, h1, z2, h2, z3, h3, y, dz4) of
// `rows` rows, each buffer 256-byte aligned; mlp_act_layout points M's
// activation buffers into base (which must be 256-byte aligned) and returns
// the bytes used, which equal mlp_act_bytes(rows)
constexpr size_t mlp_a256(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t mlp_act_bytes(size_t rows) {
  return mlp_a256(rows * MLP_NF * 2) + 3 * mlp_a256(rows * MLP_NH * 4) +
         2 * mlp_a256(rows * MLP_NH * 2) + mlp_a256(rows * MLP_NH * 4) + 2 * mlp_a256(rows * 4);
}
size_t mlp_act_layout(int rows, char* base, Mlp* M);

// forward through the hidden layers and the output layer for nb rows of X
// (rows == nullptr: rows 0..nb-1, else the device indices rows[0..nb)),
// writing y (and, if pred != nullptr, the outputs as FP64 to pred)
hipError_t mlp_forward(const Mlp& M, const float* X, const int* rows, int nb, double* pred,
                       hipStream_t s);
// loss and gradients for the last mlp_forward's batch against targets t[rows]
hipError_t mlp_backward(const Mlp& M, const float* t, const int* rows, int nb, hipStream_t s);
// one Adam update of the master weights from M.grads (and their FP16 copies)
hipError_t mlp_adam(const Mlp& M, float lr, float b1, float b2, float eps, float bc1, float bc2,
                    hipStream_t s);
// refresh the FP16 weight copies from the master weights
hipError_t mlp_refresh_half(const Mlp& M, hipStream_t s);
// per-feature mean and standard deviation of nb rows of X
hipError_t mlp_fit_norm(const Mlp& M, const float* X, int nb, hipStream_t s);

}  // namespace kpcg
