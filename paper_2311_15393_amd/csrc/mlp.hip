// Kernels of the lambda-predicting MLP (layout and network in mlp.h).
//
// Forward, hidden layers: Z = H W^T + b on v_mfma_f32_16x16x32_f16, H and W in
// FP16 (K-contiguous rows, fragments loaded straight from global memory: the
// weights are at most 128 KB and stay in L2), FP32 accumulation; the epilogue
// adds the bias, stores Z (FP32, kept for the backward pass) and the GELU
// output (FP16 for the next hidden layer, FP32 for the output layer).
// Output layer: one wave per sample, FP32.
// Backward: FP32 LDS-tiled GEMMs (64 x 64 tiles, 4 x 4 per thread) for
// dW = dZ^T H and dH = dZ W with the GELU derivative fused into the store,
// and fixed-order column sums for the biases; every reduction is
// deterministic (no atomics).  Adam: elementwise on the FP32 master weights,
// refreshing their FP16 copies in the same pass.
#include <cmath>

#include "mlp.h"

namespace kpcg {

namespace {

typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

inline unsigned blocks_for(size_t count) { return (unsigned)((count + 255) / 256); }

constexpr float kInvSqrt2 = 0.70710678118654752f;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * kInvSqrt2)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * kInvSqrt2)) + z * kInvSqrt2Pi * expf(-0.5f * z * z);
}

// ---------------------------------------------------------------------------
// input: h0[b][f] = fp16((X[row_b][f] - mu[f]) / scale[f])
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_input_kernel(const float* __restrict__ X,
                                                        const int* __restrict__ rows, int nb,
                                                        const float* __restrict__ mu,
                                                        const float* __restrict__ scale,
                                                        _Float16* __restrict__ h0) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)nb * MLP_NF) return;
  const int b = (int)(e / MLP_NF), f = (int)(e % MLP_NF);
  const int r = rows ? rows[b] : b;
  h0[e] = (_Float16)((X[(size_t)r * MLP_NF + f] - mu[f]) / scale[f]);
}

// ---------------------------------------------------------------------------
// hidden layer forward on MFMA: 64 (batch) x 64 (units) per workgroup,
// 4 waves in 2 x 2, each 32 x 32 as 2 x 2 blocks of 16 x 16
// ---------------------------------------------------------------------------
template <bool OUT_F16>
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const _Float16* __restrict__ H, int in,
                                                      const _Float16* __restrict__ W,
                                                      const float* __restrict__ bias, int nb,
                                                      float* __restrict__ Z,
                                                      void* __restrict__ Hout) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int m0 = blockIdx.y * 64 + (wv >> 1) * 32;     // batch rows
  const int n0 = blockIdx.x * 64 + (wv & 1) * 32;      // units
  f4_t acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = f4_t{0.f, 0.f, 0.f, 0.f};
  const h8_t zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < in; k += 32) {
    h8_t a[2], b[2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const int row = m0 + mi * 16 + r16;
      a[mi] = row < nb ? *reinterpret_cast<const h8_t*>(H + (size_t)row * in + k + g * 8)
                       : zero8;
    }
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
      const int unit = n0 + ni * 16 + r16;
      b[ni] = *reinterpret_cast<const h8_t*>(W + (size_t)unit * in + k + g * 8);
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
      const int unit = n0 + ni * 16 + r16;
      const float bb = bias[unit];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + mi * 16 + 4 * g + v;
        if (row >= nb) continue;
        const float z = acc[mi][ni][v] + bb;
        const size_t o = (size_t)row * MLP_NH + unit;
        Z[o] = z;
        if constexpr (OUT_F16)
          reinterpret_cast<_Float16*>(Hout)[o] = (_Float16)gelu(z);
        else
          reinterpret_cast<float*>(Hout)[o] = gelu(z);
      }
    }
}

// ---------------------------------------------------------------------------
// output layer: y[b] = h3[b] . w4 + b4, one wave per sample; with targets,
// dz4[b] = (2 / nb) (y[b] - t[row_b])
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_head_kernel(const float* __restrict__ h3,
                                                       const float* __restrict__ params, int nb,
                                                       float* __restrict__ y,
                                                       double* __restrict__ pred,
                                                       const float* __restrict__ t,
                                                       const int* __restrict__ rows,
                                                       float* __restrict__ dz4) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= nb) return;
  const float* w4 = params + MLP_OFF_W4;
  const float* h = h3 + (size_t)b * MLP_NH;
  float s = 0.f;
#pragma unroll
  for (int k = lane; k < MLP_NH; k += 64) s = fmaf(h[k], w4[k], s);
  s = wave_sum(s);
  if (lane == 0) {
    const float yb = s + params[MLP_OFF_B4];
    y[b] = yb;
    if (pred) pred[b] = (double)yb;
    if (t) dz4[b] = (2.0f / (float)nb) * (yb - t[rows ? rows[b] : b]);
  }
}

// loss = mean (y - t)^2 in FP64, one block, fixed order
__global__ __launch_bounds__(256) void mlp_loss_kernel(const float* __restrict__ y,
                                                       const float* __restrict__ t,
                                                       const int* __restrict__ rows, int nb,
                                                       double* __restrict__ out) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    const double d = (double)y[b] - (double)t[rows ? rows[b] : b];
    acc += d * d;
  }
  const double tot = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) out[0] = tot / nb;
}

// dz3[b][k] = dz4[b] w4[k] g'(z3[b][k])
__global__ __launch_bounds__(256) void mlp_head_bwd_kernel(const float* __restrict__ dz4,
                                                           const float* __restrict__ params,
                                                           const float* __restrict__ z3, int nb,
                                                           float* __restrict__ dz3) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)nb * MLP_NH) return;
  const int b = (int)(e / MLP_NH), k = (int)(e % MLP_NH);
  dz3[e] = dz4[b] * params[MLP_OFF_W4 + k] * gelu_grad(z3[e]);
}

// out[c] = sum_b s[b] M[b][c] (s == nullptr: s = 1), 64 columns per block,
// 4 row groups summed in a fixed order
__global__ __launch_bounds__(256) void mlp_colsum_kernel(const float* __restrict__ M, int ld,
                                                         int ncol, const float* __restrict__ s,
                                                         int nb, float* __restrict__ out) {
  __shared__ float part[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), rg = threadIdx.x >> 6;
  float acc = 0.f;
  if (c < ncol)
    for (int b = rg; b < nb; b += 4) {
      const float v = M[(size_t)b * ld + c];
      acc = s ? fmaf(s[b], v, acc) : acc + v;
    }
  part[rg][threadIdx.x & 63] = acc;
  __syncthreads();
  if (rg == 0 && c < ncol) {
    const int l = threadIdx.x & 63;
    out[c] = ((part[0][l] + part[1][l]) + part[2][l]) + part[3][l];
  }
}

// ---------------------------------------------------------------------------
// backward GEMM, FP32: C[m][n] = sum_k A(m,k) B(k,n), 64 x 64 tiles, BK = 16,
// each of 256 threads owns a 4 x 4 block
// ---------------------------------------------------------------------------
constexpr int BT = 64, BKK = 16;

// A(m, k) = src[k * ld + m]   (m contiguous)     -- dZ^T for dW
struct AMajorM {
  const float* p; int ld;
  static constexpr bool KFAST = false;
  __device__ float at(int m, int k) const { return p[(size_t)k * ld + m]; }
};
// A(m, k) = src[m * ld + k]   (k contiguous)     -- dZ for dH
struct AMajorK {
  const float* p; int ld;
  static constexpr bool KFAST = true;
  __device__ float at(int m, int k) const { return p[(size_t)m * ld + k]; }
};
// B(k, n) = src[k * ld + n], FP16 or FP32      -- H for dW, W for dH
template <typename T>
struct BRows {
  const T* p; int ld;
  __device__ float at(int k, int n) const { return (float)p[(size_t)k * ld + n]; }
};

struct EpiGrad {                       // grads[m * ld + n] = c
  float* g; int ld;
  __device__ void store(int m, int n, float c) const { g[(size_t)m * ld + n] = c; }
};
struct EpiGeluBack {                   // dz[m][n] = c g'(z[m][n])
  float* dz; const float* z; int ld;
  __device__ void store(int m, int n, float c) const {
    const size_t o = (size_t)m * ld + n;
    dz[o] = c * gelu_grad(z[o]);
  }
};

template <class AL, class BL, class Epi>
__device__ inline void mlp_gemm_body(int M, int N, int K, AL A, BL B, Epi epi) {
  __shared__ float sA[BKK][BT + 4];
  __shared__ float sB[BKK][BT + 4];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * BT, n0 = blockIdx.x * BT;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += BKK) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = threadIdx.x + 256 * i;
      int mm, kk;
      if constexpr (AL::KFAST) {
        kk = e % BKK; mm = e / BKK;
      } else {
        mm = e % BT; kk = e / BT;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      sA[kk][mm] = (gm < M && gk < K) ? A.at(gm, gk) : 0.f;
      const int nn = e % BT, kb = e / BT;
      const int gn = n0 + nn, gkb = k0 + kb;
      sB[kb][nn] = (gn < N && gkb < K) ? B.at(gkb, gn) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BKK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sB[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
      if (m < M && n < N) epi.store(m, n, acc[i][j]);
    }
}

template <class AL, class BL, class Epi>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(int M, int N, int K, AL A, BL B, Epi epi) {
  mlp_gemm_body(M, N, K, A, B, epi);
}

// the operands shifted to a contraction slice: A(m, k0 + k), B(k0 + k, n)
template <class AL>
struct ASlice {
  AL a; int k0;
  static constexpr bool KFAST = AL::KFAST;
  __device__ float at(int m, int k) const { return a.at(m, k0 + k); }
};
template <class BL>
struct BSlice {
  BL b; int k0;
  __device__ float at(int k, int n) const { return b.at(k0 + k, n); }
};

// the same product over the contraction slice [z kc, (z+1) kc) (z = blockIdx.z),
// raw sums to part[z][m][n]
struct EpiPart {
  float* part; int M, N;
  __device__ void store(int m, int n, float c) const {
    part[((size_t)blockIdx.z * M + m) * N + n] = c;
  }
};

template <class AL, class BL>
__global__ __launch_bounds__(256) void mlp_gemm_slice_kernel(int M, int N, int K, int kc, AL A,
                                                             BL B, float* part) {
  const int k0 = blockIdx.z * kc;
  const int kn = K - k0 < kc ? K - k0 : kc;
  mlp_gemm_body(M, N, kn, ASlice<AL>{A, k0}, BSlice<BL>{B, k0}, EpiPart{part, M, N});
}

// out[m][n] = sum over slices in order, then the epilogue
template <class Epi>
__global__ __launch_bounds__(256) void mlp_slice_sum_kernel(int M, int N, int ks,
                                                            const float* __restrict__ part,
                                                            Epi epi) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)M * N) return;
  float acc = 0.f;
  for (int z = 0; z < ks; ++z) acc += part[(size_t)z * M * N + e];
  epi.store((int)(e / N), (int)(e % N), acc);
}

// A grid of a few tiles leaves the GPU idle through a long contraction: split
// it into slices (partial products summed in a fixed order afterwards) so
// that at least ~128 workgroups run.
template <class AL, class BL, class Epi>
hipError_t run_mlp_gemm(const Mlp& M_, int M, int N, int K, AL A, BL B, Epi epi, hipStream_t s) {
  const int tiles = ((N + BT - 1) / BT) * ((M + BT - 1) / BT);
  int ks = 1;
  while (ks < MLP_KSPLIT_MAX && tiles * ks < 128 && K / (2 * ks) >= 32) ks *= 2;
  if (ks == 1 || (size_t)ks * M * N > MLP_PART_FLOATS) {
    dim3 grid((N + BT - 1) / BT, (M + BT - 1) / BT);
    hipLaunchKernelGGL((mlp_gemm_kernel<AL, BL, Epi>), grid, dim3(256), 0, s, M, N, K, A, B, epi);
    return hipGetLastError();
  }
  const int kc = (K + ks - 1) / ks;
  dim3 grid((N + BT - 1) / BT, (M + BT - 1) / BT, ks);
  hipLaunchKernelGGL((mlp_gemm_slice_kernel<AL, BL>), grid, dim3(256), 0, s, M, N, K, kc, A, B,
                     M_.gpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((mlp_slice_sum_kernel<Epi>), dim3(blocks_for((size_t)M * N)), dim3(256), 0,
                     s, M, N, ks, M_.gpart, epi);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adam on the FP32 master weights; FP16 copies of W1..W3 refreshed in place
// ---------------------------------------------------------------------------
__device__ inline void write_half(_Float16* w16, size_t i, float p) {
  if (i < MLP_OFF_B1) w16[MLP_H16_W1 + i] = (_Float16)p;
  else if (i >= MLP_OFF_W2 && i < MLP_OFF_B2) w16[MLP_H16_W2 + (i - MLP_OFF_W2)] = (_Float16)p;
  else if (i >= MLP_OFF_W3 && i < MLP_OFF_B3) w16[MLP_H16_W3 + (i - MLP_OFF_W3)] = (_Float16)p;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ params,
                                                       const float* __restrict__ grads,
                                                       float* __restrict__ m, float* __restrict__ v,
                                                       _Float16* __restrict__ w16, float lr,
                                                       float b1, float b2, float eps, float bc1,
                                                       float bc2) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  const float g = grads[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mhat = mi / bc1, vhat = vi / bc2;
  const float p = params[i] - lr * mhat / (sqrtf(vhat) + eps);
  params[i] = p;
  write_half(w16, i, p);
}

__global__ __launch_bounds__(256) void mlp_half_kernel(const float* __restrict__ params,
                                                       _Float16* __restrict__ w16) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  write_half(w16, i, params[i]);
}

// per-feature mean and (population) standard deviation, FP64 sums in a fixed
// order; features whose deviation is below 1e-6 keep scale 1
__global__ __launch_bounds__(MLP_NF) void mlp_norm_kernel(const float* __restrict__ X, int nb,
                                                          float* __restrict__ mu,
                                                          float* __restrict__ scale) {
  const int f = threadIdx.x;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += (double)X[(size_t)b * MLP_NF + f];
  const double mean = s / nb;
  double q = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double d = (double)X[(size_t)b * MLP_NF + f] - mean;
    q += d * d;
  }
  const double sd = sqrt(q / nb);
  mu[f] = (float)mean;
  scale[f] = sd < 1e-6 ? 1.0f : (float)sd;
}

}  // namespace

size_t mlp_layout(int max_batch, char* base, Mlp* M) {
  size_t cur = 0;
  auto take = [&](size_t bytes) -> char* {
    cur = (cur + 255) / 256 * 256;
    char* p = base ? base + cur : nullptr;
    cur += bytes;
    return p;
  };
  const size_t B = (size_t)max_batch;
  Mlp tmp;
  Mlp& Q = M ? *M : tmp;
  Q.params = reinterpret_cast<float*>(take(MLP_NPARAM * 4));
  Q.grads = reinterpret_cast<float*>(take(MLP_NPARAM * 4));
  Q.m = reinterpret_cast<float*>(take(MLP_NPARAM * 4));
  Q.v = reinterpret_cast<float*>(take(MLP_NPARAM * 4));
  Q.w16 = reinterpret_cast<_Float16*>(take(MLP_H16_N * 2));
  Q.mu = reinterpret_cast<float*>(take(MLP_NF * 4));
  Q.scale = reinterpret_cast<float*>(take(MLP_NF * 4));
  Q.rows = reinterpret_cast<int*>(take(B * 4));
  Q.h0 = reinterpret_cast<_Float16*>(take(B * MLP_NF * 2));
  Q.z1 = reinterpret_cast<float*>(take(B * MLP_NH * 4));
  Q.h1 = reinterpret_cast<_Float16*>(take(B * MLP_NH * 2));
  Q.z2 = reinterpret_cast<float*>(take(B * MLP_NH * 4));
  Q.h2 = reinterpret_cast<_Float16*>(take(B * MLP_NH * 2));
  Q.z3 = reinterpret_cast<float*>(take(B * MLP_NH * 4));
  Q.h3 = reinterpret_cast<float*>(take(B * MLP_NH * 4));
  Q.y = reinterpret_cast<float*>(take(B * 4));
  Q.dz4 = reinterpret_cast<float*>(take(B * 4));
  Q.dza = reinterpret_cast<float*>(take(B * MLP_NH * 4));
  Q.dzb = reinterpret_cast<float*>(take(B * MLP_NH * 4));
  Q.loss = reinterpret_cast<double*>(take(8));
  Q.gpart = reinterpret_cast<float*>(take(MLP_PART_FLOATS * 4));
  return (cur + 255) / 256 * 256;
}

size_t mlp_act_layout(int rows, char* base, Mlp* M) {
  size_t cur = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base + cur;
    cur += mlp_a256(bytes);
    return p;
  };
  const size_t B = (size_t)rows;
  M->h0 = reinterpret_cast<_Float16*>(take(B * MLP_NF * 2));
  M->z1 = reinterpret_cast<float*>(take(B * MLP_NH * 4));
  M->h1 = reinterpret_cast<_Float16*>(take(B * MLP_NH * 2));
  M->z2 = reinterpret_cast<float*>(take(B * MLP_NH * 4));
  M->h2 = reinterpret_cast<_Float16*>(take(B * MLP_NH * 2));
  M->z3 = reinterpret_cast<float*>(take(B * MLP_NH * 4));
  M->h3 = reinterpret_cast<float*>(take(B * MLP_NH * 4));
  M->y = reinterpret_cast<float*>(take(B * 4));
  M->dz4 = reinterpret_cast<float*>(take(B * 4));
  return cur;
}

hipError_t mlp_forward(const Mlp& M, const float* X, const int* rows, int nb, double* pred,
                       hipStream_t s) {
  if (nb < 1 || nb > M.max_batch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_input_kernel, dim3(blocks_for((size_t)nb * MLP_NF)), dim3(256), 0, s,
                     X, rows, nb, M.mu, M.scale, M.h0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid(MLP_NH / 64, (nb + 63) / 64);
  hipLaunchKernelGGL(mlp_fwd_kernel<true>, grid, dim3(256), 0, s, M.h0, MLP_NF,
                     M.w16 + MLP_H16_W1, M.params + MLP_OFF_B1, nb, M.z1, (void*)M.h1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_fwd_kernel<true>, grid, dim3(256), 0, s, M.h1, MLP_NH,
                     M.w16 + MLP_H16_W2, M.params + MLP_OFF_B2, nb, M.z2, (void*)M.h2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_fwd_kernel<false>, grid, dim3(256), 0, s, M.h2, MLP_NH,
                     M.w16 + MLP_H16_W3, M.params + MLP_OFF_B3, nb, M.z3, (void*)M.h3);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_head_kernel, dim3((nb + 3) / 4), dim3(256), 0, s, M.h3, M.params, nb,
                     M.y, pred, (const float*)nullptr, rows, M.dz4);
  return hipGetLastError();
}

hipError_t mlp_backward(const Mlp& M, const float* t, const int* rows, int nb, hipStream_t s) {
  if (nb < 1 || nb > M.max_batch) return hipErrorInvalidValue;
  hipError_t e;
  // dz4 and the loss
  hipLaunchKernelGGL(mlp_head_kernel, dim3((nb + 3) / 4), dim3(256), 0, s, M.h3, M.params, nb,
                     M.y, (double*)nullptr, t, rows, M.dz4);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, s, M.y, t, rows, nb, M.loss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // output layer: dW4 = dz4^T h3, db4 = sum dz4, dz3 = dz4 w4 g'(z3)
  hipLaunchKernelGGL(mlp_colsum_kernel, dim3(MLP_NH / 64), dim3(256), 0, s, M.h3, MLP_NH,
                     MLP_NH, M.dz4, nb, M.grads + MLP_OFF_W4);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_colsum_kernel, dim3(1), dim3(256), 0, s, M.dz4, 1, 1,
                     (const float*)nullptr, nb, M.grads + MLP_OFF_B4);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_head_bwd_kernel, dim3(blocks_for((size_t)nb * MLP_NH)), dim3(256), 0, s,
                     M.dz4, M.params, M.z3, nb, M.dza);
  if ((e = hipGetLastError()) != hipSuccess) return e;

  struct Layer {
    const void* hin; bool hin_f16; int in; size_t offW, offB, offH16; const float* zprev;
  };
  const Layer layers[3] = {
      {M.h0, true, MLP_NF, MLP_OFF_W1, MLP_OFF_B1, MLP_H16_W1, nullptr},
      {M.h1, true, MLP_NH, MLP_OFF_W2, MLP_OFF_B2, MLP_H16_W2, M.z1},
      {M.h2, true, MLP_NH, MLP_OFF_W3, MLP_OFF_B3, MLP_H16_W3, M.z2},
  };
  float* dz = M.dza;
  float* dzn = M.dzb;
  for (int l = 2; l >= 0; --l) {
    const Layer& L = layers[l];
    // dW[o][i] = sum_b dz[b][o] h[b][i]
    e = run_mlp_gemm(M, MLP_NH, L.in, nb, AMajorM{dz, MLP_NH},
                     BRows<_Float16>{reinterpret_cast<const _Float16*>(L.hin), L.in},
                     EpiGrad{M.grads + L.offW, L.in}, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_colsum_kernel, dim3(MLP_NH / 64), dim3(256), 0, s, dz, MLP_NH, MLP_NH,
                       (const float*)nullptr, nb, M.grads + L.offB);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (l == 0) break;
    // dz_prev[b][i] = (sum_o dz[b][o] W[o][i]) g'(z_prev[b][i])
    e = run_mlp_gemm(M, nb, L.in, MLP_NH, AMajorK{dz, MLP_NH},
                     BRows<_Float16>{M.w16 + L.offH16, L.in},
                     EpiGeluBack{dzn, L.zprev, L.in}, s);
    if (e != hipSuccess) return e;
    float* t2 = dz;
    dz = dzn;
    dzn = t2;
  }
  return hipSuccess;
}

hipError_t mlp_adam(const Mlp& M, float lr, float b1, float b2, float eps, float bc1, float bc2,
                    hipStream_t s) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(blocks_for(MLP_NPARAM)), dim3(256), 0, s, M.params,
                     M.grads, M.m, M.v, M.w16, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t mlp_refresh_half(const Mlp& M, hipStream_t s) {
  hipLaunchKernelGGL(mlp_half_kernel, dim3(blocks_for(MLP_NPARAM)), dim3(256), 0, s, M.params,
                     M.w16);
  return hipGetLastError();
}

hipError_t mlp_fit_norm(const Mlp& M, const float* X, int nb, hipStream_t s) {
  if (nb < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_norm_kernel, dim3(1), dim3(MLP_NF), 0, s, X, nb, M.mu, M.scale);
  return hipGetLastError();
}

}  // namespace kpcg
