// Construction of the Kronecker approximation and its SVD on the device.
//
// Section 3, eq. (AKronSVD) and Section 5, eq. (KronSumDecomp).  The
// paper builds the Frobenius-optimal term A_r (x) A_c with IR Tools without
// stating the construction.  Reading used: A = sum_{u,v} P[u][v] Z_v (x) Z_u
// over shift matrices with disjoint supports and ||Z_d||_F^2 = n - |d|, so
//   ||A - T(a) (x) T(c)||_F^2 = sum w_u w_v (P[u][v] - c_u a_v)^2,
//   w_k = n - |k - h|,
// minimised by the leading singular triple (s1, u1, v1) of
// W^{1/2} P W^{1/2}: c = sqrt(s1) u1 / sqrt(w), a = sqrt(s1) v1 / sqrt(w).
// A_c = T(c) (acts on the row index), A_r = T(a), T(f)[i][i'] = f[h+i-i'].
// Both factors get FP64 SVDs (the paper also computes them in double):
// rocSOLVER's symmetric eigensolver when the profile is symmetric (every
// point-symmetric PSF), its general SVD otherwise.  V_c, V_r are then stored
// in FP32 / FP16 / FP8 with block exponents, U_c, U_r in FP32 and the
// singular values in FP64.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"

namespace kpcg {

// Frobenius weight of PSF offset k - h in one factor: ||Z_d||_F^2 = n - |d|
// for the zero boundary's shift matrices, ||C_d||_F^2 = n for the periodic
// boundary's cyclic shifts (so its optimal term is the plain PSF SVD); the
// reflexive boundary takes the plain PSF SVD too (its reflected shifts have
// n entries each but overlap, so no weighting makes it exactly optimal).
__device__ inline double psf_weight(int k, int h, int n, int bc) {
  return bc != KP_BC_ZERO ? (double)n : (double)(n - abs(k - h));
}

// Weighted PSF, column-major K x K for the solver.
__global__ void weighted_psf_kernel(const double* __restrict__ psf, int K, int n, int bc,
                                    double* __restrict__ pw) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * K) return;
  const int k = idx / K, l = idx - k * K;          // psf[k][l] row-major
  const int h = (K - 1) / 2;
  const double wk = psf_weight(k, h, n, bc), wl = psf_weight(l, h, n, bc);
  pw[k + (size_t)l * K] = sqrt(wk * wl) * psf[idx];
}

// Profiles c (column factor) and a (row factor) from the leading singular
// triple; sign fixed so that sum(c) > 0.  One block.
__global__ void profiles_kernel(const double* __restrict__ S, const double* __restrict__ U,
                                const double* __restrict__ Vt, int K, int n, int bc,
                                double* __restrict__ c, double* __restrict__ a) {
  __shared__ double red[64];
  const int h = (K - 1) / 2;
  const double s1 = sqrt(S[0]);
  double part = 0.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) part += U[k];
  red[threadIdx.x] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) t += red[i];
    red[0] = t;
  }
  __syncthreads();
  const double sg = red[0] < 0.0 ? -1.0 : 1.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double w = sqrt(psf_weight(k, h, n, bc));
    c[k] = sg * s1 * U[k] / w;                      // U(k, 0)
    a[k] = sg * s1 * Vt[(size_t)k * K] / w;         // Vt(0, k)
  }
}

// All t terms of the Kronecker sum (Section 5, eq. (KronSumDecomp)) from the
// weighted PSF SVD: prof[k][d] = sqrt(s_k) U(d,k) / sqrt(w_d) (column
// profiles) and prof[t + k][d] = sqrt(s_k) V(d,k) / sqrt(w_d) (row profiles),
// so that P = sum_k c_k a_k^T.  The sign of a pair (c_k, a_k) is immaterial
// for the diagonal built from them.
__global__ void all_profiles_kernel(const double* __restrict__ S, const double* __restrict__ U,
                                    const double* __restrict__ Vt, int K, int n, int bc, int t,
                                    double* __restrict__ prof) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= t * K) return;
  const int k = idx / K, d = idx - k * K, h = (K - 1) / 2;
  const double g = sqrt(S[k]) / sqrt(psf_weight(d, h, n, bc));
  prof[idx] = g * U[d + (size_t)k * K];                  // U(d, k)
  prof[t * K + idx] = g * Vt[k + (size_t)d * K];         // Vt(k, d) = V(d, k)
}

// Per column a of one factor's V (row-major n x n, FP64): the Gram matrix of
// y_k = T(f_k) V(:, a) over the t profiles f_k of that factor,
//     G[k * t + l][a] = sum_i y_k[i] y_l[i],
// with (T(f) v)[i] = sum_d f[d] v[i + h - d] (zero outside [0, n); for the
// periodic boundary the circulant C(f), v indexed mod n).  One
// block per column; the column (zero padded by h on both sides) and the
// profiles sit in LDS, y is formed GRAM_CH rows at a time, and each thread
// accumulates up to GRAM_PAIRS of the t (t + 1) / 2 pairs k <= l in FP64.
constexpr int GRAM_NT = 256;
constexpr int GRAM_CH = 64;
constexpr int GRAM_PAIRS = 8;              // 63 * 64 / 2 = 2016 <= 256 * 8

size_t gram_lds_bytes(int t, int K, int n) {
  return sizeof(double) * ((size_t)t * K + (size_t)n + K - 1 + (size_t)t * (GRAM_CH + 1));
}

__global__ __launch_bounds__(GRAM_NT) void gram_kernel(const double* __restrict__ V,
                                                       const double* __restrict__ prof, int t,
                                                       int K, int n, int bc,
                                                       double* __restrict__ G) {
  extern __shared__ double gsm[];
  double* sp = gsm;                               // [t][K]
  double* sv = sp + t * K;                        // [n + K - 1]: sv[m] = v[m - h]
  double* sy = sv + n + K - 1;                    // [t][GRAM_CH + 1]
  const int a = blockIdx.x, tid = threadIdx.x, h = (K - 1) / 2;
  for (int i = tid; i < t * K; i += GRAM_NT) sp[i] = prof[i];
  for (int m = tid; m < n + K - 1; m += GRAM_NT) {
    int i = m - h;
    if (bc == KP_BC_PERIODIC) i = i < 0 ? i + n : (i >= n ? i - n : i);   // h < n
    else if (bc == KP_BC_REFLEXIVE) i = i < 0 ? -i - 1 : (i >= n ? 2 * n - 1 - i : i);
    sv[m] = (i >= 0 && i < n) ? V[(size_t)i * n + a] : 0.0;
  }
  // this thread's pairs p = tid + GRAM_NT q in the order (0,0), (0,1), ...
  int pk[GRAM_PAIRS], pl[GRAM_PAIRS];
  double acc[GRAM_PAIRS];
#pragma unroll
  for (int q = 0; q < GRAM_PAIRS; ++q) { pk[q] = -1; pl[q] = 0; acc[q] = 0.0; }
  {
    int p = 0;
    for (int k = 0; k < t; ++k)
      for (int l = k; l < t; ++l, ++p) {
        const int q = (p - tid) / GRAM_NT;
        if (p >= tid && (p - tid) % GRAM_NT == 0 && q < GRAM_PAIRS) { pk[q] = k; pl[q] = l; }
      }
  }
  __syncthreads();
  constexpr int LD = GRAM_CH + 1;
  for (int i0 = 0; i0 < n; i0 += GRAM_CH) {
    for (int idx = tid; idx < t * GRAM_CH; idx += GRAM_NT) {
      const int k = idx / GRAM_CH, r = idx - k * GRAM_CH, i = i0 + r;
      double y = 0.0;
      if (i < n) {
        const double* f = sp + k * K;
        const double* v = sv + i + 2 * h;         // v[i + h - d] = sv[i + 2h - d]
        for (int d = 0; d < K; ++d) y = fma(f[d], v[-d], y);
      }
      sy[k * LD + r] = y;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < GRAM_PAIRS; ++q) {
      if (pk[q] < 0) continue;
      const double* yk = sy + pk[q] * LD;
      const double* yl = sy + pl[q] * LD;
      double sum = 0.0;
      for (int r = 0; r < GRAM_CH; ++r) sum = fma(yk[r], yl[r], sum);
      acc[q] += sum;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < GRAM_PAIRS; ++q) {
    if (pk[q] < 0) continue;
    G[((size_t)pk[q] * t + pl[q]) * n + a] = acc[q];
    G[((size_t)pl[q] * t + pk[q]) * n + a] = acc[q];
  }
}

// FP32 copies of a row-major n x n FP64 matrix, as is and transposed
__global__ void to_f32_kernel(const double* __restrict__ src, int n, float* __restrict__ dst,
                              float* __restrict__ dst_t) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const float v = (float)src[idx];
  const size_t i = idx / n, j = idx - i * n;
  dst[idx] = v;
  dst_t[j * n + i] = v;
}

// Column-major factor from a profile: the banded Toeplitz T(f)[i][i'] =
// f[h + i - i'] (zero boundary), the circulant C(f)[i][i'] = f[h + d] with
// d = i - i' mod n taken in [-h, h] (periodic boundary, K <= n), or the
// reflexive R(f)[i][i'] = sum of f[h + d] over the d with refl(i - d) = i':
// d = i - i' (direct), i + i' + 1 (reflected at the top) and i + i' + 1 - 2n
// (at the bottom), each if |d| <= h (reflexive boundary, K <= n).
__global__ void toeplitz_kernel(const double* __restrict__ f, int K, int n, int bc,
                                double* __restrict__ t) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int i = (int)(idx % n), ip = (int)(idx / n);   // t[i + ip*n]
  const int h = (K - 1) / 2;
  int d = i - ip;
  if (bc == KP_BC_REFLEXIVE) {
    const int d2 = i + ip + 1, d3 = i + ip + 1 - 2 * n;
    double v = (d >= -h && d <= h) ? f[h + d] : 0.0;
    if (d2 >= -h && d2 <= h) v += f[h + d2];
    if (d3 >= -h && d3 <= h) v += f[h + d3];
    t[idx] = v;
    return;
  }
  if (bc == KP_BC_PERIODIC) {
    if (d > h) d -= n;
    else if (d < -h) d += n;
  }
  t[idx] = (d >= -h && d <= h) ? f[h + d] : 0.0;
}

// Reduced-precision construction (KP_SETUP_LOWP): the factor scaled by 2^e
// (its largest |entry| in [2^13, 2^14)) and rounded to FP16, held in FP32
// for the FP32 factorisation; and the widening of its FP32 results.
__global__ void fp16_factor_kernel(const double* __restrict__ t, size_t count, int e,
                                   float* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) out[idx] = (float)(_Float16)ldexp(t[idx], e);
}

__global__ void widen_kernel(const float* __restrict__ src, size_t count, double scale,
                             double* __restrict__ dst) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) dst[idx] = scale * (double)src[idx];
}

// From the column-major gesvd outputs: Vt (n x n, Vt(a,i) = V(i,a)) and U.
//   Vrm[i*n+a]  = V(i,a)   = Vt[a + i*n]   (same memory order)
//   VTrm[a*n+i] = V(i,a)                   (transpose)
//   UTrm[a*n+i] = U(i,a)   = U[i + a*n]    (same memory order)
__global__ void factors_kernel(const double* __restrict__ Vt, const double* __restrict__ U,
                               int n, float* __restrict__ V32, float* __restrict__ VT32,
                               _Float16* __restrict__ V16, _Float16* __restrict__ VT16,
                               float* __restrict__ UT32) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int a = (int)(idx % n), i = (int)(idx / n);
  const double v = Vt[idx];                 // V(i, a) at row-major [i][a]
  V32[idx] = (float)v;
  V16[idx] = (_Float16)v;
  VT32[(size_t)a * n + i] = (float)v;
  VT16[(size_t)a * n + i] = (_Float16)v;
  UT32[idx] = (float)U[idx];
}

// Symmetric factors (point-symmetric PSFs give symmetric Toeplitz factors):
// from the eigendecomposition T = Q diag(w) Q^T, the SVD has s_a = |w_p(a)|
// in descending order, V(:,a) = Q(:,p(a)), U(:,a) = sign(w_p(a)) Q(:,p(a)).
// rank_kernel computes the order p (ties by index), gather_eig_kernel writes
// s, Vt (column-major, Vt(a,i) = V(i,a)) and U (column-major) in the layout
// the general SVD path produces.
__global__ void rank_kernel(const double* __restrict__ w, int n, int* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ai = fabs(w[i]);
  int r = 0;
  for (int j = 0; j < n; ++j) {
    const double aj = fabs(w[j]);
    r += (aj > ai) || (aj == ai && j < i);
  }
  perm[r] = i;
}

__global__ void gather_eig_kernel(const double* __restrict__ Q, const double* __restrict__ w,
                                  const int* __restrict__ perm, int n, double* __restrict__ sig,
                                  double* __restrict__ Vt, double* __restrict__ U) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int i = (int)(idx % n), a = (int)(idx / n);      // element (i, a)
  const int p = perm[a];
  const double q = Q[i + (size_t)p * n];
  const double sg = w[p] < 0.0 ? -1.0 : 1.0;
  Vt[a + (size_t)i * n] = q;
  U[i + (size_t)a * n] = sg * q;
  if (i == 0) sig[a] = fabs(w[p]);
}

__global__ void sigma_kernel(const double* __restrict__ s, int n, float* __restrict__ s2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s2[i] = (float)(s[i] * s[i]);
}

// Taps for the direct blur: row-major K x KQ, zero padded; flip = 180 deg.
__global__ void taps_kernel(const double* __restrict__ psf, int K, int KQ,
                            float* __restrict__ t32, float* __restrict__ t32f,
                            double* __restrict__ t64, double* __restrict__ t64f) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * KQ) return;
  const int a = idx / KQ, b = idx - a * KQ;
  double v = 0.0, vf = 0.0;
  if (b < K) {
    v = psf[a * K + b];
    vf = psf[(K - 1 - a) * K + (K - 1 - b)];
  }
  t32[idx] = (float)v;
  t32f[idx] = (float)vf;
  t64[idx] = v;
  t64f[idx] = vf;
}

// ---------------------------------------------------------------------------
// FP8 e4m3 copies of the factors with one power-of-two exponent per 32
// consecutive entries along the contraction dimension of each GEMM that
// consumes them (every stored factor is K-contiguous, so: per row, per 32
// columns).
// ---------------------------------------------------------------------------
__device__ inline int e8m0_for_amax(float amax) {
  // smallest e with amax * 2^-e <= 448 ; returned biased by 127
  if (!(amax > 0.0f)) return 1;            // any exponent works for an all-zero block
  int e;
  const float m = frexpf(amax / 448.0f, &e);   // amax/448 = m 2^e, m in [0.5,1)
  if (m == 0.5f) e -= 1;
  e += 127;
  return e < 1 ? 1 : (e > 254 ? 254 : e);
}

__device__ inline uint8_t to_e4m3(float v) {
  // RNE with saturation to +-448 (the value is already scaled into range)
  const int packed = __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false);
  return (uint8_t)(packed & 0xff);
}

__global__ void quant_rows_e4m3_kernel(const float* __restrict__ src, int n,
                                       uint8_t* __restrict__ codes,
                                       uint8_t* __restrict__ exps) {
  // one thread per (row, 32-block)
  const int nb = (n + 31) / 32;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * nb) return;
  const int row = idx / nb, blk = idx - row * nb;
  const int j0 = blk * 32, j1 = min(n, j0 + 32);
  float amax = 0.0f;
  for (int j = j0; j < j1; ++j) amax = fmaxf(amax, fabsf(src[(size_t)row * n + j]));
  const int eb = e8m0_for_amax(amax);
  exps[idx] = (uint8_t)eb;
  const float inv = ldexpf(1.0f, 127 - eb);
  for (int j = j0; j < j1; ++j)
    codes[(size_t)row * n + j] = to_e4m3(src[(size_t)row * n + j] * inv);
}

#define SCHK(x)                                                     \
  do {                                                              \
    rocblas_status st_ = (x);                                       \
    if (st_ != rocblas_status_success) { rc = KP_ERR_SOLVER; goto done; } \
  } while (0)
#define HCHK(x)                                                     \
  do {                                                              \
    if ((x) != hipSuccess) { rc = KP_ERR_HIP; goto done; }           \
  } while (0)

// KPCG_GENERAL_SVD=1 forces the general SVD for every factor (used to check
// that both paths give the same preconditioner).
static bool force_general_svd() {
  const char* v = std::getenv("KPCG_GENERAL_SVD");
  return v != nullptr && v[0] == '1';
}

// ---------------------------------------------------------------------------
// Device memory of the construction.  Nothing here is allocated: every
// buffer, rocSOLVER's own workspace included, is a view into the plan's
// workspace (the region the solver's vectors use later), and rocBLAS is
// handed that workspace with rocblas_set_workspace.  One rocBLAS handle per
// device serves every construction in the process, under a lock.
// ---------------------------------------------------------------------------
namespace {

std::mutex g_setup_mu;
std::map<int, rocblas_handle> g_handles;                      // device -> handle
std::map<std::pair<int, std::pair<int, int>>, size_t> g_ws;   // (device, (n, k)) -> bytes

// the current device's handle (caller holds g_setup_mu)
rocblas_handle device_handle() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  auto it = g_handles.find(dev);
  if (it != g_handles.end()) return it->second;
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
  g_handles[dev] = h;
  return h;
}

// rocSOLVER / rocBLAS device workspace the construction's calls need, by
// rocBLAS's size query (no call computes anything in query mode; the
// pointers only have to be non-null).  Caller holds g_setup_mu.  0 on error.
size_t solver_ws_bytes_locked(int n, int K) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const auto key = std::make_pair(dev, std::make_pair(n, K));
  auto it = g_ws.find(key);
  if (it != g_ws.end()) return it->second;
  rocblas_handle h = device_handle();
  if (!h) return 0;
  double* dp = reinterpret_cast<double*>(static_cast<uintptr_t>(256));
  float* fp = reinterpret_cast<float*>(static_cast<uintptr_t>(256));
  rocblas_int* ip = reinterpret_cast<rocblas_int*>(static_cast<uintptr_t>(256));
  size_t bytes = 0;
  bool ok = rocblas_start_device_memory_size_query(h) == rocblas_status_success;
  if (ok) {
    const double one = 1.0, zero = 0.0;
    // every call the construction can make (the symmetric and general
    // paths, FP64 and the reduced-precision FP32 variants, the D0 product
    // with up to K^2 term pairs); statuses other than success are expected
    // in query mode and ignored
    rocsolver_dgesvd(h, rocblas_svect_all, rocblas_svect_all, K, K, dp, K, dp, dp, K, dp, K,
                     dp, rocblas_outofplace, ip);
    rocsolver_dgesvd(h, rocblas_svect_all, rocblas_svect_all, n, n, dp, n, dp, dp, n, dp, n, dp,
                     rocblas_outofplace, ip);
    rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, dp, n, dp, dp, ip);
    rocsolver_sgesvd(h, rocblas_svect_all, rocblas_svect_all, n, n, fp, n, fp, fp, n, fp, n, fp,
                     rocblas_outofplace, ip);
    rocsolver_ssyevd(h, rocblas_evect_original, rocblas_fill_upper, n, fp, n, fp, fp, ip);
    rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n,
                  (rocblas_int)((size_t)K * K), &one, dp, n, dp, n, &zero, dp, n);
    ok = rocblas_stop_device_memory_size_query(h, &bytes) == rocblas_status_success;
  }
  if (!ok) return 0;
  bytes = bytes < 256 ? 256 : bytes;
  g_ws[key] = bytes;
  return bytes;
}

}  // namespace

// Views of the construction's buffers; see scratch_layout.
struct SetupScratch {
  double *dpsf, *pw, *spsf, *upsf, *vpsf, *e, *prof, *T, *U, *Vt, *wv, *pall, *G2, *D64;
  rocblas_int* info;
  int* perm;
  float *T32, *U32, *Vt32, *s32, *e32;
  void* fftG;                // PSF rows' spectra of the FFT normal operator
  void* rocws;
  size_t rocws_bytes;
};

// Lay the construction's buffers out from `base` (NULL: sizes only), with
// rocws bytes of solver workspace first, and return the bytes they take.  The term count t is at most K, so the Gram matrices of the
// exact diagonal are sized for t = K.
static size_t scratch_layout(int n, int K, size_t rocws, char* base, SetupScratch* S) {
  const size_t nn = (size_t)n * n, KK = (size_t)K * K;
  size_t cur = 0;
  auto take = [&](size_t bytes) -> char* {
    cur = (cur + 255) / 256 * 256;
    char* p = base ? base + cur : nullptr;
    cur += bytes;
    return p;
  };
  SetupScratch tmp;
  SetupScratch& Q = S ? *S : tmp;
  Q.rocws = take(rocws);
  Q.rocws_bytes = rocws;
  Q.dpsf = (double*)take(8 * KK);
  Q.pw = (double*)take(8 * KK);
  Q.spsf = (double*)take(8 * (size_t)K);
  Q.upsf = (double*)take(8 * KK);
  Q.vpsf = (double*)take(8 * KK);
  Q.e = (double*)take(8 * (size_t)(n > K ? n : K));
  Q.prof = (double*)take(8 * 2 * (size_t)K);
  Q.T = (double*)take(8 * nn);
  Q.U = (double*)take(8 * nn);
  Q.Vt = (double*)take(8 * nn);
  Q.info = (rocblas_int*)take(sizeof(rocblas_int));
  Q.wv = (double*)take(8 * (size_t)n);
  Q.perm = (int*)take(sizeof(int) * (size_t)n);
  Q.T32 = (float*)take(4 * nn);
  Q.U32 = (float*)take(4 * nn);
  Q.Vt32 = (float*)take(4 * nn);
  Q.s32 = (float*)take(4 * (size_t)n);
  Q.e32 = (float*)take(4 * (size_t)n);
  Q.pall = (double*)take(8 * 2 * KK);
  Q.G2 = (double*)take(8 * 2 * KK * (size_t)n);
  Q.D64 = (double*)take(8 * nn);
  Q.fftG = take(16 * (size_t)K * (size_t)(fft_table_length(n, K) / 2 + 1));
  return (cur + 255) / 256 * 256;
}

size_t setup_scratch_bytes(int n, int K) {
  size_t rocws;
  {
    std::lock_guard<std::mutex> lk(g_setup_mu);
    rocws = solver_ws_bytes_locked(n, K);
  }
  if (rocws == 0) return 0;
  return scratch_layout(n, K, rocws, nullptr, nullptr);
}

int build_factors(Plan& P, const double* psf_host, char* scratch, hipStream_t s) {
  const int n = P.n, K = P.k;
  const size_t nn = (size_t)n * n;
  int rc = KP_OK;
  std::lock_guard<std::mutex> lk(g_setup_mu);
  rocblas_handle handle = device_handle();
  if (!handle) return KP_ERR_SOLVER;
  SetupScratch S;
  const size_t rocws = solver_ws_bytes_locked(n, K);
  if (rocws == 0) return KP_ERR_SOLVER;
  scratch_layout(n, K, rocws, scratch, &S);
  double *dpsf = S.dpsf, *pw = S.pw, *spsf = S.spsf, *upsf = S.upsf, *vpsf = S.vpsf, *e = S.e,
         *prof = S.prof, *T = S.T, *U = S.U, *Vt = S.Vt;
  rocblas_int* info = S.info;
  double* wv = S.wv;
  int* perm = S.perm;
  double *pall = S.pall, *G2 = S.G2, *D64 = S.D64;          // exact KP-basis diagonal
  float *T32 = S.T32, *U32 = S.U32, *Vt32 = S.Vt32, *s32 = S.s32, *e32 = S.e32;
  int lexp[2] = {0, 0};                                     // KP_SETUP_LOWP factor scales
  int tall = 0;
  size_t glds = 0;
  bool symmetric[2] = {false, false};
  std::vector<double> hs(K);
  rocblas_int hinfo = 0;
  const int nthr = 256;
  const unsigned gnn = (unsigned)((nn + nthr - 1) / nthr);

  SCHK(rocblas_set_stream(handle, s));
  SCHK(rocblas_set_workspace(handle, S.rocws, S.rocws_bytes));
  HCHK(hipMemcpyAsync(dpsf, psf_host, sizeof(double) * K * K, hipMemcpyHostToDevice, s));

  // blur taps
  hipLaunchKernelGGL(taps_kernel, dim3((K * P.kq + 255) / 256), dim3(256), 0, s, dpsf, K, P.kq,
                     P.taps32, P.taps32_flip, P.taps64, P.taps64_flip);
  {
    // MFMA tap fragments, scaled so the largest |tap| sits in [2^13, 2^14)
    float mx = 0.0f;
    for (int i = 0; i < K * K; ++i) mx = std::fmax(mx, std::fabs((float)psf_host[i]));
    P.mfma_exq = mx > 0.0f ? 13 - std::ilogb(mx) : 0;
    HCHK(build_mfma_taps(P, s));
  }
  HCHK(hipGetLastError());
  // tables of the FFT form of the normal operator
  HCHK(build_fft_tables(P, dpsf, S.fftG, s));

  // weighted PSF SVD
  hipLaunchKernelGGL(weighted_psf_kernel, dim3((K * K + 255) / 256), dim3(256), 0, s, dpsf, K,
                     n, P.bc, pw);
  HCHK(hipGetLastError());
  SCHK(rocsolver_dgesvd(handle, rocblas_svect_all, rocblas_svect_all, K, K, pw, K, spsf, upsf,
                        K, vpsf, K, e, rocblas_outofplace, info));
  HCHK(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
  HCHK(hipMemcpyAsync(hs.data(), spsf, sizeof(double) * K, hipMemcpyDeviceToHost, s));
  HCHK(hipStreamSynchronize(s));
  if (hinfo != 0) { rc = KP_ERR_SOLVER; goto done; }
  hipLaunchKernelGGL(profiles_kernel, dim3(1), dim3(64), 0, s, spsf, upsf, vpsf, K, n, P.bc,
                     prof, prof + K);
  HCHK(hipGetLastError());

  {
    // symmetric profiles give symmetric Toeplitz factors: use the
    // (much faster) symmetric eigensolver for them
    std::vector<double> hp(2 * K);
    HCHK(hipMemcpyAsync(hp.data(), prof, sizeof(double) * 2 * K, hipMemcpyDeviceToHost, s));
    HCHK(hipStreamSynchronize(s));
    for (int f = 0; f < 2; ++f) {
      double mx = 0.0, asym = 0.0;
      for (int k = 0; k < K; ++k) mx = std::fmax(mx, std::fabs(hp[f * K + k]));
      for (int k = 0; k < K; ++k)
        asym = std::fmax(asym, std::fabs(hp[f * K + k] - hp[f * K + K - 1 - k]));
      symmetric[f] = asym <= 1e-13 * mx && !force_general_svd();
      // the factor's entries are the profile's values at offsets |k - h| < n
      double fmx = 0.0;
      for (int k = 0; k < K; ++k)
        if (std::abs(k - (K - 1) / 2) < n) fmx = std::fmax(fmx, std::fabs(hp[f * K + k]));
      lexp[f] = fmx > 0.0 ? 13 - std::ilogb(fmx) : 0;
    }
  }
  {
    double tot = 0.0, rest = 0.0;
    for (int i = 0; i < K; ++i) tot += hs[i] * hs[i];
    for (int i = 1; i < K; ++i) rest += hs[i] * hs[i];
    P.kp_err = tot > 0 ? std::sqrt(rest / tot) : 0.0;
    int t = 0;
    for (int i = 0; i < K; ++i)
      if (hs[i] > 1e-12 * hs[0]) ++t;
    P.terms = t;
    tall = t;
  }
  // every term's profiles, and room for the per-factor Gram matrices of the
  // exact diagonal D0 = diag(V^T A^T A V) (built below)
  if (tall > 0) {
    hipLaunchKernelGGL(all_profiles_kernel, dim3((tall * K + 255) / 256), dim3(256), 0, s, spsf,
                       upsf, vpsf, K, n, P.bc, tall, pall);
    HCHK(hipGetLastError());
    glds = gram_lds_bytes(tall, K, n);
    if (glds > 65536)
      HCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(gram_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)glds));
  }

  // the two factors: c -> A_c (column factor), a -> A_r (row factor)
  for (int f = 0; f < 2; ++f) {
    const double* prof_f = prof + f * K;
    double* sig = f == 0 ? P.sc : P.sr;
    hipLaunchKernelGGL(toeplitz_kernel, dim3(gnn), dim3(nthr), 0, s, prof_f, K, n, P.bc, T);
    HCHK(hipGetLastError());
    if (P.lowp) {
      // FP16 factor, FP32 factorisation, results widened (the scale undone
      // on the singular values / eigenvalues)
      const double unscale = std::ldexp(1.0, -lexp[f]);
      hipLaunchKernelGGL(fp16_factor_kernel, dim3(gnn), dim3(nthr), 0, s, T, nn, lexp[f], T32);
      HCHK(hipGetLastError());
      if (symmetric[f]) {
        SCHK(rocsolver_ssyevd(handle, rocblas_evect_original, rocblas_fill_upper, n, T32, n, s32,
                              e32, info));
        hipLaunchKernelGGL(widen_kernel, dim3(gnn), dim3(nthr), 0, s, T32, nn, 1.0, T);
        hipLaunchKernelGGL(widen_kernel, dim3((n + 255) / 256), dim3(256), 0, s, s32,
                           (size_t)n, unscale, wv);
        hipLaunchKernelGGL(rank_kernel, dim3((n + 255) / 256), dim3(256), 0, s, wv, n, perm);
        hipLaunchKernelGGL(gather_eig_kernel, dim3(gnn), dim3(nthr), 0, s, T, wv, perm, n, sig,
                           Vt, U);
      } else {
        SCHK(rocsolver_sgesvd(handle, rocblas_svect_all, rocblas_svect_all, n, n, T32, n, s32,
                              U32, n, Vt32, n, e32, rocblas_outofplace, info));
        hipLaunchKernelGGL(widen_kernel, dim3((n + 255) / 256), dim3(256), 0, s, s32,
                           (size_t)n, unscale, sig);
        hipLaunchKernelGGL(widen_kernel, dim3(gnn), dim3(nthr), 0, s, U32, nn, 1.0, U);
        hipLaunchKernelGGL(widen_kernel, dim3(gnn), dim3(nthr), 0, s, Vt32, nn, 1.0, Vt);
      }
      HCHK(hipGetLastError());
    } else if (symmetric[f]) {
      SCHK(rocsolver_dsyevd(handle, rocblas_evect_original, rocblas_fill_upper, n, T, n, wv, e,
                            info));
      hipLaunchKernelGGL(rank_kernel, dim3((n + 255) / 256), dim3(256), 0, s, wv, n, perm);
      hipLaunchKernelGGL(gather_eig_kernel, dim3(gnn), dim3(nthr), 0, s, T, wv, perm, n, sig, Vt,
                         U);
      HCHK(hipGetLastError());
    } else {
      SCHK(rocsolver_dgesvd(handle, rocblas_svect_all, rocblas_svect_all, n, n, T, n, sig, U, n,
                            Vt, n, e, rocblas_outofplace, info));
    }
    HCHK(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
    HCHK(hipStreamSynchronize(s));
    if (hinfo != 0) { rc = KP_ERR_SOLVER; goto done; }
    if (tall > 0) {
      // Gram matrices of T(f_k) V(:, a) over this factor's profiles (Vt holds
      // V row-major here)
      hipLaunchKernelGGL(gram_kernel, dim3(n), dim3(GRAM_NT), glds, s, Vt, pall + f * tall * K,
                         tall, K, n, P.bc, G2 + (size_t)f * tall * tall * n);
      HCHK(hipGetLastError());
    }
    if (f == 0) {
      hipLaunchKernelGGL(factors_kernel, dim3(gnn), dim3(nthr), 0, s, Vt, U, n, P.Vc32, P.VcT32,
                         reinterpret_cast<_Float16*>(P.Vc16),
                         reinterpret_cast<_Float16*>(P.VcT16), P.UcT32);
      hipLaunchKernelGGL(sigma_kernel, dim3((n + 255) / 256), dim3(256), 0, s, P.sc, n, P.sc2);
    } else {
      hipLaunchKernelGGL(factors_kernel, dim3(gnn), dim3(nthr), 0, s, Vt, U, n, P.Vr32, P.VrT32,
                         reinterpret_cast<_Float16*>(P.Vr16),
                         reinterpret_cast<_Float16*>(P.VrT16), P.UrT32);
      hipLaunchKernelGGL(sigma_kernel, dim3((n + 255) / 256), dim3(256), 0, s, P.sr, n, P.sr2);
    }
    HCHK(hipGetLastError());
  }

  // D0[i][j] = sum_p Gc[p][i] Gr[p][j] (p over term pairs): as column-major
  // BLAS, D0^T (n x n) = Gr^T-layout (n x t^2) times Gc^T-layout^T
  if (tall > 0) {
    const double one = 1.0, zero = 0.0;
    const size_t tt = (size_t)tall * tall;
    SCHK(rocblas_dgemm(handle, rocblas_operation_none, rocblas_operation_transpose, n, n,
                       (rocblas_int)tt, &one, G2 + tt * n, n, G2, n, &zero, D64, n));
    hipLaunchKernelGGL(to_f32_kernel, dim3(gnn), dim3(nthr), 0, s, D64, n, P.d0, P.d0t);
    HCHK(hipGetLastError());
  } else {
    HCHK(hipMemsetAsync(P.d0, 0, sizeof(float) * nn, s));
    HCHK(hipMemsetAsync(P.d0t, 0, sizeof(float) * nn, s));
  }

  // FP8 copies with 32-entry block exponents along each row
  {
    const int nb = (n + 31) / 32;
    const unsigned g8 = (unsigned)((n * nb + 255) / 256);
    hipLaunchKernelGGL(quant_rows_e4m3_kernel, dim3(g8), dim3(256), 0, s, P.Vc32, n, P.Vc8,
                       P.Vc8s);
    hipLaunchKernelGGL(quant_rows_e4m3_kernel, dim3(g8), dim3(256), 0, s, P.VcT32, n, P.VcT8,
                       P.VcT8s);
    hipLaunchKernelGGL(quant_rows_e4m3_kernel, dim3(g8), dim3(256), 0, s, P.Vr32, n, P.Vr8,
                       P.Vr8s);
    hipLaunchKernelGGL(quant_rows_e4m3_kernel, dim3(g8), dim3(256), 0, s, P.VrT32, n, P.VrT8,
                       P.VrT8s);
    HCHK(hipGetLastError());
  }

  {
    double v[4];
    HCHK(hipMemcpyAsync(&v[0], P.sc, sizeof(double), hipMemcpyDeviceToHost, s));
    HCHK(hipMemcpyAsync(&v[1], P.sc + n - 1, sizeof(double), hipMemcpyDeviceToHost, s));
    HCHK(hipMemcpyAsync(&v[2], P.sr, sizeof(double), hipMemcpyDeviceToHost, s));
    HCHK(hipMemcpyAsync(&v[3], P.sr + n - 1, sizeof(double), hipMemcpyDeviceToHost, s));
    HCHK(hipStreamSynchronize(s));
    P.sc_max = v[0]; P.sc_min = v[1]; P.sr_max = v[2]; P.sr_min = v[3];
  }

done:
  hipStreamSynchronize(s);
  // the workspace belongs to this plan: leave the handle without it
  rocblas_set_workspace(handle, nullptr, 0);
  return rc;
}


}  // namespace kpcg
