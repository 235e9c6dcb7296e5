// The blur matvecs (A p and A^T q, Section 5.2: the most expensive part of an
// iteration) on FP16 MFMA with a two-term split of both operands.
//
//     out[i][j] = sum_{a,b < K} Q[a][b] in[i + a - h][j + b - h]
//
// For each tap row a, a 16 x 16 block of outputs is a product of the 16 x 32
// input windows (row-shifted by a) with the banded Toeplitz 32 x 16 matrices
// T_{a,t}[k][c] = Q[a][32 t + k - c], t = 0 .. NCH-1, NCH = ceil((K+15)/32);
// T_{a,t} does not depend on where the block sits, so its MFMA fragments are
// built once per plan (mfma_taps_kernel).  The band of one block and tap row
// is 16 + K - 1 columns wide; for NCH = 3 (K = 51 .. 63) its last K - 49
// <= 14 columns are shorter than a chunk, so tap rows go in pairs: each row
// takes NCH - 1 full chunks, and one MFMA takes the last 16 columns of both
// rows (k < 16 from row a, k >= 16 from row a + 1, taps R_a[k][c] = Q[a +
// k div 16][64 + k mod 16 - c]), 5 chunk MFMAs per pair instead of 6.
// v_mfma_f32_16x16x32_f16 takes the
// inputs and taps as hi + lo FP16 pairs (power-of-two scaled: per tile for the
// input, per plan for the taps, so the hi parts sit in [2^13, 2^14)), and the
// three products hi*hi, hi*lo, lo*hi accumulate in FP32.  FP16 x FP16
// products are exact in FP32, so the only extra error over an FP32 direct
// convolution is the dropped lo*lo term (2^-22 relative) and FP16 underflow of
// entries below 2^-27 of their tile's largest.
//
// Workgroup: 64 x 64 outputs, two groups of 4 waves of 16 rows x 64 columns,
// each group taking half of the tap rows (sums added in LDS).  The
// (64+K-1) x mb_width(NCH) input tile is read once from global memory into
// registers, scaled, and written to LDS as hi and lo planes; per tap row a
// wave reads NU = 2 NCH + 2 A-fragment pairs from LDS and 2 NCH tap fragments
// from the L2-resident table (prefetched two rows ahead), and issues 12 NCH
// MFMAs (paired rows: 4 NCH + 4 A-fragment pairs, 4 NCH - 2 tap
// fragments and 24 NCH - 12 MFMAs per pair, the next pair's fragments
// prefetched).
#include "blur_mfma.h"

namespace kpcg {

// tap fragments: entry ((a * nch + t) * 2 + part) * 64 + lane holds the 8
// halves T_{a,t}[8 g + e][c] (c = lane mod 16, g = lane div 16), part 0 = hi,
// 1 = lo of Q * 2^exq
__global__ __launch_bounds__(256) void mfma_taps_kernel(const float* __restrict__ taps, int K,
                                                        int KQ, int nch, int exq,
                                                        mh8_t* __restrict__ out) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= K * nch * 2 * 64) return;
  const int lane = idx & 63;
  int rest = idx >> 6;
  const int part = rest & 1;
  rest >>= 1;
  const int t = rest % nch, a = rest / nch;
  const int c = lane & 15, g = lane >> 4;
  // paired rows (mb_pair): the last chunk of row a is the remainder of rows
  // a (k < 16) and a + 1 (k >= 16), both at window columns 32 t + (k mod 16)
  const bool rem = mb_pair(nch) && t == nch - 1;
  const int arow = rem && g >= 2 ? a + 1 : a;
  const int kk = rem ? 8 * (g & 1) : 8 * g;
  mh8_t v;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int b = 32 * t + kk + e - c;
    const float q = (b >= 0 && b < K && arow < K) ? taps[arow * KQ + b] : 0.0f;
    const float s = ldexpf(q, exq);
    const _Float16 hi = (_Float16)s;
    v[e] = part == 0 ? hi : (_Float16)(s - (float)hi);
  }
  out[idx] = v;
}

// 32 x 32 x 16 tap fragments: entry ((a * nc + t) * 2 + part) * 64 + lane
// holds T32_{a,t}[8 g + e][c] = Q[a][16 t + 8 g + e - c] (c = lane mod 32,
// g = lane div 32), part 0 = hi, 1 = lo of Q * 2^exq
__global__ __launch_bounds__(256) void mfma32_taps_kernel(const float* __restrict__ taps, int K,
                                                          int KQ, int nc, int exq,
                                                          mh8_t* __restrict__ out) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= K * nc * 2 * 64) return;
  const int lane = idx & 63;
  int rest = idx >> 6;
  const int part = rest & 1;
  rest >>= 1;
  const int t = rest % nc, a = rest / nc;
  const int c = lane & 31, g = lane >> 5;
  mh8_t v;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int b = 16 * t + 8 * g + e - c;
    const float q = (b >= 0 && b < K) ? taps[a * KQ + b] : 0.0f;
    const float sc = ldexpf(q, exq);
    const _Float16 hi = (_Float16)sc;
    v[e] = part == 0 ? hi : (_Float16)(sc - (float)hi);
  }
  out[idx] = v;
}

template <int NC, class Epi>
__global__ __launch_bounds__(MB_NT) void blur_mfma32_kernel(const float* __restrict__ src,
                                                            const mh8_t* __restrict__ bfrag,
                                                            int n, int K, int exq, Epi epi,
                                                            Ctrl* ctrl, int skip_if_done,
                                                            double* partials, int bc) {
  extern __shared__ __align__(16) unsigned char mb_lds[];
  if (skip_if_done && ctrl->done != RUNNING) return;
  blur_mfma32_tile<NC, Epi>(src, bfrag, n, K, exq, blockIdx.y * MB_TM, blockIdx.x * MB_TN, epi,
                            partials + Epi::kSlot * MAX_PARTIALS + blockIdx.y * gridDim.x +
                                blockIdx.x,
                            mb_lds, bc);
}

size_t mfma32_taps_count(int K) { return (size_t)K * m32_nch(K) * 2 * 64; }

template <int NCH, class Epi>
__global__ __launch_bounds__(MB_NT) void blur_mfma_kernel(const float* __restrict__ src,
                                                          const mh8_t* __restrict__ bfrag,
                                                          int n, int K, int exq, Epi epi,
                                                          Ctrl* ctrl, int skip_if_done,
                                                          double* partials, int bc) {
  extern __shared__ __align__(16) unsigned char mb_lds[];
  if (skip_if_done && ctrl->done != RUNNING) return;
  blur_mfma_tile<NCH, Epi>(src, bfrag, n, K, exq, blockIdx.y * MB_TM, blockIdx.x * MB_TN, epi,
                           partials + Epi::kSlot * MAX_PARTIALS + blockIdx.y * gridDim.x +
                               blockIdx.x,
                           mb_lds, bc);
}

int mfma_nch(int K) { return (K + 15 + 31) / 32; }

size_t mfma_taps_count(int K) { return (size_t)K * mfma_nch(K) * 2 * 64; }

hipError_t build_mfma_taps(const Plan& P, hipStream_t s) {
  const int K = P.k, nch = mfma_nch(K);
  const size_t cnt = mfma_taps_count(K);
  const unsigned blocks = (unsigned)((cnt + 255) / 256);
  mh8_t* tab = reinterpret_cast<mh8_t*>(P.mfma_taps);
  hipLaunchKernelGGL(mfma_taps_kernel, dim3(blocks), dim3(256), 0, s, P.taps32, K, P.kq, nch,
                     P.mfma_exq, tab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mfma_taps_kernel, dim3(blocks), dim3(256), 0, s, P.taps32_flip, K, P.kq,
                     nch, P.mfma_exq, tab + cnt);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nc = m32_nch(K);
  const size_t cnt32 = mfma32_taps_count(K);
  const unsigned blocks32 = (unsigned)((cnt32 + 255) / 256);
  mh8_t* tab32 = reinterpret_cast<mh8_t*>(P.mfma32_taps);
  hipLaunchKernelGGL(mfma32_taps_kernel, dim3(blocks32), dim3(256), 0, s, P.taps32, K, P.kq, nc,
                     P.mfma_exq, tab32);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mfma32_taps_kernel, dim3(blocks32), dim3(256), 0, s, P.taps32_flip, K,
                     P.kq, nc, P.mfma_exq, tab32 + cnt32);
  return hipGetLastError();
}


template <int NCH, class Epi>
static hipError_t run_mfma(const Plan& P, const float* src, const mh8_t* tab, Epi epi,
                           Ctrl* ctrl, int skip, hipStream_t s) {
  const int n = P.n;
  dim3 grid((n + MB_TN - 1) / MB_TN, (n + MB_TM - 1) / MB_TM);
  if ((long)grid.x * grid.y > MAX_PARTIALS) return hipErrorInvalidValue;
  const size_t lds = mb_lds_bytes(NCH, P.k);
  auto kern = blur_mfma_kernel<NCH, Epi>;
  if (lds > 65536) {
    static size_t granted = 65536;      // once per instantiation, the largest K seen
    if (lds > granted) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      granted = lds;
    }
  }
  hipLaunchKernelGGL(kern, grid, dim3(MB_NT), lds, s, src, tab, n, P.k, P.mfma_exq, epi, ctrl,
                     skip, P.partials, P.bc);
  return hipGetLastError();
}

int mfma_blocks(int n) { return ((n + MB_TN - 1) / MB_TN) * ((n + MB_TM - 1) / MB_TM); }

// transpose: A^T (taps32, table 0), else A (taps32_flip, table 1)
template <class Epi>
hipError_t launch_blur_mfma(const Plan& P, const float* src, bool transpose, Epi epi,
                            Ctrl* ctrl, int skip, hipStream_t s) {
  const mh8_t* tab = reinterpret_cast<const mh8_t*>(P.mfma_taps) +
                     (transpose ? 0 : mfma_taps_count(P.k));
  switch (mfma_nch(P.k)) {
    case 1: return run_mfma<1>(P, src, tab, epi, ctrl, skip, s);
    case 2: return run_mfma<2>(P, src, tab, epi, ctrl, skip, s);
    default: return run_mfma<3>(P, src, tab, epi, ctrl, skip, s);
  }
}

template <int NC, class Epi>
static hipError_t run_mfma32(const Plan& P, const float* src, const mh8_t* tab, Epi epi,
                             Ctrl* ctrl, int skip, hipStream_t s) {
  const int n = P.n;
  dim3 grid((n + MB_TN - 1) / MB_TN, (n + MB_TM - 1) / MB_TM);
  if ((long)grid.x * grid.y > MAX_PARTIALS) return hipErrorInvalidValue;
  const size_t lds = m32_lds_bytes(NC, P.k);
  auto kern = blur_mfma32_kernel<NC, Epi>;
  if (lds > 65536) {
    static size_t granted = 65536;      // once per instantiation, the largest K seen
    if (lds > granted) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      granted = lds;
    }
  }
  hipLaunchKernelGGL(kern, grid, dim3(MB_NT), lds, s, src, tab, n, P.k, P.mfma_exq, epi, ctrl,
                     skip, P.partials, P.bc);
  return hipGetLastError();
}

// transpose: A^T (taps32, table 0), else A (taps32_flip, table 1)
template <class Epi>
hipError_t launch_blur_mfma32(const Plan& P, const float* src, bool transpose, Epi epi,
                              Ctrl* ctrl, int skip, hipStream_t s) {
  const mh8_t* tab = reinterpret_cast<const mh8_t*>(P.mfma32_taps) +
                     (transpose ? 0 : mfma32_taps_count(P.k));
  switch (m32_nch(P.k)) {
    case 2: return run_mfma32<2>(P, src, tab, epi, ctrl, skip, s);
    case 3: return run_mfma32<3>(P, src, tab, epi, ctrl, skip, s);
    case 4: return run_mfma32<4>(P, src, tab, epi, ctrl, skip, s);
    case 5: return run_mfma32<5>(P, src, tab, epi, ctrl, skip, s);
    default: return run_mfma32<6>(P, src, tab, epi, ctrl, skip, s);
  }
}

template hipError_t launch_blur_mfma<EpiStoreF32>(const Plan&, const float*, bool, EpiStoreF32,
                                                  Ctrl*, int, hipStream_t);
template hipError_t launch_blur_mfma<EpiNormalW>(const Plan&, const float*, bool, EpiNormalW,
                                                 Ctrl*, int, hipStream_t);
template hipError_t launch_blur_mfma<EpiAnchorRes>(const Plan&, const float*, bool,
                                                   EpiAnchorRes, Ctrl*, int, hipStream_t);
template hipError_t launch_blur_mfma<EpiRhs>(const Plan&, const float*, bool, EpiRhs, Ctrl*,
                                             int, hipStream_t);
template hipError_t launch_blur_mfma<EpiTrueRes>(const Plan&, const float*, bool, EpiTrueRes,
                                                 Ctrl*, int, hipStream_t);
template hipError_t launch_blur_mfma<EpiResid>(const Plan&, const float*, bool, EpiResid, Ctrl*,
                                               int, hipStream_t);

template hipError_t launch_blur_mfma32<EpiStoreF32>(const Plan&, const float*, bool, EpiStoreF32,
                                                    Ctrl*, int, hipStream_t);
template hipError_t launch_blur_mfma32<EpiNormalW>(const Plan&, const float*, bool, EpiNormalW,
                                                   Ctrl*, int, hipStream_t);
template hipError_t launch_blur_mfma32<EpiAnchorRes>(const Plan&, const float*, bool,
                                                     EpiAnchorRes, Ctrl*, int, hipStream_t);
template hipError_t launch_blur_mfma32<EpiRhs>(const Plan&, const float*, bool, EpiRhs, Ctrl*,
                                               int, hipStream_t);
template hipError_t launch_blur_mfma32<EpiTrueRes>(const Plan&, const float*, bool, EpiTrueRes,
                                                   Ctrl*, int, hipStream_t);
template hipError_t launch_blur_mfma32<EpiResid>(const Plan&, const float*, bool, EpiResid,
                                                 Ctrl*, int, hipStream_t);

}  // namespace kpcg
