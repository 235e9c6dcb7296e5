// The blur matvecs (A p and A^T q, Section 5.2: the most expensive part of an
// iteration) on FP16 MFMA with a two-term split of both operands.
//
//     out[i][j] = sum_{a,b < K} Q[a][b] in[i + a - h][j + b - h]
//
// For each tap row a, a 16 x 16 block of outputs is a product of the 16 x 32
// input windows (row-shifted by a) with the banded Toeplitz 32 x 16 matrices
// T_{a,t}[k][c] = Q[a][32 t + k - c], t = 0 .. NCH-1, NCH = ceil((K+15)/32);
// T_{a,t} does not depend on where the block sits, so its MFMA fragments are
// built once per plan (mfma_taps_kernel).  v_mfma_f32_16x16x32_f16 takes the
// inputs and taps as hi + lo FP16 pairs (power-of-two scaled: per tile for the
// input, per plan for the taps, so the hi parts sit in [2^13, 2^14)), and the
// three products hi*hi, hi*lo, lo*hi accumulate in FP32.  FP16 x FP16
// products are exact in FP32, so the only extra error over an FP32 direct
// convolution is the dropped lo*lo term (2^-22 relative) and FP16 underflow of
// entries below 2^-27 of their tile's largest.
//
// Workgroup: 64 x 64 outputs, two groups of 4 waves of 16 rows x 64 columns,
// each group taking half of the tap rows (sums added in LDS).  The
// (64+K-1) x (48+32 NCH) input tile is read once from global memory into
// registers, scaled, and written to LDS as hi and lo planes; per tap row a
// wave reads NU = 2 NCH + 2 A-fragment pairs from LDS and 2 NCH tap fragments
// from the L2-resident table (prefetched two rows ahead), and issues 12 NCH
// MFMAs.
#include "blur_core.h"

namespace kpcg {

typedef _Float16 mh8_t __attribute__((ext_vector_type(8)));
typedef float mf4_t __attribute__((ext_vector_type(4)));
typedef _Float16 mh2_t __attribute__((ext_vector_type(2)));

constexpr int MB_TM = 64, MB_TN = 64, MB_NT = 512;   // 2 groups of 4 waves

__host__ __device__ constexpr int mb_width(int nch) { return MB_TN - 16 + 32 * nch; }
__host__ __device__ constexpr int mb_pitch(int nch) { return mb_width(nch) + 8; }
// hi and lo planes, then the second wave group's partial accumulators
inline size_t mb_lds_bytes(int nch, int K) {
  return (size_t)2 * (MB_TM + K - 1) * mb_pitch(nch) * sizeof(_Float16) +
         (size_t)4 * 16 * 64 * sizeof(float);
}

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
  mh8_t v;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int b = 32 * t + 8 * g + e - c;
    const float q = (b >= 0 && b < K) ? taps[a * KQ + b] : 0.0f;
    const float s = ldexpf(q, exq);
    const _Float16 hi = (_Float16)s;
    v[e] = part == 0 ? hi : (_Float16)(s - (float)hi);
  }
  out[idx] = v;
}

template <int NCH, class Epi>
__global__ __launch_bounds__(MB_NT) void blur_mfma_kernel(const float* __restrict__ src,
                                                          const mh8_t* __restrict__ bfrag,
                                                          int n, int K, int exq, Epi epi,
                                                          Ctrl* ctrl, int skip_if_done,
                                                          double* partials) {
  extern __shared__ __align__(16) unsigned char mb_lds[];
  if (skip_if_done && ctrl->done != RUNNING) return;
  constexpr int W = mb_width(NCH), PITCH = mb_pitch(NCH), W2 = W / 2;
  constexpr int NU = 4 + 2 * (NCH - 1);       // distinct 16-column window offsets
  constexpr int PF = 2;                       // tap rows of fragments in flight
  // column pairs per thread: the tile is at most (48 + 32 NCH)^2 entries
  constexpr int NVP = ((48 + 32 * NCH) * (48 + 32 * NCH) / 2 + MB_NT - 1) / MB_NT;
  const int h = (K - 1) >> 1;
  const int rows = MB_TM + K - 1;
  const int cvalid = MB_TN + K - 1;
  const int i0 = blockIdx.y * MB_TM, j0 = blockIdx.x * MB_TN;
  _Float16* shi = reinterpret_cast<_Float16*>(mb_lds);
  _Float16* slo = shi + rows * PITCH;
  __shared__ float red[MB_NT / 64];

  // stage the tile once through registers (two columns per slot), find its
  // largest |x|, then write the scaled hi / lo planes: the scale 2^ex puts
  // that largest value in [2^13, 2^14)
  float v0[NVP], v1[NVP];
  float mx = 0.0f;
#pragma unroll
  for (int q = 0; q < NVP; ++q) {
    const int idx = threadIdx.x + q * MB_NT;
    float a0 = 0.0f, a1 = 0.0f;
    if (idx < rows * W2) {
      const int r = idx / W2, c = 2 * (idx - r * W2);
      const int gi = i0 - h + r, gj = j0 - h + c;
      if ((unsigned)gi < (unsigned)n) {
        if (c < cvalid && (unsigned)gj < (unsigned)n) a0 = src[(size_t)gi * n + gj];
        if (c + 1 < cvalid && (unsigned)(gj + 1) < (unsigned)n) a1 = src[(size_t)gi * n + gj + 1];
      }
    }
    v0[q] = a0;
    v1[q] = a1;
    mx = fmaxf(mx, fmaxf(fabsf(a0), fabsf(a1)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = red[0];
#pragma unroll
  for (int i = 1; i < MB_NT / 64; ++i) mx = fmaxf(mx, red[i]);
  const int ex = (mx > 0.0f && mx <= 3.0e38f) ? 13 - ilogbf(mx) : 0;
#pragma unroll
  for (int q = 0; q < NVP; ++q) {
    const int idx = threadIdx.x + q * MB_NT;
    if (idx < rows * W2) {
      const int r = idx / W2, c = 2 * (idx - r * W2);
      const float a0 = ldexpf(v0[q], ex), a1 = ldexpf(v1[q], ex);
      const _Float16 h0 = (_Float16)a0, h1 = (_Float16)a1;
      const mh2_t hh = {h0, h1};
      const mh2_t ll = {(_Float16)(a0 - (float)h0), (_Float16)(a1 - (float)h1)};
      *reinterpret_cast<mh2_t*>(shi + r * PITCH + c) = hh;
      *reinterpret_cast<mh2_t*>(slo + r * PITCH + c) = ll;
    }
  }
  __syncthreads();

  // wave group grp (4 waves, one 16-row strip each) takes tap rows
  // [grp * ceil(K/2), ...); the groups' sums meet in LDS at the end
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int w = wv & 3, grp = wv >> 2;
  const int m = lane & 15, g = lane >> 4;
  const int half = (K + 1) >> 1;
  const int abeg = grp * half, aend = grp ? K : half;
  mf4_t acc[4];
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) acc[jb] = mf4_t{0.f, 0.f, 0.f, 0.f};

  // tap fragments of rows a .. a + PF in a ring of PF + 1 register slots;
  // slot entries 2t / 2t+1 are the hi / lo fragments of chunk t
  mh8_t bq[PF + 1][2 * NCH];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    const int ap = abeg + p < aend ? abeg + p : aend - 1;
#pragma unroll
    for (int t = 0; t < 2 * NCH; ++t) bq[p][t] = bfrag[(ap * NCH * 2 + t) * 64 + lane];
  }
  for (int a0 = abeg; a0 < aend; a0 += PF + 1) {
#pragma unroll
    for (int sl = 0; sl <= PF; ++sl) {
      const int a = a0 + sl;
      if (a < aend) {
        const int an = a + PF < aend ? a + PF : aend - 1;
#pragma unroll
        for (int t = 0; t < 2 * NCH; ++t)
          bq[(sl + PF) % (PF + 1)][t] = bfrag[(an * NCH * 2 + t) * 64 + lane];
        const int off = (w * 16 + a + m) * PITCH + 8 * g;
        mh8_t ah[NU], al[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          ah[u] = *reinterpret_cast<const mh8_t*>(shi + off + 16 * u);
          al[u] = *reinterpret_cast<const mh8_t*>(slo + off + 16 * u);
        }
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
          const mh8_t bh = bq[sl][2 * t], bl = bq[sl][2 * t + 1];
#pragma unroll
          for (int jb = 0; jb < 4; ++jb)
            acc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[jb + 2 * t], bh, acc[jb], 0, 0, 0);
#pragma unroll
          for (int jb = 0; jb < 4; ++jb)
            acc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[jb + 2 * t], bl, acc[jb], 0, 0, 0);
#pragma unroll
          for (int jb = 0; jb < 4; ++jb)
            acc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[jb + 2 * t], bh, acc[jb], 0, 0, 0);
        }
      }
    }
  }

  float* redacc = reinterpret_cast<float*>(slo + rows * PITCH);
  if (grp == 1) {
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) redacc[((w * 4 + jb) * 4 + v) * 64 + lane] = acc[jb][v];
  }
  __syncthreads();
  double d = 0.0;
  if (grp == 0) {
    const float oscale = ldexpf(1.0f, -(ex + exq));
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      const int j = j0 + 16 * jb + m;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + w * 16 + 4 * g + v;
        const float tot = acc[jb][v] + redacc[((w * 4 + jb) * 4 + v) * 64 + lane];
        if (i < n && j < n) {
          const float val = tot * oscale;
          epi.row(i, j, 1, &val, d);
        }
      }
    }
  }
  if constexpr (Epi::kReduce) {
    __shared__ double sh[MB_NT / 64];
    const double s = block_sum<MB_NT>(d, sh);
    if (threadIdx.x == 0)
      partials[Epi::kSlot * MAX_PARTIALS + blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
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
                     skip, P.partials);
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

template hipError_t launch_blur_mfma<EpiStoreF32>(const Plan&, const float*, bool, EpiStoreF32,
                                                  Ctrl*, int, hipStream_t);
template hipError_t launch_blur_mfma<EpiNormalW>(const Plan&, const float*, bool, EpiNormalW,
                                                 Ctrl*, int, hipStream_t);
template hipError_t launch_blur_mfma<EpiAnchorRes>(const Plan&, const float*, bool,
                                                   EpiAnchorRes, Ctrl*, int, hipStream_t);

}  // namespace kpcg
