// FP8 (e4m3) GEMM tile with block scaling, shared by the plan's
// preconditioner chain (gemm_fp8.hip) and the batched form (batch.hip).
//
// Same four-GEMM sandwich as the FP16/FP32 chain (Section 3, eq.
// (PreconSolve)), with every operand stored as OCP e4m3 codes plus one
// power-of-two (E8M0) exponent per 32 consecutive entries along the
// contraction dimension.  gfx950's block-scaled MFMA
// (v_mfma_scale_f32_16x16x128_f8f6f4) applies those exponents in hardware.
// Operand layout of one 16x16x128 step, measured on the device: lane l
// serves row (l mod 16); its 32 codes are k in [16 g, 16 g + 16) and
// [64 + 16 g, 64 + 16 g + 16) with g = l div 16, and its scale operand is the
// exponent of k-block [32 g, 32 g + 32) of that row.  The blocks and the
// lanes' k-ranges do not coincide; only the pairing of A and B k-ranges and
// the block-to-lane map of the scales matter.
//
// Block scaling replaces the single power-of-two residual scale of the FP16
// chain: e4m3 has 3 mantissa bits and a range of 2^-9 .. 448, too narrow for
// one scale per matrix.  GEMM epilogues quantise their FP32 outputs with the
// block exponents the next GEMM needs (a 32-wide wave tile holds whole
// blocks), so no intermediate ever goes through HBM in FP32.
#pragma once
#include "common.h"

namespace kpcg {

typedef int v8i_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int G8T = 256;
constexpr int B8M = 64, B8N = 64, B8K = 128;
constexpr int LD8 = B8K + 16;   // bytes per LDS row (16-byte pad)

// E8M0 exponent (biased by 127) of the smallest power of two 2^e with
// amax * 2^-e <= 448; all-zero blocks get 1 (any exponent works).
__device__ inline int e8m0_of(float amax) {
  if (!(amax > 0.0f)) return 1;
  int e;
  const float m = frexpf(amax / 448.0f, &e);
  if (m == 0.5f) e -= 1;
  e += 127;
  return e < 1 ? 1 : (e > 254 ? 254 : e);
}

// 32 codes of one lane for a block-scaled 16x16x128 step (see the kernel)
__device__ inline v8i_t frag8(const uint8_t* row, int gk) {
  const uint4 lo = *reinterpret_cast<const uint4*>(row + 16 * gk);
  const uint4 hi = *reinterpret_cast<const uint4*>(row + 64 + 16 * gk);
  v8i_t v;
  v[0] = (int)lo.x; v[1] = (int)lo.y; v[2] = (int)lo.z; v[3] = (int)lo.w;
  v[4] = (int)hi.x; v[5] = (int)hi.y; v[6] = (int)hi.z; v[7] = (int)hi.w;
  return v;
}

__device__ inline uint32_t pack4_e4m3(float a, float b, float c, float d) {
  int lo = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, lo, true);
}

__device__ inline uint8_t one_e4m3(float v) {
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xff);
}

// ---------------------------------------------------------------------------
// epilogues (lane holds C[i0 + 4*(lane>>4) + v][j0 + (lane&15)], v = 0..3)
// ---------------------------------------------------------------------------
enum Epi8 : int {
  E8_ROWS = 0,     // store codes row-major, exponents per (row, 32 columns)
  E8_SPRIME_T = 1, // multiply by S', store transposed, exponents per (col, 32 rows)
  E8_FINAL = 2,    // FP32 z with the dots r.z and z.Hp
  E8_FINAL_NR = 3, // FP32 z only
};

struct Gemm8Args {
  const uint8_t* A; const uint8_t* As;      // A codes [n][n], exponents [n][n/32]
  const uint8_t* B; const uint8_t* Bs;      // Bt codes / exponents (unless b_f32)
  const float* Bf32;                        // FP32 row-major source for B (GEMM 1)
  uint8_t* C; uint8_t* Cs;                  // quantised output (E8_ROWS / E8_SPRIME_T)
  float* z; const float* r; const float* w; // final stage
  const float* sc2; const float* sr2; float lam2;
  const float* d0;                          // exact KP-basis diagonal, or nullptr
  int n;
};

// No step folded in (the batched form).
struct NoFold8 {
  __device__ bool operator()() const { return true; }
};

// One 64 x 64 output tile at (m0, n0).  `fold` runs once the first operand
// loads are in flight and before they are staged; it returns false when the
// workgroup has nothing to do (the same answer in every thread).  E8_FINAL
// writes the block's sums of r.z and z.Hp to partial_out[0] and
// partial_out[slot_stride]; E8_FINAL* scale z by ctrl->zscale.
template <bool B_F32, int EPI, class Fold>
__device__ inline void gemm8_tile(const Gemm8Args& g, int m0, int n0, const Ctrl* ctrl,
                                  double* partial_out, int slot_stride, Fold fold) {
  const int n = g.n, nb32 = n / 32;
  __shared__ __align__(16) uint8_t sA[2][B8M][LD8];
  __shared__ __align__(16) uint8_t sB[2][B8N][LD8];
  __shared__ uint8_t sAs[2][B8M][B8K / 32];
  __shared__ uint8_t sBs[2][B8N][B8K / 32];
  __shared__ __align__(16) float sF[B_F32 ? B8N : 1][B_F32 ? (B8K + 4) : 1];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;

  // register staging of one K-stage: 2 x 16 B of A (and of B unless FP32)
  uint4 ra[2], rb[2];
  uint32_t ras = 0, rbs = 0;
  float4 rf[8];

  auto load = [&](int k0) {
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int id = tid + G8T * v;
      const int row = id >> 3, kc = (id & 7) * 16;
      ra[v] = *reinterpret_cast<const uint4*>(g.A + (size_t)(m0 + row) * n + k0 + kc);
      if constexpr (!B_F32)
        rb[v] = *reinterpret_cast<const uint4*>(g.B + (size_t)(n0 + row) * n + k0 + kc);
    }
    if (tid < B8M) ras = *reinterpret_cast<const uint32_t*>(g.As + (size_t)(m0 + tid) * nb32 + k0 / 32);
    if constexpr (!B_F32) {
      if (tid >= 64 && tid < 64 + B8N)
        rbs = *reinterpret_cast<const uint32_t*>(g.Bs + (size_t)(n0 + tid - 64) * nb32 + k0 / 32);
    } else {
      // 128 x 64 floats of the row-major source, rows k0.., columns n0..
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int id = tid + G8T * v;
        const int k = id >> 4, jc = (id & 15) * 4;
        rf[v] = *reinterpret_cast<const float4*>(g.Bf32 + (size_t)(k0 + k) * n + n0 + jc);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int id = tid + G8T * v;
      const int row = id >> 3, kc = (id & 7) * 16;
      *reinterpret_cast<uint4*>(&sA[buf][row][kc]) = ra[v];
      if constexpr (!B_F32) *reinterpret_cast<uint4*>(&sB[buf][row][kc]) = rb[v];
    }
    if (tid < B8M) *reinterpret_cast<uint32_t*>(&sAs[buf][tid][0]) = ras;
    if constexpr (!B_F32) {
      if (tid >= 64 && tid < 64 + B8N) *reinterpret_cast<uint32_t*>(&sBs[buf][tid - 64][0]) = rbs;
    } else {
      // transpose into sF[j][k], then quantise per (j, 32-block of k)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int id = tid + G8T * v;
        const int k = id >> 4, jc = (id & 15) * 4;
        sF[jc + 0][k] = rf[v].x;
        sF[jc + 1][k] = rf[v].y;
        sF[jc + 2][k] = rf[v].z;
        sF[jc + 3][k] = rf[v].w;
      }
      __syncthreads();
      {
        const int j = tid >> 2, blk = tid & 3;         // 64 columns x 4 blocks
        const float* src = &sF[j][blk * 32];
        float amax = 0.0f;
#pragma unroll
        for (int e = 0; e < 32; ++e) amax = fmaxf(amax, fabsf(src[e]));
        const int eb = e8m0_of(amax);
        const float inv = ldexpf(1.0f, 127 - eb);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&sB[buf][j][blk * 32]);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          dst[e] = pack4_e4m3(src[4 * e] * inv, src[4 * e + 1] * inv, src[4 * e + 2] * inv,
                              src[4 * e + 3] * inv);
        sBs[buf][j][blk] = (uint8_t)eb;
      }
    }
  };

  f4_t acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int nk = n / B8K;
  load(0);
  if (!fold()) return;
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * B8K);
    const int r16 = lane & 15, gk = lane >> 4;
    v8i_t a[2], b[2];
    int sa[2], sb[2];
    // operand layout of the block-scaled 16x16x128 step: lane group gk holds
    // k in [16 gk, 16 gk + 16) and [64 + 16 gk, 64 + 16 gk + 16) of the
    // 128-wide chunk, and supplies the exponent of k-block [32 gk, 32 gk + 32)
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const int row = wm * 32 + mi * 16 + r16;
      a[mi] = frag8(&sA[cur][row][0], gk);
      sa[mi] = sAs[cur][row][gk];
    }
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
      const int row = wn * 32 + ni * 16 + r16;
      b[ni] = frag8(&sB[cur][row][0], gk);
      sb[ni] = sBs[cur][row][gk];
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
        acc[mi][ni] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
            a[mi], b[ni], acc[mi][ni], 0, 0, 0, sa[mi], 0, sb[ni]);
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  // ---- epilogue ----
  const int c16 = lane & 15, g4 = lane >> 4;
  if constexpr (EPI == E8_ROWS) {
    // rows i, 32 columns of this wave form one block per row
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float am = fmaxf(fabsf(acc[mi][0][v]), fabsf(acc[mi][1][v]));
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) am = fmaxf(am, __shfl_xor(am, off, 64));
        const int eb = e8m0_of(am);
        const float inv = ldexpf(1.0f, 127 - eb);
        const int i = m0 + wm * 32 + mi * 16 + 4 * g4 + v;
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
          const int j = n0 + wn * 32 + ni * 16 + c16;
          g.C[(size_t)i * n + j] = one_e4m3(acc[mi][ni][v] * inv);
        }
        if (c16 == 0) g.Cs[(size_t)i * nb32 + (n0 + wn * 32) / 32] = (uint8_t)eb;
      }
  } else if constexpr (EPI == E8_SPRIME_T) {
    // T2[i][j] = S'[i][j] T[i][j]; stored as T2^T[j][i]; block = 32 rows i
    float t[2][2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        const int j = n0 + wn * 32 + ni * 16 + c16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = m0 + wm * 32 + mi * 16 + 4 * g4 + v;
          const float den = g.d0 ? g.d0[(size_t)i * n + j] + g.lam2
                                 : fmaf(g.sc2[i], g.sr2[j], g.lam2);
          const float sp = g.lam2 / den;
          t[mi][ni][v] = sp * acc[mi][ni][v];
        }
      }
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
      float am = 0.0f;
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int v = 0; v < 4; ++v) am = fmaxf(am, fabsf(t[mi][ni][v]));
      am = fmaxf(am, __shfl_xor(am, 16, 64));
      am = fmaxf(am, __shfl_xor(am, 32, 64));
      const int eb = e8m0_of(am);
      const float inv = ldexpf(1.0f, 127 - eb);
      const int j = n0 + wn * 32 + ni * 16 + c16;
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) {
        const int i0 = m0 + wm * 32 + mi * 16 + 4 * g4;
        const uint32_t pk = pack4_e4m3(t[mi][ni][0] * inv, t[mi][ni][1] * inv,
                                       t[mi][ni][2] * inv, t[mi][ni][3] * inv);
        *reinterpret_cast<uint32_t*>(&g.C[(size_t)j * n + i0]) = pk;
      }
      if (g4 == 0) g.Cs[(size_t)j * nb32 + (m0 + wm * 32) / 32] = (uint8_t)eb;
    }
  } else {
    const float zs = ctrl->zscale;
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        const int j = n0 + wn * 32 + ni * 16 + c16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = m0 + wm * 32 + mi * 16 + 4 * g4 + v;
          const size_t o = (size_t)i * n + j;
          const float zv = acc[mi][ni][v] * zs;
          g.z[o] = zv;
          if constexpr (EPI == E8_FINAL) {
            d0 += (double)g.r[o] * zv;
            d1 += (double)zv * g.w[o];
          }
        }
      }
    if constexpr (EPI == E8_FINAL) {
      __shared__ double sh[G8T / 64];
      const double s0 = block_sum<G8T>(d0, sh);
      const double s1 = block_sum<G8T>(d1, sh);
      if (threadIdx.x == 0) {
        partial_out[0] = s0;
        partial_out[slot_stride] = s1;
      }
    }
  }
}

}  // namespace kpcg
