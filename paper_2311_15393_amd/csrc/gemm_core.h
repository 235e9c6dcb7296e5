// Shared body of the MFMA GEMM kernels of the preconditioner solve
// (single-problem and batched launches): one workgroup computes one 64 x 64
// tile of C = A * Bt^T, both operands K-contiguous, or of C = A * B with B
// read from a row-major FP32 matrix, scaled and rounded while staged.
// 4 waves in 2 x 2, each wave 32 x 32 as 2 x 2 MFMA 16x16 blocks; FP32 uses
// v_mfma_f32_16x16x4_f32, FP16 v_mfma_f32_16x16x32_f16, both accumulating in
// FP32.  Stages are double-buffered in LDS with the next stage's global loads
// in flight during the MFMAs.
#pragma once

#include <type_traits>

#include "common.h"

namespace kpcg {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));



template <typename T> struct MT;
template <> struct MT<float> {
  static constexpr int BK = 32;     // k per LDS stage
  static constexpr int VEC = 4;     // elements per 16-byte load
  static constexpr int PAD = 4;
  static constexpr int KM = 4;      // k per MFMA
};
// FP16 stage rows are padded to 40 dwords: the MFMA operand reads (lane l:
// 16 bytes at row l % 16, column 8 (l / 16)) measured free of LDS bank
// conflicts on gfx950 at row pitches of 8 mod 16 dwords, and 2-way
// conflicted at the other multiples of 4 dwords tried.  (The FP32 stages are
// read 4 bytes per lane and keep the 36-dword pitch, measured faster.)
template <> struct MT<_Float16> {
  static constexpr int BK = 64;
  static constexpr int VEC = 8;
  static constexpr int PAD = 16;
  static constexpr int KM = 32;
};

constexpr int GT = 256;  // threads per GEMM workgroup
constexpr int BM = 64, BN = 64;

template <typename T>
using Tile = T[BM][MT<T>::BK + MT<T>::PAD];

// ---------------------------------------------------------------------------
// operand staging: global -> registers (issued one stage ahead) -> LDS
// (s[row][k], k contiguous).  Each thread moves two 16-byte vectors per
// K-contiguous operand and BK*BN/(4*GT) float4 of an FP32 row-major source.
//
// VK (n % 8 == 0): every 16-byte vector lies wholly inside or wholly outside
// the matrix, so each load is one unconditional vector read of a clamped,
// in-range address and the out-of-range vectors are zeroed only when staged
// into LDS.  No register written by a load is touched before the staging
// step, so the loads of a stage stay in flight together across the MFMAs
// (a bounds branch around each load would make the compiler wait for every
// load as soon as it is issued).  Otherwise every element is read on its own.
// ---------------------------------------------------------------------------
template <typename T, bool VK>
struct KContig {
  static constexpr int BK = MT<T>::BK, VEC = MT<T>::VEC, PER_ROW = BK / VEC;
  static constexpr int NV = BM * BK / VEC / GT;      // = 2
  float4 reg[NV];
  bool in[NV];
  __device__ void load(const T* __restrict__ g, int row0, int k0, int n,
                       int tid = threadIdx.x) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int id = tid + GT * v;
      const int row = id / PER_ROW, kc = (id % PER_ROW) * VEC;
      const int gr = row0 + row, gk = k0 + kc;
      if constexpr (VK) {
        in[v] = gr < n && gk < n;
        const int cr = gr < n ? gr : n - 1, ck = gk < n ? gk : n - VEC;
        reg[v] = *reinterpret_cast<const float4*>(g + (size_t)cr * n + ck);
      } else {
        T tmp[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          tmp[e] = (gr < n && gk + e < n) ? g[(size_t)gr * n + gk + e] : T(0);
        reg[v] = *reinterpret_cast<const float4*>(tmp);
      }
    }
  }
  __device__ void store(Tile<T>& s, int tid = threadIdx.x) const {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int id = tid + GT * v;
      const int row = id / PER_ROW, kc = (id % PER_ROW) * VEC;
      float4 val = reg[v];
      if constexpr (VK)
        if (!in[v]) val = make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<float4*>(&s[row][kc]) = val;
    }
  }
};

// B tile from a row-major FP32 matrix src[k][j] (contraction over its rows):
// scaled and rounded to T, transposed into s[j][k].  Lane j of a wave reads
// column j0 + j of NG groups of 8 consecutive rows (each read of the wave is
// one contiguous 256-byte row segment), and writes each group as one 16-byte
// (T = FP16) or two (T = FP32) vectors along k of s[j][.], so the staging
// stores are vector writes without bank conflicts.
template <typename T, bool VK>
struct FromF32Rows {
  static constexpr int BK = MT<T>::BK;
  static constexpr int KQ = GT / BN;                  // row groups in flight at once (4)
  static constexpr int NG = BK / 8 / KQ;              // groups of 8 rows per thread
  static_assert(NG >= 1 && NG * 8 * KQ == BK, "k tile must split into groups of 8 rows");
  float reg[NG][8];
  bool in[NG];
  __device__ void load(const float* __restrict__ src, int j0, int k0, int n,
                       int tid = threadIdx.x) {
    const int j = tid % BN, kq = tid / BN;
    const int gj = j0 + j;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int gk0 = k0 + (kq + g * KQ) * 8;
      if constexpr (VK) {
        // n % 8 == 0: the 8 rows lie wholly inside or wholly outside
        in[g] = gk0 < n && gj < n;
        const int cj = gj < n ? gj : n - 1, ck = gk0 < n ? gk0 : n - 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) reg[g][e] = src[(size_t)(ck + e) * n + cj];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          reg[g][e] = (gk0 + e < n && gj < n) ? src[(size_t)(gk0 + e) * n + gj] : 0.f;
      }
    }
  }
  __device__ void store(Tile<T>& s, float scale, int tid = threadIdx.x) const {
    const int j = tid % BN, kq = tid / BN;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int kl = (kq + g * KQ) * 8;
      bool ok = true;
      if constexpr (VK) ok = in[g];
      if constexpr (sizeof(T) == 2) {
        half8_t h;
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = ok ? (T)(reg[g][e] * scale) : T(0);
        *reinterpret_cast<half8_t*>(&s[j][kl]) = h;
      } else {
        float4 lo, hi;
        lo.x = ok ? reg[g][0] * scale : 0.f; lo.y = ok ? reg[g][1] * scale : 0.f;
        lo.z = ok ? reg[g][2] * scale : 0.f; lo.w = ok ? reg[g][3] * scale : 0.f;
        hi.x = ok ? reg[g][4] * scale : 0.f; hi.y = ok ? reg[g][5] * scale : 0.f;
        hi.z = ok ? reg[g][6] * scale : 0.f; hi.w = ok ? reg[g][7] * scale : 0.f;
        *reinterpret_cast<float4*>(&s[j][kl]) = lo;
        *reinterpret_cast<float4*>(&s[j][kl + 4]) = hi;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// MFMA over one LDS stage: wave (wm, wn) owns a 32 x 32 block of C
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void mma_stage(const Tile<T>& sA, const Tile<T>& sB, float4_t (&acc)[2][2],
                                 int wm, int wn, int lane) {
  const int r16 = lane & 15, g = lane >> 4;
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int kk = 0; kk < MT<T>::BK; kk += 4) {
      float a[2], b[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) a[mi] = sA[wm * 32 + mi * 16 + r16][kk + g];
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) b[ni] = sB[wn * 32 + ni * 16 + r16][kk + g];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < MT<T>::BK; kk += 32) {
      half8_t a[2], b[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
        a[mi] = *reinterpret_cast<const half8_t*>(&sA[wm * 32 + mi * 16 + r16][kk + g * 8]);
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
        b[ni] = *reinterpret_cast<const half8_t*>(&sB[wn * 32 + ni * 16 + r16][kk + g * 8]);
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] =
              __builtin_amdgcn_mfma_f32_16x16x32_f16(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
  }
}

// ---------------------------------------------------------------------------
// epilogues: apply(i, j, v) for C[i][j] = v.  kColMajor asks the split-K
// kernel to hand consecutive threads consecutive i (for stores along i).
// ---------------------------------------------------------------------------
template <class Epi, class = void>
struct ColMajorEpi : std::false_type {};
template <class Epi>
struct ColMajorEpi<Epi, std::void_t<decltype(Epi::kColMajor)>>
    : std::integral_constant<bool, Epi::kColMajor> {};

template <typename T>
struct GEpiStore {                       // row-major store
  T* C; int n;
  static constexpr bool kReduce = false;
  __device__ void apply(int i, int j, float v, double&, double&) const {
    C[(size_t)i * n + j] = (T)v;
  }
};

template <typename T>
struct GEpiSPrimeT {                     // T2^T[j][i] = S'[i][j] * T[i][j]
  // S' = lam2 / (s_c[i]^2 s_r[j]^2 + lam2), or lam2 / (d0[i][j] + lam2) with
  // the exact KP-basis diagonal d0
  // the exact KP-basis diagonal d0 ([i][j]), or its transpose d0t ([j][i],
  // read along i like the stores)
  T* C; const float* sc2; const float* sr2; float lam2; int n; const float* d0;
  const float* d0t = nullptr;
  static constexpr bool kReduce = false;
  static constexpr bool kColMajor = true;
  __device__ void apply(int i, int j, float v, double&, double&) const {
    const float den = d0t  ? d0t[(size_t)j * n + i] + lam2
                      : d0 ? d0[(size_t)i * n + j] + lam2
                           : fmaf(sc2[i], sr2[j], lam2);
    const float sp = lam2 / den;
    C[(size_t)j * n + i] = (T)(sp * v);
  }
};

template <bool REDUCE>
struct GEpiFinal {                       // z (already scaled) ; r.z ; z.w
  float* z; const float* r; const float* w; int n;
  static constexpr bool kReduce = REDUCE;
  __device__ void apply(int i, int j, float v, double& d0, double& d1) const {
    const size_t o = (size_t)i * n + j;
    const float zv = v;
    z[o] = zv;
    if constexpr (REDUCE) {
      d0 += (double)r[o] * zv;
      d1 += (double)zv * w[o];
    }
  }
};

// ---------------------------------------------------------------------------
// the GEMM kernel: C[n x n] = A[n x n] * Bt^T (or * B from FP32 rows)
// ---------------------------------------------------------------------------
template <typename T, bool B_FROM_F32, class Epi, bool VK>
__device__ inline void gemm_tile_vk(const T* __restrict__ A, const void* __restrict__ Bsrc,
                                    int n, int m0, int n0, Epi epi, float bscale, float oscale,
                                    double* partial_out, int slot_stride, Tile<T>* sA,
                                    Tile<T>* sB) {
  constexpr int BK = MT<T>::BK;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;

  float4_t acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = float4_t{0.f, 0.f, 0.f, 0.f};

  KContig<T, VK> la;
  using BL = typename std::conditional<B_FROM_F32, FromF32Rows<T, VK>, KContig<T, VK>>::type;
  BL lb;
  auto load = [&](int k0) {
    la.load(A, m0, k0, n);
    if constexpr (B_FROM_F32)
      lb.load(reinterpret_cast<const float*>(Bsrc), n0, k0, n);
    else
      lb.load(reinterpret_cast<const T*>(Bsrc), n0, k0, n);
  };
  auto store = [&](int buf) {
    la.store(sA[buf]);
    if constexpr (B_FROM_F32) lb.store(sB[buf], bscale);
    else lb.store(sB[buf]);
  };

  const int nk = (n + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);       // next stage in flight during the MFMAs
    mma_stage<T>(sA[cur], sB[cur], acc, wm, wn, lane);
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  double d0 = 0.0, d1 = 0.0;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
      const int j = n0 + wn * 32 + ni * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = m0 + wm * 32 + mi * 16 + 4 * (lane >> 4) + v;
        if (i < n && j < n) epi.apply(i, j, acc[mi][ni][v] * oscale, d0, d1);
      }
    }
  if constexpr (Epi::kReduce) {
    // block-sum scratch in the stage buffers, free after the k-loop's last
    // barrier: a static array beside them would push four workgroups' LDS
    // just past the 160 KiB of a CU and cost one of them
    double* sh = reinterpret_cast<double*>(&sA[0][0][0]);
    const double s0 = block_sum<GT>(d0, sh);
    const double s1 = block_sum<GT>(d1, sh);
    if (threadIdx.x == 0) {
      partial_out[0] = s0;
      partial_out[slot_stride] = s1;
    }
  }
}

// ---------------------------------------------------------------------------
// the same tile with the contraction split over KS groups of four waves
// (GT * KS threads): group g walks k-tiles [g nk / KS, (g+1) nk / KS) with
// its own double-buffered LDS stages, then groups 1..KS-1 hand their
// accumulators to group 0 through LDS, which adds them in group order and
// runs the epilogue.  KS times the waves of gemm_tile per CU hide the global
// latency of the k-loop; the order of the sums is fixed, so results are
// deterministic.  `lds` is dynamic shared memory of gemm_splitk_lds<T>(KS)
// bytes.
// ---------------------------------------------------------------------------
template <typename T>
constexpr size_t gemm_splitk_lds(int ks) {
  return (size_t)4 * ks * sizeof(Tile<T>);
}
constexpr int RED_LD = BN + 1;           // row pitch of the reduction tiles (floats)

// A fold runs once the first stage's operand loads are in flight and before
// they are staged: it may change the B scale, and returns false when the
// workgroup has nothing to do (the same answer in every thread).  It may use
// the start of the LDS buffer; it ends with a barrier.
struct NoFold {
  __device__ bool operator()(float&, char*) const { return true; }
};

template <typename T, bool B_FROM_F32, class Epi, int KS, bool VK, class Fold = NoFold>
__device__ inline void gemm_tile_splitk_vk(const T* __restrict__ A,
                                           const void* __restrict__ Bsrc, int n, int m0, int n0,
                                           Epi epi, float bscale, float oscale,
                                           double* partial_out, int slot_stride, char* lds,
                                           Fold fold = Fold{}) {
  constexpr int BK = MT<T>::BK;
  static_assert((size_t)KS * BM * RED_LD * sizeof(float) + GT * KS / 64 * sizeof(double) <=
                    gemm_splitk_lds<T>(KS),
                "reduction tiles and the block-sum scratch must fit in the stage buffers");
  static_assert((BM * BN) % (GT * KS) == 0, "outputs must split evenly over the threads");
  Tile<T>* sA = reinterpret_cast<Tile<T>*>(lds);     // [KS][2]
  Tile<T>* sB = sA + 2 * KS;                          // [KS][2]
  const int kg = threadIdx.x / GT, tid = threadIdx.x % GT;
  const int lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;

  float4_t acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = float4_t{0.f, 0.f, 0.f, 0.f};

  KContig<T, VK> la;
  using BL = typename std::conditional<B_FROM_F32, FromF32Rows<T, VK>, KContig<T, VK>>::type;
  BL lb;
  Tile<T>* myA = sA + 2 * kg;
  Tile<T>* myB = sB + 2 * kg;
  auto load = [&](int k0) {
    la.load(A, m0, k0, n, tid);
    if constexpr (B_FROM_F32)
      lb.load(reinterpret_cast<const float*>(Bsrc), n0, k0, n, tid);
    else
      lb.load(reinterpret_cast<const T*>(Bsrc), n0, k0, n, tid);
  };
  auto store = [&](int buf) {
    la.store(myA[buf], tid);
    if constexpr (B_FROM_F32) lb.store(myB[buf], bscale, tid);
    else lb.store(myB[buf], tid);
  };

  const int nk = (n + BK - 1) / BK;
  const int kb = kg * nk / KS, ke = (kg + 1) * nk / KS;
  const int cnt = ke - kb;
  const int steps = (nk + KS - 1) / KS;              // the same barrier count in every group
  if (cnt > 0) load(kb * BK);
  if (!fold(bscale, lds)) return;
  if (cnt > 0) store(0);
  __syncthreads();
  for (int st = 0; st < steps; ++st) {
    const int cur = st & 1;
    const bool more = st + 1 < cnt;
    if (more) load((kb + st + 1) * BK);
    if (st < cnt) mma_stage<T>(myA[cur], myB[cur], acc, wm, wn, lane);
    if (more) store(cur ^ 1);
    __syncthreads();
  }

  // cross-group reduction (the stage buffers are free after the last barrier):
  // every group leaves its 64 x 64 partial tile in LDS, then all GT * KS
  // threads add the KS partials of their outputs in group order and run the
  // epilogue, consecutive threads on consecutive j (or i for kColMajor) so
  // that global accesses coalesce
  float* red = reinterpret_cast<float*>(lds);        // [KS][BM][RED_LD]
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int il = wm * 32 + mi * 16 + 4 * (lane >> 4) + v;
        const int jl = wn * 32 + ni * 16 + (lane & 15);
        red[((size_t)kg * BM + il) * RED_LD + jl] = acc[mi][ni][v];
      }
  __syncthreads();
  double d0 = 0.0, d1 = 0.0;
  constexpr bool kCol = ColMajorEpi<Epi>::value;
#pragma unroll
  for (int q = 0; q < BM * BN / (GT * KS); ++q) {
    const int idx = threadIdx.x + q * GT * KS;
    const int il = kCol ? idx % BM : idx / BN;
    const int jl = kCol ? idx / BM : idx % BN;
    float v = red[(size_t)il * RED_LD + jl];
#pragma unroll
    for (int g = 1; g < KS; ++g) v += red[((size_t)g * BM + il) * RED_LD + jl];
    const int i = m0 + il, j = n0 + jl;
    if (i < n && j < n) epi.apply(i, j, v * oscale, d0, d1);
  }
  if constexpr (Epi::kReduce) {
    // block-sum scratch after the reduction tiles (the stage buffers take
    // all of the LDS a workgroup may have, so it cannot be static)
    double* sh = reinterpret_cast<double*>(lds + (size_t)KS * BM * RED_LD * sizeof(float));
    const double s0 = block_sum<GT * KS>(d0, sh);
    const double s1 = block_sum<GT * KS>(d1, sh);
    if (threadIdx.x == 0) {
      partial_out[0] = s0;
      partial_out[slot_stride] = s1;
    }
  }
}

// the kernels' entry points: the vector-load body when n % 8 == 0 (a uniform
// branch), else the element-wise one
template <typename T, bool B_FROM_F32, class Epi>
__device__ inline void gemm_tile(const T* __restrict__ A, const void* __restrict__ Bsrc,
                                 int n, int m0, int n0, Epi epi, float bscale, float oscale,
                                 double* partial_out, int slot_stride) {
  // one set of stage buffers for both bodies (each declaring its own would
  // double the workgroup's LDS and halve the workgroups per CU)
  __shared__ __align__(16) Tile<T> sA[2];
  __shared__ __align__(16) Tile<T> sB[2];
  if ((n % 8) == 0)
    gemm_tile_vk<T, B_FROM_F32, Epi, true>(A, Bsrc, n, m0, n0, epi, bscale, oscale,
                                           partial_out, slot_stride, sA, sB);
  else
    gemm_tile_vk<T, B_FROM_F32, Epi, false>(A, Bsrc, n, m0, n0, epi, bscale, oscale,
                                            partial_out, slot_stride, sA, sB);
}

template <typename T, bool B_FROM_F32, class Epi, int KS, class Fold = NoFold>
__device__ inline void gemm_tile_splitk(const T* __restrict__ A, const void* __restrict__ Bsrc,
                                        int n, int m0, int n0, Epi epi, float bscale,
                                        float oscale, double* partial_out, int slot_stride,
                                        char* lds, Fold fold = Fold{}) {
  if ((n % 8) == 0)
    gemm_tile_splitk_vk<T, B_FROM_F32, Epi, KS, true, Fold>(A, Bsrc, n, m0, n0, epi, bscale,
                                                            oscale, partial_out, slot_stride,
                                                            lds, fold);
  else
    gemm_tile_splitk_vk<T, B_FROM_F32, Epi, KS, false, Fold>(A, Bsrc, n, m0, n0, epi, bscale,
                                                             oscale, partial_out, slot_stride,
                                                             lds, fold);
}

}  // namespace kpcg
