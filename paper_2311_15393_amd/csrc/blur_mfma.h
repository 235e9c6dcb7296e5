// Tile body of the MFMA blur (see blur_mfma.hip for the method), shared by
// the single-problem kernel and the batched tile-table kernel.
#pragma once

#include <type_traits>

#include "blur_core.h"

namespace kpcg {

typedef _Float16 mh8_t __attribute__((ext_vector_type(8)));
typedef float mf4_t __attribute__((ext_vector_type(4)));
typedef _Float16 mh2_t __attribute__((ext_vector_type(2)));

constexpr int MB_TM = 64, MB_TN = 64, MB_NT = 512;   // 2 groups of 4 waves

// NCH = 3 (K = 51 .. 63) pairs tap rows: two full 32-column chunks per row,
// and one MFMA whose k = 32 holds the last 16 columns of two rows (the band
// needs K + 15 - 64 <= 14 of them), so a row pair takes 5 chunk MFMAs
// where unpaired rows take 6.
__host__ __device__ constexpr bool mb_pair(int nch) { return nch == 3; }
// staged input columns: the windows of the full chunks reach column
// 48 + 32 nch (unpaired), the paired remainder column 32 (nch - 1) + 64
__host__ __device__ constexpr int mb_width(int nch) {
  return mb_pair(nch) ? 32 * nch + 32 : MB_TN - 16 + 32 * nch;
}
// Row pitch of the LDS planes.  The A-fragment reads (lane l: 16 bytes at
// row l % 16, column 8 (l / 16)) measured free of bank conflicts on gfx950
// when the pitch is 8 mod 16 dwords, and 2-way conflicted at the other
// multiples of 4 dwords tried.  The unpaired width, 24 + 16 nch dwords, is
// such a pitch; the paired one, 16 nch + 16 dwords, is padded by 8.
__host__ __device__ constexpr int mb_pitch(int nch) {
  return mb_pair(nch) ? mb_width(nch) + 16 : mb_width(nch);
}
// hi and lo planes, then the second wave group's partial accumulators
inline size_t mb_lds_bytes(int nch, int K) {
  return (size_t)2 * (MB_TM + K - 1) * mb_pitch(nch) * sizeof(_Float16) +
         (size_t)4 * 16 * 64 * sizeof(float);
}

// Register staging of a tile whose top-left input is (r0, c0): slot q of
// each thread holds the column pair (c, c + 1) of row r at
// idx = threadIdx.x + q MB_NT, idx = r W2 + c / 2, with boundary indices
// mapped by bc_index_c; entries outside the image (zero boundary) or past
// cvalid read as 0.  Returns the thread's largest |value|.
template <int BCV, int NVP, int W2>
__device__ inline float mb_stage_load_c(const float* __restrict__ src, int n, int r0, int c0,
                                        int rows, int cvalid, float (&v0)[NVP],
                                        float (&v1)[NVP]) {
  float mx = 0.0f;
#pragma unroll
  for (int q = 0; q < NVP; ++q) {
    const int idx = threadIdx.x + q * MB_NT;
    float a0 = 0.0f, a1 = 0.0f;
    if (idx < rows * W2) {
      const int r = idx / W2, c = 2 * (idx - r * W2);
      const int gi = bc_index_c<BCV>(r0 + r, n);
      const int gj = bc_index_c<BCV>(c0 + c, n), gj1 = bc_index_c<BCV>(c0 + c + 1, n);
      if ((unsigned)gi < (unsigned)n) {
        if (c < cvalid && (unsigned)gj < (unsigned)n) a0 = src[(size_t)gi * n + gj];
        if (c + 1 < cvalid && (unsigned)gj1 < (unsigned)n) a1 = src[(size_t)gi * n + gj1];
      }
    }
    v0[q] = a0;
    v1[q] = a1;
    mx = fmaxf(mx, fmaxf(fabsf(a0), fabsf(a1)));
  }
  return mx;
}
// The boundary is uniform over the launch: branch on it once, outside the
// unrolled slots.
template <int NVP, int W2>
__device__ inline float mb_stage_load(const float* __restrict__ src, int n, int r0, int c0,
                                      int rows, int cvalid, int bc, float (&v0)[NVP],
                                      float (&v1)[NVP]) {
  if (bc == KP_BC_ZERO)
    return mb_stage_load_c<KP_BC_ZERO, NVP, W2>(src, n, r0, c0, rows, cvalid, v0, v1);
  if (bc == KP_BC_PERIODIC)
    return mb_stage_load_c<KP_BC_PERIODIC, NVP, W2>(src, n, r0, c0, rows, cvalid, v0, v1);
  return mb_stage_load_c<KP_BC_REFLEXIVE, NVP, W2>(src, n, r0, c0, rows, cvalid, v0, v1);
}

// One 64 x 64 output tile at (i0, j0): src is the n x n FP32 input, bfrag
// the plan's tap-fragment table for this orientation, mb_lds dynamic LDS of
// mb_lds_bytes(NCH, K) bytes; partial_out receives the tile's FP64 epilogue
// sum when Epi::kReduce.  Called by MB_NT threads.
template <int NCH, class Epi>
__device__ inline void blur_mfma_tile(const float* __restrict__ src,
                                      const mh8_t* __restrict__ bfrag, int n, int K, int exq,
                                      int i0, int j0, Epi epi, double* partial_out,
                                      unsigned char* mb_lds, int bc = 0) {
  constexpr int W = mb_width(NCH), PITCH = mb_pitch(NCH), W2 = W / 2;
  constexpr int NU = 4 + 2 * (NCH - 1);       // distinct 16-column window offsets
  constexpr int PF = 2;                       // tap rows of fragments in flight
  // column pairs per thread: the tile is at most (48 + 32 NCH)^2 entries
  constexpr int NVP = ((48 + 32 * NCH) * (48 + 32 * NCH) / 2 + MB_NT - 1) / MB_NT;
  const int h = (K - 1) >> 1;
  const int rows = MB_TM + K - 1;
  const int cvalid = MB_TN + K - 1;
  _Float16* shi = reinterpret_cast<_Float16*>(mb_lds);
  _Float16* slo = shi + rows * PITCH;
  __shared__ float red[MB_NT / 64];

  // stage the tile once through registers (two columns per slot), find its
  // largest |x|, then write the scaled hi / lo planes: the scale 2^ex puts
  // that largest value in [2^13, 2^14)
  float v0[NVP], v1[NVP];
  float mx = mb_stage_load<NVP, W2>(src, n, i0 - h, j0 - h, rows, cvalid, bc, v0, v1);
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
  // (paired: group 0 takes an even number of rows, so only the last row,
  // K - 1, can be left without a partner)
  const int half = mb_pair(NCH) ? ((((K + 1) >> 1) + 1) & ~1) : (K + 1) >> 1;
  const int abeg = grp * half, aend = grp ? K : half;
  mf4_t acc[4];
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) acc[jb] = mf4_t{0.f, 0.f, 0.f, 0.f};

  if constexpr (mb_pair(NCH)) {
    constexpr int F = NCH - 1;             // full 32-column chunks per row
    constexpr int NF = 2 * F;              // their hi / lo fragments
    constexpr int NUF = 2 * F + 2;         // 16-column windows they read
    // a ring of two pair slots: fragments [0, NF) of row a, [NF, 2 NF) of
    // row a + 1, then the hi / lo remainder fragment of the pair
    mh8_t bp[2][2 * NF + 2];
    auto fetch = [&](mh8_t (&dst)[2 * NF + 2], int ap) {
      const int a1 = ap + 1 < K ? ap + 1 : ap;       // (row K - 1 has no partner)
#pragma unroll
      for (int t = 0; t < NF; ++t) dst[t] = bfrag[(ap * NCH * 2 + t) * 64 + lane];
#pragma unroll
      for (int t = 0; t < NF; ++t) dst[NF + t] = bfrag[(a1 * NCH * 2 + t) * 64 + lane];
      dst[2 * NF] = bfrag[(ap * NCH * 2 + NF) * 64 + lane];
      dst[2 * NF + 1] = bfrag[(ap * NCH * 2 + NF + 1) * 64 + lane];
    };
    // the full chunks of tap row a (fragments bfr[0 .. NF))
    auto full_row = [&](const mh8_t* bfr, int a) {
      const int off = (w * 16 + a + m) * PITCH + 8 * g;
      mh8_t ah[NUF], al[NUF];
#pragma unroll
      for (int u = 0; u < NUF; ++u) {
        ah[u] = *reinterpret_cast<const mh8_t*>(shi + off + 16 * u);
        al[u] = *reinterpret_cast<const mh8_t*>(slo + off + 16 * u);
      }
#pragma unroll
      for (int t = 0; t < F; ++t) {
        const mh8_t bh = bfr[2 * t], bl = bfr[2 * t + 1];
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
    };
    // the remainder of rows a and a + 1: lanes g < 2 read row a, g >= 2 row
    // a + 1, each at window columns 32 F + 8 (g mod 2); a row without a
    // partner reads itself twice against zero taps
    auto remainder = [&](const mh8_t* bfr, int a, bool partner) {
      const int r = w * 16 + a + m + (partner && g >= 2 ? 1 : 0);
      const int off = r * PITCH + 32 * F + 8 * (g & 1);
      mh8_t ah[4], al[4];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        ah[jb] = *reinterpret_cast<const mh8_t*>(shi + off + 16 * jb);
        al[jb] = *reinterpret_cast<const mh8_t*>(slo + off + 16 * jb);
      }
      const mh8_t bh = bfr[0], bl = bfr[1];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
        acc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[jb], bh, acc[jb], 0, 0, 0);
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
        acc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[jb], bl, acc[jb], 0, 0, 0);
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
        acc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[jb], bh, acc[jb], 0, 0, 0);
    };
    // rows a, a + 1 from ring slot SL, prefetching the next pair into the
    // other slot (pinned at the head of the step, as in the unpaired loop)
    auto pair = [&](auto slc, int a, auto lonec) {
      constexpr int SL = decltype(slc)::value;
      constexpr bool LONE = decltype(lonec)::value;
      if constexpr (!LONE) fetch(bp[SL ^ 1], a + 2 < aend ? a + 2 : a);
      __builtin_amdgcn_sched_barrier(0);
      full_row(&bp[SL][0], a);
      if constexpr (!LONE) full_row(&bp[SL][NF], a + 1);
      remainder(&bp[SL][2 * NF], a, !LONE);
    };
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    using Two = std::false_type;
    using One = std::true_type;
    fetch(bp[0], abeg);
    int a0 = abeg;
    for (; a0 + 4 <= aend; a0 += 4) {
      pair(S0{}, a0, Two{});
      pair(S1{}, a0 + 2, Two{});
    }
    if (a0 + 2 <= aend) {
      pair(S0{}, a0, Two{});
      if (a0 + 2 < aend) pair(S1{}, a0 + 2, One{});
    } else if (a0 < aend) {
      pair(S0{}, a0, One{});
    }
  } else {
    // tap fragments of rows a .. a + PF in a ring of PF + 1 register slots;
    // slot entries 2t / 2t+1 are the hi / lo fragments of chunk t
    mh8_t bq[PF + 1][2 * NCH];
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int ap = abeg + p < aend ? abeg + p : aend - 1;
#pragma unroll
      for (int t = 0; t < 2 * NCH; ++t) bq[p][t] = bfrag[(ap * NCH * 2 + t) * 64 + lane];
    }
    // tap row a in ring slot SL (= (a - abeg) mod (PF + 1)): prefetch row
    // a + PF into the slot row a - 1 used, read the row-shifted input
    // windows, and issue the MFMAs
    auto row = [&](auto slc, int a) {
      constexpr int SL = decltype(slc)::value;
      const int an = a + PF < aend ? a + PF : aend - 1;
#pragma unroll
      for (int t = 0; t < 2 * NCH; ++t)
        bq[(SL + PF) % (PF + 1)][t] = bfrag[(an * NCH * 2 + t) * 64 + lane];
      // keep the prefetch at the head of its row (the scheduler would sink it
      // below the MFMAs, next to its first use)
      __builtin_amdgcn_sched_barrier(0);
      const int off = (w * 16 + a + m) * PITCH + 8 * g;
      mh8_t ah[NU], al[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        ah[u] = *reinterpret_cast<const mh8_t*>(shi + off + 16 * u);
        al[u] = *reinterpret_cast<const mh8_t*>(slo + off + 16 * u);
      }
#pragma unroll
      for (int t = 0; t < NCH; ++t) {
        const mh8_t bh = bq[SL][2 * t], bl = bq[SL][2 * t + 1];
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
    };
    // whole rounds of PF + 1 rows run without a per-row branch, so the
    // compiler's wait counts keep the prefetched rows in flight (a branch per
    // row made it wait for every outstanding load); then the 0 .. PF rows left
    static_assert(PF == 2, "the unrolled round below holds PF + 1 = 3 rows");
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    using S2 = std::integral_constant<int, 2>;
    int a0 = abeg;
    for (; a0 + PF + 1 <= aend; a0 += PF + 1) {
      row(S0{}, a0);
      row(S1{}, a0 + 1);
      row(S2{}, a0 + 2);
    }
    if (a0 < aend) row(S0{}, a0);
    if (a0 + 1 < aend) row(S1{}, a0 + 1);
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
    if (threadIdx.x == 0) *partial_out = s;
  }
}


// ---------------------------------------------------------------------------
// The same blur on v_mfma_f32_32x32x16_f16: one A fragment covers 32 output
// rows, so a wave reads half the LDS bytes per flop of the 16 x 16 x 32 form.
// For a 32-column output block and tap row a, the Toeplitz chunks are
// T32_{a,t}[k][c] = Q[a][16 t + k - c] (k < 16, c < 32), t < NC = ceil((K +
// 31) / 16); lane l of a fragment holds rows 8 (l / 32) .. + 7 of column
// l % 32 (B), or row l % 32, entries 8 (l / 32) .. + 7 (A); the accumulator
// holds C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in register r.
// Workgroup: 64 x 64 outputs, 8 waves = 2 row halves (32 rows, both 32-column
// blocks) x 4 groups that split the tap rows; the input tile, 64 + K - 1 rows
// of 16 (NC + 2) columns, is staged once as hi / lo FP16 planes (pitch
// 16 (NC + 2) + 8 halves: conflict-free 16-byte reads of 32 rows), and the
// four groups' partial tiles are added in group order over the freed planes.
// Measured at 1024^2, K = 63 it is slower than blur_mfma_tile (about 41 against
// 34 us); the autotuner keeps whichever is faster for the plan.
// ---------------------------------------------------------------------------
typedef float mf16_t __attribute__((ext_vector_type(16)));

__host__ __device__ constexpr int m32_nch(int K) { return (K + 31 + 15) / 16; }
__host__ __device__ constexpr int m32_width(int nc) { return 16 * (nc + 2); }
__host__ __device__ constexpr int m32_pitch(int nc) { return m32_width(nc) + 8; }
inline size_t m32_lds_bytes(int nc, int K) {
  const size_t planes = (size_t)2 * (MB_TM + K - 1) * m32_pitch(nc) * sizeof(_Float16);
  const size_t partials = (size_t)4 * MB_TM * (MB_TN + 1) * sizeof(float);
  return planes > partials ? planes : partials;
}

template <int NC, class Epi>
__device__ inline void blur_mfma32_tile(const float* __restrict__ src,
                                        const mh8_t* __restrict__ bfrag, int n, int K, int exq,
                                        int i0, int j0, Epi epi, double* partial_out,
                                        unsigned char* mb_lds, int bc = 0) {
  constexpr int W = m32_width(NC), PITCH = m32_pitch(NC), W2 = W / 2;
  constexpr int NU = NC + 2;                  // A fragments: 16-column windows
  constexpr int NVP = ((MB_TM + 62) * W2 + MB_NT - 1) / MB_NT;   // K <= 63
  const int h = (K - 1) >> 1;
  const int rows = MB_TM + K - 1;
  const int cvalid = MB_TN + K - 1;
  _Float16* shi = reinterpret_cast<_Float16*>(mb_lds);
  _Float16* slo = shi + rows * PITCH;
  __shared__ float red[MB_NT / 64];

  // stage: as blur_mfma_tile (two columns per slot, tile max, 2^ex scale)
  float v0[NVP], v1[NVP];
  float mx = mb_stage_load<NVP, W2>(src, n, i0 - h, j0 - h, rows, cvalid, bc, v0, v1);
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

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rw = wv & 1, grp = wv >> 1;       // row half, tap-row group
  const int lr = lane & 31, lg = lane >> 5;
  const int quarter = (K + 3) >> 2;
  const int abeg = grp * quarter;
  const int aend = abeg + quarter < K ? abeg + quarter : K;
  mf16_t acc[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[cb][r] = 0.0f;

  // tap fragments of the next row in flight while the current one is used
  mh8_t bq[2][2 * NC];
  if (abeg < aend) {
#pragma unroll
    for (int t = 0; t < 2 * NC; ++t) bq[0][t] = bfrag[(abeg * NC * 2 + t) * 64 + lane];
  }
  for (int a0 = abeg; a0 < aend; a0 += 2) {
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int a = a0 + sl;
      if (a < aend) {
        const int an = a + 1 < aend ? a + 1 : a;
#pragma unroll
        for (int t = 0; t < 2 * NC; ++t) bq[sl ^ 1][t] = bfrag[(an * NC * 2 + t) * 64 + lane];
        const int off = (rw * 32 + a + lr) * PITCH + 8 * lg;
        mh8_t ah[NU], al[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          ah[u] = *reinterpret_cast<const mh8_t*>(shi + off + 16 * u);
          al[u] = *reinterpret_cast<const mh8_t*>(slo + off + 16 * u);
        }
#pragma unroll
        for (int t = 0; t < NC; ++t) {
          const mh8_t bh = bq[sl][2 * t], bl = bq[sl][2 * t + 1];
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[2 * cb + t], bh, acc[cb], 0, 0, 0);
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[2 * cb + t], bl, acc[cb], 0, 0, 0);
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al[2 * cb + t], bh, acc[cb], 0, 0, 0);
        }
      }
    }
  }

  // the four groups' partial tiles over the freed planes, then every thread
  // adds them in group order for its outputs (consecutive threads on
  // consecutive columns) and runs the epilogue
  __syncthreads();
  float* part = reinterpret_cast<float*>(mb_lds);       // [4][64][65]
  constexpr int LD = MB_TN + 1;
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int il = rw * 32 + 8 * (r >> 2) + 4 * lg + (r & 3);
      const int jl = 32 * cb + lr;
      part[((size_t)grp * MB_TM + il) * LD + jl] = acc[cb][r];
    }
  __syncthreads();
  const float oscale = ldexpf(1.0f, -(ex + exq));
  double d = 0.0;
#pragma unroll
  for (int q = 0; q < MB_TM * MB_TN / MB_NT; ++q) {
    const int idx = threadIdx.x + q * MB_NT;
    const int il = idx / MB_TN, jl = idx % MB_TN;
    float tot = part[(size_t)il * LD + jl];
#pragma unroll
    for (int g2 = 1; g2 < 4; ++g2) tot += part[((size_t)g2 * MB_TM + il) * LD + jl];
    const int i = i0 + il, j = j0 + jl;
    if (i < n && j < n) {
      const float val = tot * oscale;
      epi.row(i, j, 1, &val, d);
    }
  }
  if constexpr (Epi::kReduce) {
    __shared__ double sh[MB_NT / 64];
    const double s = block_sum<MB_NT>(d, sh);
    if (threadIdx.x == 0) *partial_out = s;
  }
}

}  // namespace kpcg
