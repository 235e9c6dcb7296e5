// Batched solves: many (problem, lambda) items of uneven size in one set of
// launches.
//
// Each phase of the (P)CG iteration is ONE launch over the tiles of every
// item that is still active: a device tile table maps blockIdx.x to (item,
// tile), and a per-item descriptor gives the item's size, PSF taps, KP-SVD
// factors, vectors and control block.  Items converge, break down or hit
// maxit independently (every kernel checks its item's state first).  Items
// are grouped by the blur tile shape the setup-time autotuner chose for
// their plan, so each group's blur launch uses its own shape.  The host
// enqueues a block of iterations once into a hipGraph (on a private stream)
// and replays it, reading back the items' control blocks between replays to
// run the FP64 true-residual recomputations the items ask for.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "blur_core.h"
#include "blur_mfma.h"
#include "gemm_core.h"
#include "gemm_fp8.h"

namespace kpcg {

constexpr int MAXP_ITEM = 1024;   // partial sums per item and slot
constexpr int VCH = 4096;         // floats per vector-kernel block

struct ItemDesc {
  int n, k, kq;
  int nb_blur, nb_blur64, nb_gemm, nb_vec;   // blocks per item of each launch kind
  int ntx_blur, ntx_blur64, ntx_gemm;        // tiles across of each launch kind
  int prec;
  float lam2f;
  double lam2;
  const float *taps32, *taps32_flip;
  const double *taps64, *taps64_flip;
  const _Float16 *VcT16, *Vc16, *Vr16, *VrT16;
  const float *VcT32, *Vc32, *Vr32, *VrT32;
  const uint8_t *VcT8, *Vc8, *Vr8, *VrT8;        // e4m3 codes and their block exponents
  const uint8_t *VcT8s, *Vc8s, *Vr8s, *VrT8s;
  uint8_t *t1s, *t2s, *t3s;                      // block exponents of the FP8 intermediates
  const float *sc2, *sr2;
  const float* d0;                           // exact KP-basis diagonal (KP_EXACT_DIAG) or null
  const float* b;
  float* x;
  float *r, *p, *q, *w, *z;
  double *x64, *y64;                         // FP64 iterate, b - A x scratch
  double *xa64, *ra64;                       // anchor (x_a, r_a) of the true residuals
  void *t1, *t2, *t3;
  Ctrl* ctrl;
  double* partials;                          // [NSLOTS][MAXP_ITEM]
  // fast blur (A p, A^T q, anchored residuals): MFMA if the plan's autotuner
  // chose it, else its fastest VALU shape
  int use_mfma, nch, exq, ntx_mfma, nb_fast;
  const void* mfma_taps;                     // table for taps32, then for taps32_flip
  size_t mfma_count;                         // entries per orientation
  int bc;                                    // the plan's boundary (KP_BC_ZERO / KP_BC_PERIODIC)
  int warm;                                  // x holds the initial guess (KP_WARM)
};

struct TileRef {
  int item;
  int t;                                     // tile index within the item
};

enum RunMode : int { RM_RUNNING = 0, RM_PENDING = 1, RM_ALL = 2, RM_RESUME = 3, RM_FINISHED = 4,
                     RM_PEND_FULL = 5, RM_PEND_ANCH = 6, RM_PEND_FULL_FASTU = 7,
                     RM_PEND_FULL_F64U = 8 };

// batched scalar kind: a true residual whose last blur ran on the fast blur
// (anchored, or A^T (b - A x) on it), partials per fast-blur tile
constexpr int SC_TRUE_FAST = 100;

__device__ inline bool item_active(const Ctrl* c, int mode) {
  const int d = c->done;
  switch (mode) {
    case RM_RUNNING: return d == RUNNING;
    case RM_PENDING: return d == PENDING;
    case RM_PEND_FULL: return d == PENDING && !c->anchor;
    case RM_PEND_ANCH: return d == PENDING && c->anchor;
    case RM_PEND_FULL_FASTU: return d == PENDING && !c->anchor && c->fastu;
    case RM_PEND_FULL_F64U: return d == PENDING && !c->anchor && !c->fastu;
    case RM_RESUME: return d == RUNNING && c->resume;
    case RM_FINISHED: return d == MAXIT || d == BREAKDOWN;
    default: return true;
  }
}

// ---------------------------------------------------------------------------
// batched blur
// ---------------------------------------------------------------------------
// BK_TRUE1: u = b - A x (FP64); BK_TRUE2: r = A^T u - lambda^2 x with A^T in
// FP64, BK_TRUE2F: the same on the fast blur; BK_TRUE1F: u = b - A z on the
// fast blur, z = fp32(x)
enum BlurKind : int { BK_A = 0, BK_AT_NORMAL = 1, BK_RHS = 2, BK_TRUE1 = 3, BK_TRUE2 = 4,
                      BK_MISFIT = 5, BK_ANC1 = 6, BK_ANC2 = 7, BK_TRUE2F = 8, BK_TRUE1F = 9 };

// ||A x - b||^2 for the data-misfit report
struct EpiMisfit {
  const float* b; int n;
  static constexpr bool kReduce = true;
  static constexpr int kSlot = SLOT_NORM;
  template <typename Acc>
  __device__ void row(int i, int j0, int cnt, const Acc* v, double& d) const {
    const size_t o = (size_t)i * n + j0;
    for (int c = 0; c < cnt; ++c) {
      const double e = (double)v[c] - (double)b[o + c];
      d += e * e;
    }
  }
};

template <int TX, int TY, int RX, int RY, int KIND>
__global__ __launch_bounds__(TX* TY) void blur_batched_kernel(const ItemDesc* __restrict__ items,
                                                              const TileRef* __restrict__ tiles,
                                                              int mode) {
  const TileRef tr = tiles[blockIdx.x];
  const ItemDesc& it = items[tr.item];
  if (!item_active(it.ctrl, mode)) return;
  constexpr int TW = TX * RX, TH = TY * RY;
  const int n = it.n;
  if constexpr (KIND == BK_TRUE1 || KIND == BK_TRUE2) {
    const int ty = tr.t / it.ntx_blur64, tx = tr.t - ty * it.ntx_blur64;
    const int ldw = lds_width<TX, TY, RX, RY, double>(it.kq);
    double* out = it.partials + SLOT_TRUE * MAXP_ITEM + tr.t;
    if constexpr (KIND == BK_TRUE1) {
      EpiResid e{it.b, it.q, it.y64, n};
      blur_tile<TX, TY, RX, RY, BC, double, double, double, EpiResid>(
          it.x64, it.taps64_flip, n, it.k, it.kq, ldw, ty * TH, tx * TW, e, out, it.bc);
    } else {
      EpiTrueRes e{it.x64, it.r, it.lam2, n, it.xa64, it.ra64};
      blur_tile<TX, TY, RX, RY, BC, double, double, double, EpiTrueRes>(
          it.y64, it.taps64, n, it.k, it.kq, ldw, ty * TH, tx * TW, e, out, it.bc);
    }
  } else {
    const int ty = tr.t / it.ntx_blur, tx = tr.t - ty * it.ntx_blur;
    const int ldw = lds_width<TX, TY, RX, RY, float>(it.kq);
    if constexpr (KIND == BK_A) {
      EpiStoreF32 e{it.q, n};
      blur_tile<TX, TY, RX, RY, BC, float, float, float, EpiStoreF32>(
          it.p, it.taps32_flip, n, it.k, it.kq, ldw, ty * TH, tx * TW, e, nullptr, it.bc);
    } else if constexpr (KIND == BK_AT_NORMAL) {
      EpiNormalW e{it.p, it.w, it.lam2f, n};
      blur_tile<TX, TY, RX, RY, BC, float, float, float, EpiNormalW>(
          it.q, it.taps32, n, it.k, it.kq, ldw, ty * TH, tx * TW, e,
          it.partials + SLOT_DELTA * MAXP_ITEM + tr.t, it.bc);
    } else if constexpr (KIND == BK_ANC1) {
      EpiStoreF32 e{it.z, n};
      blur_tile<TX, TY, RX, RY, BC, float, float, float, EpiStoreF32>(
          it.q, it.taps32_flip, n, it.k, it.kq, ldw, ty * TH, tx * TW, e, nullptr, it.bc);
    } else if constexpr (KIND == BK_ANC2) {
      EpiAnchorRes e{it.x64, it.xa64, it.ra64, it.r, it.lam2, n};
      blur_tile<TX, TY, RX, RY, BC, float, float, float, EpiAnchorRes>(
          it.z, it.taps32, n, it.k, it.kq, ldw, ty * TH, tx * TW, e,
          it.partials + SLOT_TRUE * MAXP_ITEM + tr.t, it.bc);
    } else if constexpr (KIND == BK_TRUE1F) {
      EpiResid e{it.b, it.q, nullptr, n};
      blur_tile<TX, TY, RX, RY, BC, float, float, float, EpiResid>(
          it.z, it.taps32_flip, n, it.k, it.kq, ldw, ty * TH, tx * TW, e, nullptr, it.bc);
    } else if constexpr (KIND == BK_TRUE2F) {
      EpiTrueRes e{it.x64, it.r, it.lam2, n, it.xa64, it.ra64};
      blur_tile<TX, TY, RX, RY, BC, float, float, float, EpiTrueRes>(
          it.q, it.taps32, n, it.k, it.kq, ldw, ty * TH, tx * TW, e,
          it.partials + SLOT_TRUE * MAXP_ITEM + tr.t, it.bc);
    } else if constexpr (KIND == BK_RHS) {
      EpiRhs e{it.r, n};
      blur_tile<TX, TY, RX, RY, BC, float, float, float, EpiRhs>(
          it.b, it.taps32, n, it.k, it.kq, ldw, ty * TH, tx * TW, e,
          it.partials + SLOT_RHS * MAXP_ITEM + tr.t, it.bc);
    } else {
      EpiMisfit e{it.b, n};
      blur_tile<TX, TY, RX, RY, BC, float, double, double, EpiMisfit>(
          it.x, it.taps64_flip, n, it.k, it.kq, ldw, ty * TH, tx * TW, e,
          it.partials + SLOT_NORM * MAXP_ITEM + tr.t, it.bc);
    }
  }
}

// the MFMA blur over the tile table (items whose plan chose it), 64 x 64 tiles
template <int NCH, int KIND>
__global__ __launch_bounds__(MB_NT) void blur_mfma_batched_kernel(
    const ItemDesc* __restrict__ items, const TileRef* __restrict__ tiles, int mode) {
  extern __shared__ __align__(16) unsigned char mb_lds[];
  const TileRef tr = tiles[blockIdx.x];
  const ItemDesc& it = items[tr.item];
  if (!item_active(it.ctrl, mode)) return;
  const int n = it.n;
  const int ty = tr.t / it.ntx_mfma, tx = tr.t - ty * it.ntx_mfma;
  const mh8_t* tabT = reinterpret_cast<const mh8_t*>(it.mfma_taps);   // A^T
  const mh8_t* tabA = tabT + it.mfma_count;                            // A
  const int i0 = ty * MB_TM, j0 = tx * MB_TN;
  if constexpr (KIND == BK_A) {
    blur_mfma_tile<NCH>(it.p, tabA, n, it.k, it.exq, i0, j0, EpiStoreF32{it.q, n}, nullptr,
                        mb_lds, it.bc);
  } else if constexpr (KIND == BK_AT_NORMAL) {
    blur_mfma_tile<NCH>(it.q, tabT, n, it.k, it.exq, i0, j0,
                        EpiNormalW{it.p, it.w, it.lam2f, n},
                        it.partials + SLOT_DELTA * MAXP_ITEM + tr.t, mb_lds, it.bc);
  } else if constexpr (KIND == BK_ANC1) {
    blur_mfma_tile<NCH>(it.q, tabA, n, it.k, it.exq, i0, j0, EpiStoreF32{it.z, n}, nullptr,
                        mb_lds, it.bc);
  } else if constexpr (KIND == BK_TRUE1F) {
    blur_mfma_tile<NCH>(it.z, tabA, n, it.k, it.exq, i0, j0, EpiResid{it.b, it.q, nullptr, n},
                        nullptr, mb_lds, it.bc);
  } else if constexpr (KIND == BK_TRUE2F) {
    blur_mfma_tile<NCH>(it.q, tabT, n, it.k, it.exq, i0, j0,
                        EpiTrueRes{it.x64, it.r, it.lam2, n, it.xa64, it.ra64},
                        it.partials + SLOT_TRUE * MAXP_ITEM + tr.t, mb_lds, it.bc);
  } else {
    blur_mfma_tile<NCH>(it.z, tabT, n, it.k, it.exq, i0, j0,
                        EpiAnchorRes{it.x64, it.xa64, it.ra64, it.r, it.lam2, n},
                        it.partials + SLOT_TRUE * MAXP_ITEM + tr.t, mb_lds, it.bc);
  }
}

// ---------------------------------------------------------------------------
// batched GEMM stages of the preconditioner solve
// ---------------------------------------------------------------------------
// One GEMM tile of the batch: the 256-thread tile of gemm_core.h (KS = 1)
// or the tile with its contraction split over KS wave groups (dynamic LDS
// `lds`), which hides the k-loop's global latency when the live items leave
// CUs without a tile.
template <typename T, bool BF, class Epi, int KS>
__device__ __forceinline__ void batched_tile(const T* A, const void* B, int n, int m0, int n0,
                                             Epi epi, float bscale, float oscale, double* pout,
                                             char* lds) {
  if constexpr (KS == 1)
    gemm_tile<T, BF, Epi>(A, B, n, m0, n0, epi, bscale, oscale, pout, MAXP_ITEM);
  else
    gemm_tile_splitk<T, BF, Epi, KS>(A, B, n, m0, n0, epi, bscale, oscale, pout, MAXP_ITEM, lds);
}

template <typename T, int STAGE, int KS>
__global__ __launch_bounds__(GT * KS) void gemm_batched_kernel(const ItemDesc* __restrict__ items,
                                                               const TileRef* __restrict__ tiles,
                                                               int mode) {
  extern __shared__ __align__(16) char gk_lds[];      // split-K stages (KS > 1)
  const TileRef tr = tiles[blockIdx.x];
  const ItemDesc& it = items[tr.item];
  if (!item_active(it.ctrl, mode)) return;
  const int n = it.n;
  const int ty = tr.t / it.ntx_gemm, tx = tr.t - ty * it.ntx_gemm;
  const int m0 = ty * BM, n0 = tx * BN;
  T* t1 = reinterpret_cast<T*>(it.t1);
  T* t2 = reinterpret_cast<T*>(it.t2);
  T* t3 = reinterpret_cast<T*>(it.t3);
  const bool f16 = sizeof(T) == 2;
  const T* VcT = f16 ? (const T*)it.VcT16 : (const T*)it.VcT32;
  const T* Vc = f16 ? (const T*)it.Vc16 : (const T*)it.Vc32;
  const T* Vr = f16 ? (const T*)it.Vr16 : (const T*)it.Vr32;
  const T* VrT = f16 ? (const T*)it.VrT16 : (const T*)it.VrT32;
  if constexpr (STAGE == 1) {
    batched_tile<T, true, GEpiStore<T>, KS>(VcT, it.r, n, m0, n0, GEpiStore<T>{t1, n},
                                            it.ctrl->pscale, 1.0f, nullptr, gk_lds);
  } else if constexpr (STAGE == 2) {
    batched_tile<T, false, GEpiSPrimeT<T>, KS>(
        t1, VrT, n, m0, n0, GEpiSPrimeT<T>{t2, it.sc2, it.sr2, it.lam2f, n, it.d0}, 1.0f, 1.0f,
        nullptr, gk_lds);
  } else if constexpr (STAGE == 3) {
    batched_tile<T, false, GEpiStore<T>, KS>(Vc, t2, n, m0, n0, GEpiStore<T>{t3, n}, 1.0f, 1.0f,
                                             nullptr, gk_lds);
  } else {
    batched_tile<T, false, GEpiFinal<true>, KS>(t3, Vr, n, m0, n0,
                                                GEpiFinal<true>{it.z, it.r, it.w, n}, 1.0f,
                                                it.ctrl->zscale,
                                                it.partials + SLOT_RZ * MAXP_ITEM + tr.t, gk_lds);
  }
}

// the same four stages in FP8 (e4m3 codes with E8M0 block exponents, the
// plan's chain of gemm_fp8.hip) over the same 64 x 64 tile table; the FP32
// residual is quantised per block while staged, so no residual scale
template <int STAGE>
__global__ __launch_bounds__(G8T) void gemm8_batched_kernel(const ItemDesc* __restrict__ items,
                                                            const TileRef* __restrict__ tiles,
                                                            int mode) {
  const TileRef tr = tiles[blockIdx.x];
  const ItemDesc& it = items[tr.item];
  if (!item_active(it.ctrl, mode)) return;
  const int ty = tr.t / it.ntx_gemm, tx = tr.t - ty * it.ntx_gemm;
  const int m0 = ty * B8M, n0 = tx * B8N;
  uint8_t* t1 = reinterpret_cast<uint8_t*>(it.t1);
  uint8_t* t2 = reinterpret_cast<uint8_t*>(it.t2);
  uint8_t* t3 = reinterpret_cast<uint8_t*>(it.t3);
  Gemm8Args a{};
  a.n = it.n;
  a.sc2 = it.sc2;
  a.sr2 = it.sr2;
  a.d0 = it.d0;
  a.lam2 = it.lam2f;
  if constexpr (STAGE == 1) {
    a.A = it.VcT8; a.As = it.VcT8s; a.Bf32 = it.r; a.C = t1; a.Cs = it.t1s;
    gemm8_tile<true, E8_ROWS>(a, m0, n0, it.ctrl, nullptr, 0, NoFold8{});
  } else if constexpr (STAGE == 2) {
    a.A = t1; a.As = it.t1s; a.B = it.VrT8; a.Bs = it.VrT8s; a.C = t2; a.Cs = it.t2s;
    gemm8_tile<false, E8_SPRIME_T>(a, m0, n0, it.ctrl, nullptr, 0, NoFold8{});
  } else if constexpr (STAGE == 3) {
    a.A = it.Vc8; a.As = it.Vc8s; a.B = t2; a.Bs = it.t2s; a.C = t3; a.Cs = it.t3s;
    gemm8_tile<false, E8_ROWS>(a, m0, n0, it.ctrl, nullptr, 0, NoFold8{});
  } else {
    a.A = t3; a.As = it.t3s; a.B = it.Vr8; a.Bs = it.Vr8s; a.z = it.z; a.r = it.r; a.w = it.w;
    gemm8_tile<false, E8_FINAL>(a, m0, n0, it.ctrl, it.partials + SLOT_RZ * MAXP_ITEM + tr.t,
                                MAXP_ITEM, NoFold8{});
  }
}

// ---------------------------------------------------------------------------
// batched vector kernels (one block per VCH floats of an item)
// ---------------------------------------------------------------------------
enum VecKind : int { VK_UPDATE = 0, VK_PUPDATE_Z = 1, VK_PUPDATE_R = 2, VK_INIT = 3,
                     VK_TO_F32 = 4, VK_FROM_F32 = 5, VK_DIFF = 6, VK_X_TO_Z = 7 };

template <int KIND>
__global__ __launch_bounds__(256) void vec_batched_kernel(const ItemDesc* __restrict__ items,
                                                          const TileRef* __restrict__ tiles,
                                                          int mode) {
  const TileRef tr = tiles[blockIdx.x];
  const ItemDesc& it = items[tr.item];
  if (!item_active(it.ctrl, mode)) return;
  const int N = it.n * it.n;
  const int e0 = tr.t * VCH, e1 = min(N, e0 + VCH);
  double d = 0.0;
  // the two HBM-bound steps of every iteration move 16 bytes per lane and
  // access (e0 is a multiple of VCH; vectors are 256-byte aligned); an
  // item's last block finishes a ragged n^2 element by element
  const int v0 = e0 >> 2, v1 = e1 >> 2;
  if constexpr (KIND == VK_UPDATE) {
    const double ad = it.ctrl->alpha;
    const float a = (float)ad;
    double2* x2 = reinterpret_cast<double2*>(it.x64);
    float4* r4 = reinterpret_cast<float4*>(it.r);
    const float4* p4 = reinterpret_cast<const float4*>(it.p);
    const float4* w4 = reinterpret_cast<const float4*>(it.w);
    for (int i = v0 + threadIdx.x; i < v1; i += 256) {
      double2 xa = x2[2 * i], xb = x2[2 * i + 1];
      float4 rv = r4[i];
      const float4 pv = p4[i], wv = w4[i];
      xa.x = fma(ad, (double)pv.x, xa.x); xa.y = fma(ad, (double)pv.y, xa.y);
      xb.x = fma(ad, (double)pv.z, xb.x); xb.y = fma(ad, (double)pv.w, xb.y);
      rv.x = fmaf(-a, wv.x, rv.x); rv.y = fmaf(-a, wv.y, rv.y);
      rv.z = fmaf(-a, wv.z, rv.z); rv.w = fmaf(-a, wv.w, rv.w);
      x2[2 * i] = xa;
      x2[2 * i + 1] = xb;
      r4[i] = rv;
      d += (double)rv.x * rv.x + (double)rv.y * rv.y + (double)rv.z * rv.z +
           (double)rv.w * rv.w;
    }
    for (int i = 4 * v1 + threadIdx.x; i < e1; i += 256) {
      it.x64[i] = fma(ad, (double)it.p[i], it.x64[i]);
      const float rv = fmaf(-a, it.w[i], it.r[i]);
      it.r[i] = rv;
      d += (double)rv * rv;
    }
  } else if constexpr (KIND == VK_PUPDATE_Z || KIND == VK_PUPDATE_R) {
    const float bt = (float)it.ctrl->beta;
    const float* z = KIND == VK_PUPDATE_Z ? it.z : it.r;
    float4* p4 = reinterpret_cast<float4*>(it.p);
    const float4* z4 = reinterpret_cast<const float4*>(z);
    for (int i = v0 + threadIdx.x; i < v1; i += 256) {
      float4 pv = p4[i];
      const float4 zv = z4[i];
      pv.x = fmaf(bt, pv.x, zv.x); pv.y = fmaf(bt, pv.y, zv.y);
      pv.z = fmaf(bt, pv.z, zv.z); pv.w = fmaf(bt, pv.w, zv.w);
      p4[i] = pv;
    }
    for (int i = 4 * v1 + threadIdx.x; i < e1; i += 256) it.p[i] = fmaf(bt, it.p[i], z[i]);
  } else if constexpr (KIND == VK_INIT) {
    // x_0 = 0, or the caller's x for a warm start (KP_WARM)
    const bool warm = it.warm != 0;
    for (int i = e0 + threadIdx.x; i < e1; i += 256) {
      it.p[i] = 0.0f;
      it.w[i] = 0.0f;
      it.x64[i] = warm ? (double)it.x[i] : 0.0;
    }
  } else if constexpr (KIND == VK_TO_F32) {
    for (int i = e0 + threadIdx.x; i < e1; i += 256) it.x[i] = (float)it.x64[i];
  } else if constexpr (KIND == VK_DIFF) {         // q = fp32(x - x_a)
    for (int i = e0 + threadIdx.x; i < e1; i += 256) it.q[i] = (float)(it.x64[i] - it.xa64[i]);
  } else if constexpr (KIND == VK_X_TO_Z) {       // z = fp32(x)
    for (int i = e0 + threadIdx.x; i < e1; i += 256) it.z[i] = (float)it.x64[i];
  } else {
    for (int i = e0 + threadIdx.x; i < e1; i += 256) it.x64[i] = (double)it.x[i];
  }
  if constexpr (KIND == VK_UPDATE) {
    __shared__ double sh[4];
    const double s = block_sum<256>(d, sh);
    if (threadIdx.x == 0) it.partials[SLOT_RR * MAXP_ITEM + tr.t] = s;
  }
}

// ---------------------------------------------------------------------------
// batched scalar kernel: one block per item
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void scalar_batched_kernel(const ItemDesc* __restrict__ items,
                                                             const TileRef* __restrict__ list,
                                                             int kind, int mode) {
  const ItemDesc& it = items[list[blockIdx.x].item];
  Ctrl* c = it.ctrl;
  if (!item_active(c, mode)) return;
  __shared__ double sh[4];
  const int done = c->done;
  int slot, nb;
  switch (kind) {
    case SC_ALPHA: slot = SLOT_DELTA; nb = it.nb_fast; break;
    case SC_TRUE_FAST: slot = SLOT_TRUE; nb = it.nb_fast; break;
    case SC_RR: slot = SLOT_RR; nb = it.nb_vec; break;
    case SC_BETA: slot = SLOT_RZ; nb = it.nb_gemm; break;
    case SC_RHS: slot = SLOT_RHS; nb = it.nb_blur; break;
    case SC_NORM: slot = SLOT_NORM; nb = it.nb_blur; break;
    default: slot = SLOT_TRUE; nb = it.nb_blur64; break;
  }
  double s = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    s += it.partials[slot * MAXP_ITEM + i];
    if (kind == SC_BETA) s2 += it.partials[SLOT_ZW * MAXP_ITEM + i];
  }
  const double S = block_sum<256>(s, sh);
  const double S2 = block_sum<256>(s2, sh);
  if (threadIdx.x != 0) return;
  switch (kind) {
    case SC_ALPHA:
      c->delta = S;
      if (!(S > 0.0) || !isfinite(S)) c->done = BREAKDOWN;
      else c->alpha = c->rho / S;
      break;
    case SC_RR:
      c->rr = S;
      c->iter += 1;
      if (c->solver == KP_CG) {
        c->rho_prev = c->rho;
        c->beta = S / c->rho;
        c->rho = S;
      }
      set_scales(c, S);
      if (!isfinite(S)) c->done = BREAKDOWN;
      else if (S <= c->tol2 || S <= c->repl2) c->done = PENDING;
      else if (c->iter >= c->maxit) c->done = MAXIT;
      break;
    case SC_BETA:
      c->rz = S;
      c->zw = S2;
      if (!(S > 0.0) || !isfinite(S) || !isfinite(S2)) {
        c->done = BREAKDOWN;
      } else {
        if (c->first) { c->beta = 0.0; c->first = 0; }
        else if (c->solver == KP_PCG || c->fr_next) c->beta = S / c->rho;
        else c->beta = -S2 / c->delta;
        c->rho = S;
        c->fr_next = 0;
      }
      break;
    case SC_RHS:
      c->gamma0sq = S;
      c->rr = S;
      c->rho = S;
      c->tol2 = c->tol_rel2 * S;
      c->repl2 = REPLACE_DROP * REPLACE_DROP * S;
      set_scales(c, S);
      if (!(S > 0.0) || !isfinite(S)) c->done = S == 0.0 ? CONVERGED : BREAKDOWN;
      break;
    case SC_TRUE:
    case SC_TRUE_FAST:
      c->true_rr = S;
      c->anchor = anchor_eligible(c, S) ? 1 : 0;
      c->rr = S;
      c->repl2 = REPLACE_DROP * REPLACE_DROP * S;
      set_scales(c, S);
      if (c->solver == KP_CG) {
        if (done == PENDING) c->beta = S / c->rho_prev;
        c->rho = S;
      } else {
        c->fr_next = 1;
      }
      if (!isfinite(S)) c->done = BREAKDOWN;
      else if (S <= c->tol2) c->done = CONVERGED;
      else if (c->iter >= c->maxit) c->done = MAXIT;
      else { c->done = RUNNING; c->resume = 1; }
      c->repl += 1;
      break;
    case SC_TRUE_INFO:
      c->true_rr = S;
      break;
    case SC_NORM:
      c->misfit2 = S;
      break;
  }
}

__global__ void clear_resume_kernel(const ItemDesc* __restrict__ items, int nitems) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nitems) items[i].ctrl->resume = 0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Batch {
  int nitems = 0;
  int mode = 0, solver = 0, prec = 0;
  bool fast_tr = false;                      // tol >= TR_FAST_TOL
  std::vector<ItemDesc> h_items;
  ItemDesc* d_items = nullptr;
  // tile tables (device) and their lengths
  struct Group { int cfg; TileRef* tiles; int ntiles; size_t lds; };
  std::vector<Group> blur_groups;            // FP32 blur, one per tile shape (all items)
  // fast blur groups (A, A^T A, anchored residuals): cfg 0..5 VALU shapes
  // of items without MFMA, BLUR_CFG_MFMA + nch for MFMA items
  std::vector<Group> fast_groups;
  TileRef *t_blur64 = nullptr, *t_gemm = nullptr, *t_vec = nullptr;
  int n_blur64 = 0, n_gemm = 0, n_vec = 0;
  TileRef* t_items = nullptr;                // the items in the tables (scalar steps)
  int n_items = 0;
  size_t lds64 = 0;
  // per item: its FP32-blur group (tile shape) and fast group, with their LDS
  std::vector<int> blur_cfg, fast_gid;
  std::vector<size_t> blur_lds, fast_lds;
  TileRef* d_tab = nullptr;                  // device region of the tables
  std::vector<TileRef> h_tab;                // their host staging
  void* mem = nullptr;                       // one allocation for everything
  Ctrl* h_ctrl = nullptr;                    // pinned mirror of the items' Ctrl
  Ctrl* d_ctrl = nullptr;
  hipStream_t s = nullptr;
};

// Kernels needing more than 64 KB of LDS must opt in before their first
// launch (done for every shape before graph capture starts).
template <int TX, int TY, int RX, int RY, int KIND>
static hipError_t ensure_lds(size_t lds) {
  static size_t granted = 65536;
  if (lds <= granted) return hipSuccess;
  auto kern = blur_batched_kernel<TX, TY, RX, RY, KIND>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) granted = lds;
  return e;
}

template <int TX, int TY, int RX, int RY, int KIND>
static hipError_t launch_blur_b(const Batch& B, const TileRef* tiles, int ntiles, size_t lds,
                                int mode) {
  if (ntiles == 0) return hipSuccess;
  hipError_t e = ensure_lds<TX, TY, RX, RY, KIND>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((blur_batched_kernel<TX, TY, RX, RY, KIND>), dim3(ntiles), dim3(TX * TY),
                     lds, B.s, B.d_items, tiles, mode);
  return hipGetLastError();
}

template <int KIND>
static hipError_t ensure_groups(const Batch& B) {
  for (const auto& g : B.blur_groups) {
    hipError_t e;
    switch (g.cfg) {
      case 1: e = ensure_lds<KP_CFG1, KIND>(g.lds); break;
      case 2: e = ensure_lds<KP_CFG2, KIND>(g.lds); break;
      case 3: e = ensure_lds<KP_CFG3, KIND>(g.lds); break;
      case 4: e = ensure_lds<KP_CFG4, KIND>(g.lds); break;
      case 5: e = ensure_lds<KP_CFG5, KIND>(g.lds); break;
      default: e = ensure_lds<KP_CFG0, KIND>(g.lds); break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int KIND>
static hipError_t blur_groups_launch(const Batch& B, int mode) {
  for (const auto& g : B.blur_groups) {
    hipError_t e;
    switch (g.cfg) {
      case 1: e = launch_blur_b<KP_CFG1, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
      case 2: e = launch_blur_b<KP_CFG2, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
      case 3: e = launch_blur_b<KP_CFG3, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
      case 4: e = launch_blur_b<KP_CFG4, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
      case 5: e = launch_blur_b<KP_CFG5, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
      default: e = launch_blur_b<KP_CFG0, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int NCH, int KIND>
static hipError_t ensure_lds_mfma(size_t lds) {
  static size_t granted = 65536;
  if (lds <= granted) return hipSuccess;
  auto kern = blur_mfma_batched_kernel<NCH, KIND>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) granted = lds;
  return e;
}

template <int NCH, int KIND>
static hipError_t launch_mfma_b(const Batch& B, const TileRef* tiles, int ntiles, size_t lds,
                                int mode) {
  if (ntiles == 0) return hipSuccess;
  hipError_t e = ensure_lds_mfma<NCH, KIND>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((blur_mfma_batched_kernel<NCH, KIND>), dim3(ntiles), dim3(MB_NT), lds, B.s,
                     B.d_items, tiles, mode);
  return hipGetLastError();
}

// A p, A^T q (+ lambda^2 p, delta) and the anchored residual's two blurs, on
// each item's fast blur
template <int KIND>
static hipError_t fast_launch(const Batch& B, int mode) {
  for (const auto& g : B.fast_groups) {
    hipError_t e;
    if (g.cfg >= BLUR_CFG_MFMA) {
      switch (g.cfg - BLUR_CFG_MFMA) {
        case 1: e = launch_mfma_b<1, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
        case 2: e = launch_mfma_b<2, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
        default: e = launch_mfma_b<3, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
      }
    } else {
      switch (g.cfg) {
        case 1: e = launch_blur_b<KP_CFG1, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
        case 2: e = launch_blur_b<KP_CFG2, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
        case 3: e = launch_blur_b<KP_CFG3, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
        case 4: e = launch_blur_b<KP_CFG4, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
        case 5: e = launch_blur_b<KP_CFG5, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
        default: e = launch_blur_b<KP_CFG0, KIND>(B, g.tiles, g.ntiles, g.lds, mode); break;
      }
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// LDS opt-in of every fast-group kernel, before graph capture
template <int KIND>
static hipError_t ensure_fast(const Batch& B) {
  for (const auto& g : B.fast_groups) {
    hipError_t e;
    if (g.cfg >= BLUR_CFG_MFMA) {
      switch (g.cfg - BLUR_CFG_MFMA) {
        case 1: e = ensure_lds_mfma<1, KIND>(g.lds); break;
        case 2: e = ensure_lds_mfma<2, KIND>(g.lds); break;
        default: e = ensure_lds_mfma<3, KIND>(g.lds); break;
      }
    } else {
      switch (g.cfg) {
        case 1: e = ensure_lds<KP_CFG1, KIND>(g.lds); break;
        case 2: e = ensure_lds<KP_CFG2, KIND>(g.lds); break;
        case 3: e = ensure_lds<KP_CFG3, KIND>(g.lds); break;
        case 4: e = ensure_lds<KP_CFG4, KIND>(g.lds); break;
        case 5: e = ensure_lds<KP_CFG5, KIND>(g.lds); break;
        default: e = ensure_lds<KP_CFG0, KIND>(g.lds); break;
      }
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int KIND>
static hipError_t vec_launch(const Batch& B, int mode) {
  if (B.n_vec == 0) return hipSuccess;
  hipLaunchKernelGGL(vec_batched_kernel<KIND>, dim3(B.n_vec), dim3(256), 0, B.s, B.d_items,
                     B.t_vec, mode);
  return hipGetLastError();
}

static hipError_t scalar_launch(const Batch& B, int kind, int mode) {
  if (B.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(scalar_batched_kernel, dim3(B.n_items), dim3(256), 0, B.s, B.d_items,
                     B.t_items, kind, mode);
  return hipGetLastError();
}

// Split-K tiles (two wave groups, 80 KiB of LDS: two workgroups per CU)
// once the live items have at most two GEMM tiles per CU; below that a
// 256-thread tile alone on its CU waits on its k-loop's global latency.
constexpr int BATCH_KS = 2;
constexpr int BATCH_SPLITK_TILES = 512;

template <typename T, int KS>
static hipError_t precond_stages_b(const Batch& B, int mode) {
  hipError_t e;
  const size_t lds = KS > 1 ? gemm_splitk_lds<T>(KS) : 0;
  hipLaunchKernelGGL((gemm_batched_kernel<T, 1, KS>), dim3(B.n_gemm), dim3(GT * KS), lds, B.s,
                     B.d_items, B.t_gemm, mode);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((gemm_batched_kernel<T, 2, KS>), dim3(B.n_gemm), dim3(GT * KS), lds, B.s,
                     B.d_items, B.t_gemm, mode);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((gemm_batched_kernel<T, 3, KS>), dim3(B.n_gemm), dim3(GT * KS), lds, B.s,
                     B.d_items, B.t_gemm, mode);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((gemm_batched_kernel<T, 4, KS>), dim3(B.n_gemm), dim3(GT * KS), lds, B.s,
                     B.d_items, B.t_gemm, mode);
  return hipGetLastError();
}

// LDS opt-in of the split-K stages, before graph capture
template <typename T>
static hipError_t ensure_splitk_b() {
  static bool granted = false;
  if (granted) return hipSuccess;
  const int lds = (int)gemm_splitk_lds<T>(BATCH_KS);
  const void* k[4] = {reinterpret_cast<const void*>(gemm_batched_kernel<T, 1, BATCH_KS>),
                      reinterpret_cast<const void*>(gemm_batched_kernel<T, 2, BATCH_KS>),
                      reinterpret_cast<const void*>(gemm_batched_kernel<T, 3, BATCH_KS>),
                      reinterpret_cast<const void*>(gemm_batched_kernel<T, 4, BATCH_KS>)};
  for (const void* f : k) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  granted = true;
  return hipSuccess;
}

template <typename T>
static hipError_t precond_b(const Batch& B, int mode) {
  if (B.n_gemm <= BATCH_SPLITK_TILES) return precond_stages_b<T, BATCH_KS>(B, mode);
  return precond_stages_b<T, 1>(B, mode);
}

// z = M^{-1} r, r.z, beta, p = z + beta p (or the CG direction update)
static hipError_t precond8_b(const Batch& B, int mode) {
  hipLaunchKernelGGL(gemm8_batched_kernel<1>, dim3(B.n_gemm), dim3(G8T), 0, B.s, B.d_items,
                     B.t_gemm, mode);
  hipLaunchKernelGGL(gemm8_batched_kernel<2>, dim3(B.n_gemm), dim3(G8T), 0, B.s, B.d_items,
                     B.t_gemm, mode);
  hipLaunchKernelGGL(gemm8_batched_kernel<3>, dim3(B.n_gemm), dim3(G8T), 0, B.s, B.d_items,
                     B.t_gemm, mode);
  hipLaunchKernelGGL(gemm8_batched_kernel<4>, dim3(B.n_gemm), dim3(G8T), 0, B.s, B.d_items,
                     B.t_gemm, mode);
  return hipGetLastError();
}

static hipError_t tail_b(const Batch& B, int mode) {
  hipError_t e;
  if (B.solver == KP_CG) return vec_launch<VK_PUPDATE_R>(B, mode);
  e = B.prec == KP_P16  ? precond_b<_Float16>(B, mode)
      : B.prec == KP_P8 ? precond8_b(B, mode)
                        : precond_b<float>(B, mode);
  if (e != hipSuccess) return e;
  if ((e = scalar_launch(B, SC_BETA, mode)) != hipSuccess) return e;
  return vec_launch<VK_PUPDATE_Z>(B, mode);
}

static hipError_t iteration_b(const Batch& B) {
  hipError_t e;
  if ((e = fast_launch<BK_A>(B, RM_RUNNING)) != hipSuccess) return e;
  if ((e = fast_launch<BK_AT_NORMAL>(B, RM_RUNNING)) != hipSuccess) return e;
  if ((e = scalar_launch(B, SC_ALPHA, RM_RUNNING)) != hipSuccess) return e;
  if ((e = vec_launch<VK_UPDATE>(B, RM_RUNNING)) != hipSuccess) return e;
  if ((e = scalar_launch(B, SC_RR, RM_RUNNING)) != hipSuccess) return e;
  return tail_b(B, RM_RUNNING);
}

template <int KIND>
static hipError_t blur64_b(const Batch& B, int mode) {
  if (B.n_blur64 == 0) return hipSuccess;
  auto k = blur_batched_kernel<KP_F64IN_CFG, KIND>;
  if (B.lds64 > 65536) {
    static size_t granted = 65536;       // once per instantiation
    if (B.lds64 > granted) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)B.lds64);
      if (e != hipSuccess) return e;
      granted = B.lds64;
    }
  }
  hipLaunchKernelGGL(k, dim3(B.n_blur64), dim3(512), B.lds64, B.s, B.d_items, B.t_blur64, mode);
  return hipGetLastError();
}

// r = A^T (b - A x) - lambda^2 x, both blurs with FP64 accumulation
static hipError_t true_residual_b(const Batch& B, int mode, int kind) {
  hipError_t e;
  if ((e = blur64_b<BK_TRUE1>(B, mode)) != hipSuccess) return e;
  if ((e = blur64_b<BK_TRUE2>(B, mode)) != hipSuccess) return e;
  return scalar_launch(B, kind, mode);
}

// true residuals of the items that asked for one: A^T (b - A x) - lambda^2 x
// for items without a usable anchor (u = b - A x on the item's fast blur or
// in FP64 as its tolerance allows, A^T of it on the fast blur when the
// tolerance allows, else in FP64), r_a - H (x - x_a) on the fast blur for
// the others
static hipError_t pending_residuals_b(const Batch& B) {
  hipError_t e;
  if (B.fast_tr) {
    if ((e = vec_launch<VK_X_TO_Z>(B, RM_PEND_FULL_FASTU)) != hipSuccess) return e;
    if ((e = fast_launch<BK_TRUE1F>(B, RM_PEND_FULL_FASTU)) != hipSuccess) return e;
    if ((e = blur64_b<BK_TRUE1>(B, RM_PEND_FULL_F64U)) != hipSuccess) return e;
    if ((e = fast_launch<BK_TRUE2F>(B, RM_PEND_FULL)) != hipSuccess) return e;
  } else {
    if ((e = true_residual_b(B, RM_PEND_FULL, SC_TRUE)) != hipSuccess) return e;
  }
  if ((e = vec_launch<VK_DIFF>(B, RM_PEND_ANCH)) != hipSuccess) return e;
  if ((e = fast_launch<BK_ANC1>(B, RM_PEND_ANCH)) != hipSuccess) return e;
  if ((e = fast_launch<BK_ANC2>(B, RM_PEND_ANCH)) != hipSuccess) return e;
  // one scalar step for every pending item whose partials are per fast tile
  return scalar_launch(B, SC_TRUE_FAST, B.fast_tr ? RM_PENDING : RM_PEND_ANCH);
}

static int read_ctrls(Batch& B) {
  if (hipMemcpyAsync(B.h_ctrl, B.d_ctrl, sizeof(Ctrl) * B.nitems, hipMemcpyDeviceToHost, B.s) !=
          hipSuccess ||
      hipStreamSynchronize(B.s) != hipSuccess)
    return KP_ERR_HIP;
  return KP_OK;
}

// The tile tables of the items with live[i] set, in a fixed order (FP32
// blur groups by tile shape, fast groups, FP64 blur, GEMM, vector, the item
// list), copied to the device region on the batch stream.  The host staging
// is reused only after a synchronisation of that stream (read_ctrls).
static hipError_t build_tables(Batch& B, const std::vector<char>& live) {
  const int ng = NUM_BLUR_CFG + 3;
  B.h_tab.clear();
  B.blur_groups.clear();
  B.fast_groups.clear();
  size_t cur = 0;
  auto add_group = [&](std::vector<Batch::Group>& out, int gid, int which) {
    const size_t start = cur;
    size_t lds = 0;
    for (int i = 0; i < B.nitems; ++i) {
      if (!live[i]) continue;
      const ItemDesc& d = B.h_items[i];
      const bool in = which == 0 ? B.blur_cfg[i] == gid : B.fast_gid[i] == gid;
      if (!in) continue;
      const int cnt = which == 0 ? d.nb_blur : d.nb_fast;
      for (int t = 0; t < cnt; ++t) B.h_tab.push_back(TileRef{i, t});
      cur += cnt;
      const size_t l = which == 0 ? B.blur_lds[i] : B.fast_lds[i];
      lds = lds > l ? lds : l;
    }
    if (cur > start) {
      const int cfg = which == 0 || gid < NUM_BLUR_CFG ? gid
                                                       : BLUR_CFG_MFMA + (gid - NUM_BLUR_CFG + 1);
      out.push_back(Batch::Group{cfg, B.d_tab + start, (int)(cur - start), lds});
    }
  };
  for (int c = 0; c < NUM_BLUR_CFG; ++c) add_group(B.blur_groups, c, 0);
  for (int c = 0; c < ng; ++c) add_group(B.fast_groups, c, 1);
  auto add_plain = [&](TileRef*& ptr, int& count, int ItemDesc::*nb) {
    const size_t start = cur;
    for (int i = 0; i < B.nitems; ++i) {
      if (!live[i]) continue;
      const int cnt = B.h_items[i].*nb;
      for (int t = 0; t < cnt; ++t) B.h_tab.push_back(TileRef{i, t});
      cur += cnt;
    }
    ptr = B.d_tab + start;
    count = (int)(cur - start);
  };
  add_plain(B.t_blur64, B.n_blur64, &ItemDesc::nb_blur64);
  add_plain(B.t_gemm, B.n_gemm, &ItemDesc::nb_gemm);
  add_plain(B.t_vec, B.n_vec, &ItemDesc::nb_vec);
  const size_t start = cur;
  for (int i = 0; i < B.nitems; ++i)
    if (live[i]) B.h_tab.push_back(TileRef{i, 0});
  cur = B.h_tab.size();
  B.t_items = B.d_tab + start;
  B.n_items = (int)(cur - start);
  if (B.h_tab.empty()) return hipSuccess;
  return hipMemcpyAsync(B.d_tab, B.h_tab.data(), sizeof(TileRef) * B.h_tab.size(),
                        hipMemcpyHostToDevice, B.s);
}

// The batch's device memory is the caller's workspace and its stream the
// device's AUX_BATCH stream: neither is released here.
static void destroy_batch(Batch& B) {
  if (B.s) hipStreamSynchronize(B.s);
  if (B.h_ctrl) hipHostFree(B.h_ctrl);
  B.mem = nullptr;
  B.h_ctrl = nullptr;
  B.s = nullptr;
}

// one batched solve at a time per process: they share the AUX_BATCH streams
static std::mutex g_batch_mu;

int batched_solve(Plan* const* plans, const int* plan_of_item, int nitems, int mode,
                  double tol, int maxit, const float* const* b, const double* lambdas,
                  float* const* x, kp_info_t* infos, void* ws, size_t ws_bytes,
                  size_t* need_out, hipStream_t user_stream) {
  Batch B;
  B.nitems = nitems;
  B.mode = mode;
  B.solver = mode & KP_SOLVER_MASK;
  B.prec = mode & KP_PREC_MASK;
  B.fast_tr = tol >= TR_FAST_TOL;
  const bool eager = (mode & KP_BATCH_EAGER) != 0;

  // ---- sizes of the batch allocation
  size_t total = 0;
  auto align = [](size_t v) { return (v + 255) / 256 * 256; };
  std::vector<size_t> off_item(nitems);
  for (int i = 0; i < nitems; ++i) {
    const size_t nn = (size_t)plans[plan_of_item[i]]->n * plans[plan_of_item[i]]->n;
    off_item[i] = total;
    total += align(nn * 4) * 5;              // r p q w z
    total += align(nn * 8) * 4;              // x64 y64 xa64 ra64
    total += align(nn * 4) * 3;              // t1 t2 t3
    total += align((nn + 31) / 32) * 3;      // their FP8 block exponents
    total += align(sizeof(double) * NSLOTS * MAXP_ITEM);
  }
  const size_t off_ctrl = total;
  total += align(sizeof(Ctrl) * nitems);
  const size_t off_desc = total;
  total += align(sizeof(ItemDesc) * nitems);

  // ---- per-item tile counts and groups (the tables are built by build_tables):
  // FP32 blur groups by VALU tile shape 0..5; fast groups: VALU shapes 0..5,
  // then MFMA with nch = 1, 2, 3 (group 6 + nch - 1)
  size_t ntab = 0;
  B.h_items.resize(nitems);
  B.blur_cfg.assign(nitems, 0);
  B.fast_gid.assign(nitems, 0);
  B.blur_lds.assign(nitems, 0);
  B.fast_lds.assign(nitems, 0);
  for (int i = 0; i < nitems; ++i) {
    const Plan& P = *plans[plan_of_item[i]];
    ItemDesc& d = B.h_items[i];
    std::memset(&d, 0, sizeof(d));
    const int n = P.n, cfg = P.blur_cfg_valu;
    d.n = n; d.k = P.k; d.kq = P.kq; d.prec = B.prec;
    int tw, th;
    size_t lds;
    switch (cfg) {
      case 1: tw = 64; th = 16; lds = (size_t)(16 + P.k - 1) * lds_width<KP_CFG1, float>(P.kq) * 4; break;
      case 2: tw = 64; th = 64; lds = (size_t)(64 + P.k - 1) * lds_width<KP_CFG2, float>(P.kq) * 4; break;
      case 3: tw = 128; th = 16; lds = (size_t)(16 + P.k - 1) * lds_width<KP_CFG3, float>(P.kq) * 4; break;
      case 4: tw = 64; th = 64; lds = (size_t)(64 + P.k - 1) * lds_width<KP_CFG4, float>(P.kq) * 4; break;
      case 5: tw = 64; th = 32; lds = (size_t)(32 + P.k - 1) * lds_width<KP_CFG5, float>(P.kq) * 4; break;
      default: tw = 64; th = 32; lds = (size_t)(32 + P.k - 1) * lds_width<KP_CFG0, float>(P.kq) * 4; break;
    }
    d.ntx_blur = (n + tw - 1) / tw;
    d.nb_blur = d.ntx_blur * ((n + th - 1) / th);
    B.blur_cfg[i] = cfg;
    B.blur_lds[i] = lds;
    d.use_mfma = blur_cfg_is_mfma(P.blur_cfg) ? 1 : 0;     // (16 x 16 x 32 form)
    d.nch = mfma_nch(P.k);
    d.exq = P.mfma_exq;
    d.mfma_taps = P.mfma_taps;
    d.mfma_count = mfma_taps_count(P.k);
    d.bc = P.bc;
    d.ntx_mfma = (n + MB_TN - 1) / MB_TN;
    if (d.use_mfma) {
      d.nb_fast = d.ntx_mfma * ((n + MB_TM - 1) / MB_TM);
      B.fast_gid[i] = NUM_BLUR_CFG + d.nch - 1;
      B.fast_lds[i] = mb_lds_bytes(d.nch, P.k);
    } else {
      d.nb_fast = d.nb_blur;
      B.fast_gid[i] = cfg;
      B.fast_lds[i] = lds;
    }
    d.ntx_blur64 = (n + 63) / 64;
    d.nb_blur64 = d.ntx_blur64 * d.ntx_blur64;
    const size_t l64 = (size_t)(64 + P.k - 1) * lds_width<KP_F64IN_CFG, double>(P.kq) * 8;
    B.lds64 = B.lds64 > l64 ? B.lds64 : l64;
    d.ntx_gemm = (n + BN - 1) / BN;
    d.nb_gemm = d.ntx_gemm * ((n + BM - 1) / BM);
    d.nb_vec = (n * n + VCH - 1) / VCH;
    // the FP8 chain takes whole 128-wide contraction steps (as a plan's does)
    static_assert(BM == B8M && BN == B8N, "the FP8 stages share the GEMM tile table");
    if (B.prec == KP_P8 && !fp8_supported_size(n)) return KP_ERR_UNSUPPORTED;
    ntab += (size_t)d.nb_blur + d.nb_fast + d.nb_blur64 + d.nb_gemm + d.nb_vec + 1;
    if (d.nb_blur > MAXP_ITEM || d.nb_blur64 > MAXP_ITEM || d.nb_gemm > MAXP_ITEM ||
        d.nb_vec > MAXP_ITEM || d.nb_fast > MAXP_ITEM)
      return KP_ERR_UNSUPPORTED;
  }
  const size_t off_tab = total;
  total += align(sizeof(TileRef) * ntab);

  if (need_out) {
    *need_out = total;
    if (!ws) return KP_OK;
  }
  if (!ws || ws_bytes < total) return KP_ERR_WORKSPACE;
  std::lock_guard<std::mutex> lk(g_batch_mu);
  B.s = aux_stream(AUX_BATCH);
  if (!B.s) return KP_ERR_HIP;
  B.mem = ws;
  if (hipHostMalloc(reinterpret_cast<void**>(&B.h_ctrl), sizeof(Ctrl) * nitems) != hipSuccess) {
    destroy_batch(B);
    return KP_ERR_HIP;
  }
  char* base = reinterpret_cast<char*>(B.mem);
  B.d_ctrl = reinterpret_cast<Ctrl*>(base + off_ctrl);
  B.d_items = reinterpret_cast<ItemDesc*>(base + off_desc);

  for (int i = 0; i < nitems; ++i) {
    const Plan& P = *plans[plan_of_item[i]];
    ItemDesc& d = B.h_items[i];
    const size_t nn = (size_t)P.n * P.n;
    char* p = base + off_item[i];
    auto take = [&](size_t bytes) { char* q = p; p += align(bytes); return q; };
    d.r = (float*)take(nn * 4); d.p = (float*)take(nn * 4); d.q = (float*)take(nn * 4);
    d.w = (float*)take(nn * 4); d.z = (float*)take(nn * 4);
    d.x64 = (double*)take(nn * 8); d.y64 = (double*)take(nn * 8);
    d.xa64 = (double*)take(nn * 8); d.ra64 = (double*)take(nn * 8);
    d.t1 = take(nn * 4); d.t2 = take(nn * 4); d.t3 = take(nn * 4);
    d.t1s = (uint8_t*)take((nn + 31) / 32); d.t2s = (uint8_t*)take((nn + 31) / 32);
    d.t3s = (uint8_t*)take((nn + 31) / 32);
    d.partials = (double*)take(sizeof(double) * NSLOTS * MAXP_ITEM);
    d.ctrl = B.d_ctrl + i;
    d.lam2 = lambdas[i] * lambdas[i];
    d.lam2f = (float)d.lam2;
    d.taps32 = P.taps32; d.taps32_flip = P.taps32_flip;
    d.taps64 = P.taps64; d.taps64_flip = P.taps64_flip;
    d.VcT16 = (const _Float16*)P.VcT16; d.Vc16 = (const _Float16*)P.Vc16;
    d.Vr16 = (const _Float16*)P.Vr16; d.VrT16 = (const _Float16*)P.VrT16;
    d.VcT32 = P.VcT32; d.Vc32 = P.Vc32; d.Vr32 = P.Vr32; d.VrT32 = P.VrT32;
    d.VcT8 = P.VcT8; d.Vc8 = P.Vc8; d.Vr8 = P.Vr8; d.VrT8 = P.VrT8;
    d.VcT8s = P.VcT8s; d.Vc8s = P.Vc8s; d.Vr8s = P.Vr8s; d.VrT8s = P.VrT8s;
    d.sc2 = P.sc2; d.sr2 = P.sr2;
    d.d0 = (mode & KP_EXACT_DIAG) ? P.d0 : nullptr;
    d.b = b[i];
    d.x = x[i];
    d.warm = (mode & KP_WARM) ? 1 : 0;
    Ctrl& c = B.h_ctrl[i];
    std::memset(&c, 0, sizeof(c));
    c.tol_rel2 = tol * tol;
    c.lam2 = d.lam2;
    c.maxit = maxit;
    c.solver = B.solver;
    c.prec = B.prec;
    c.first = 1;
    c.done = RUNNING;
    c.pscale = 1.0f;
    c.zscale = (float)(1.0 / d.lam2);
    c.fastu = B.fast_tr && tol >= (d.use_mfma ? TR_FASTU_TOL_MFMA : TR_FASTU_TOL_VALU) ? 1 : 0;
  }
  B.d_tab = reinterpret_cast<TileRef*>(base + off_tab);
  B.h_tab.reserve(ntab);

  int rc = KP_OK;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev = nullptr;
#define BCHK(x)                                  \
  do {                                           \
    if ((x) != hipSuccess) { rc = KP_ERR_HIP; goto out; } \
  } while (0)
  // order after the caller's stream
  BCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  BCHK(hipEventRecord(ev, user_stream));
  BCHK(hipStreamWaitEvent(B.s, ev, 0));
  BCHK(hipMemcpyAsync(B.d_items, B.h_items.data(), sizeof(ItemDesc) * nitems,
                      hipMemcpyHostToDevice, B.s));
  {
    const std::vector<char> every(nitems, 1);
    BCHK(build_tables(B, every));
  }
  BCHK(hipMemcpyAsync(B.d_ctrl, B.h_ctrl, sizeof(Ctrl) * nitems, hipMemcpyHostToDevice, B.s));
  BCHK(hipStreamSynchronize(B.s));

  BCHK(ensure_splitk_b<_Float16>());
  BCHK(ensure_splitk_b<float>());
  // x_0 = 0 (or the caller's x), r = c = A^T b, ||c||; for a warm start
  // the residual r = c - H x_0 is a full FP64 true residual (which may find
  // the item converged already); then the first direction
  BCHK(vec_launch<VK_INIT>(B, RM_ALL));
  BCHK(blur_groups_launch<BK_RHS>(B, RM_ALL));          // r = c = A^T b (FP32 blur)
  BCHK(scalar_launch(B, SC_RHS, RM_ALL));
  if (mode & KP_WARM) {
    BCHK(true_residual_b(B, RM_RUNNING, SC_TRUE));
    BCHK(tail_b(B, RM_RUNNING));
    hipLaunchKernelGGL(clear_resume_kernel, dim3((nitems + 255) / 256), dim3(256), 0, B.s,
                       B.d_items, nitems);
    BCHK(hipGetLastError());
  } else {
    BCHK(tail_b(B, RM_RUNNING));
  }
  if ((rc = read_ctrls(B)) != KP_OK) goto out;

  {
    const int block = 8;
    BCHK(ensure_fast<BK_A>(B));
    BCHK(ensure_fast<BK_AT_NORMAL>(B));
    // the block of iterations as a graph of the current tables
    auto capture = [&]() -> hipError_t {
      if (exec) hipGraphExecDestroy(exec);
      if (graph) hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
      hipError_t e = hipStreamBeginCapture(B.s, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return e;
      for (int it = 0; it < block && e == hipSuccess; ++it) e = iteration_b(B);
      hipError_t e2 = hipStreamEndCapture(B.s, &graph);
      if (e != hipSuccess) return e;
      if (e2 != hipSuccess) return e2;
      return hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    };
    if (!eager) BCHK(capture());
    int in_tables = nitems;                    // items the tables cover
    std::vector<char> live(nitems, 0);
    for (int guard = 0; guard < 1000000; ++guard) {
      int running = 0, pending = 0;
      for (int i = 0; i < nitems; ++i) {
        running += B.h_ctrl[i].done == RUNNING;
        pending += B.h_ctrl[i].done == PENDING;
        live[i] = B.h_ctrl[i].done == RUNNING || B.h_ctrl[i].done == PENDING;
      }
      if (!running && !pending) break;
      // once half of the items in the tables have finished, rebuild them for
      // the live items only (finished items' blocks would otherwise still be
      // launched, only to return at once) and capture the graph anew
      if (2 * (running + pending) <= in_tables) {
        BCHK(build_tables(B, live));
        in_tables = running + pending;
        if (!eager) BCHK(capture());
      }
      if (pending) {
        BCHK(pending_residuals_b(B));
        BCHK(tail_b(B, RM_RESUME));
        hipLaunchKernelGGL(clear_resume_kernel, dim3((nitems + 255) / 256), dim3(256), 0, B.s,
                           B.d_items, nitems);
        BCHK(hipGetLastError());
      }
      if (running || pending) {
        if (eager) {
          for (int it = 0; it < block; ++it) BCHK(iteration_b(B));
        } else {
          BCHK(hipGraphLaunch(exec, B.s));
        }
      }
      if ((rc = read_ctrls(B)) != KP_OK) goto out;
    }
  }
  // report: true residual of unconverged items, x in FP32, data misfit (the
  // tables cover every item again)
  {
    const std::vector<char> every(nitems, 1);
    BCHK(build_tables(B, every));
  }
  BCHK(true_residual_b(B, RM_FINISHED, SC_TRUE_INFO));
  BCHK(vec_launch<VK_TO_F32>(B, RM_ALL));
  BCHK(blur_groups_launch<BK_MISFIT>(B, RM_ALL));
  BCHK(scalar_launch(B, SC_NORM, RM_ALL));
  if ((rc = read_ctrls(B)) != KP_OK) goto out;
  for (int i = 0; i < nitems; ++i) {
    const Ctrl& c = B.h_ctrl[i];
    kp_info_t& inf = infos[i];
    std::memset(&inf, 0, sizeof(inf));
    inf.iters = c.iter;
    inf.status = c.done == CONVERGED ? KP_OK : (c.done == BREAKDOWN ? KP_BREAKDOWN : KP_MAXIT);
    if (c.done == MAXIT && c.true_rr <= c.tol2) inf.status = KP_OK;
    inf.relres_rec = c.gamma0sq > 0 ? std::sqrt(c.rr / c.gamma0sq) : 0.0;
    inf.relres_true = c.gamma0sq > 0 ? std::sqrt(c.true_rr / c.gamma0sq) : 0.0;
    inf.lambda = lambdas[i];
    inf.rhs_norm = std::sqrt(c.gamma0sq);
    inf.misfit = std::sqrt(c.misfit2);
    inf.replacements = c.repl;
  }
  BCHK(hipEventRecord(ev, B.s));
  BCHK(hipStreamWaitEvent(user_stream, ev, 0));
out:
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  if (ev) hipEventDestroy(ev);
  destroy_batch(B);
  return rc;
#undef BCHK
}

}  // namespace kpcg
