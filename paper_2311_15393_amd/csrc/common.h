// Internal declarations shared by the HIP translation units of libkpcg.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stddef.h>
#include <stdint.h>

#include "kpcg.h"

namespace kpcg {

// ---------------------------------------------------------------------------
// Device-resident solver state.  Every kernel of an iteration reads `done`
// on entry and returns at once if it is set, so the host can enqueue a block
// of iterations and synchronise only at block boundaries.
// ---------------------------------------------------------------------------
enum DoneState : int {
  RUNNING = 0,
  CONVERGED = 1,   // set only after the FP64 true residual met the tolerance
  MAXIT = 2,
  BREAKDOWN = 3,
  PENDING = 4,     // the recurrence residual met the tolerance; the host
                   // must confirm with the true residual
};

enum Slot : int {
  SLOT_DELTA = 0,  // p . Hp
  SLOT_RR = 1,     // ||r||^2
  SLOT_RZ = 2,     // r . z
  SLOT_ZW = 3,     // z . Hp (flexible update)
  SLOT_TRUE = 4,   // true residual ||c - Hx||^2
  SLOT_RHS = 5,    // ||A^T b||^2
  SLOT_NORM = 6,   // standalone norms
  NSLOTS = 8
};

constexpr int MAX_PARTIALS = 16384;

// The recurrence residual is replaced by the FP64 true residual whenever it
// has fallen by this factor (in norm) since the last recomputation: beyond
// that, FP32 matvec rounding (about 1e-6 of ||r|| at the last recomputation)
// would no longer be small against ||r||.
constexpr double REPLACE_DROP = 1e-3;

struct Ctrl {
  double rho;       // r . z (r . r for CG)
  double rho_prev;
  double delta;     // p . Hp
  double alpha, beta;
  double rr;        // ||r||^2 (recurrence, or the last true residual)
  double rz, zw;
  double gamma0sq;  // ||A^T b||^2
  double tol2;      // tol^2 ||A^T b||^2
  double tol_rel2;  // tol^2
  double lam2;      // lambda^2
  double true_rr;
  double repl2;     // recompute the true residual once ||r||^2 falls below this
  float pscale;     // power-of-two scale applied to r before FP16 rounding
  float zscale;     // 1 / (pscale * lambda^2)
  int iter, maxit;
  int done;
  int solver;       // KP_CG / KP_PCG / KP_FPCG
  int prec;         // KP_P32 / KP_P16 / KP_P8
  int first;        // 1 while the initial z is being formed (beta = 0)
  int resume;       // batched solves: the direction update is still owed after
                    // a true-residual recomputation
  int repl;         // true-residual recomputations that replaced r
  double misfit2;   // ||A x - b||^2 (batched solves)
  int anchor;       // batched solves: (x_a, r_a) holds a true residual small
                    // enough (<= ANCHOR_REL ||A^T b||) to anchor the next one
  int pub;          // publications to the host mirror so far (CtrlMirror)
  int fastu;        // batched solves: u = b - A x of a full true residual is
                    // formed on the item's fast blur (TR_FASTU_TOL_*)
  int fr_next;      // a true residual replaced r: the next beta is
                    // Fletcher-Reeves (the Polak-Ribiere form -z.Hp / delta
                    // assumes r_new = r_old - alpha Hp, which the
                    // replacement breaks; with one unknown it cancels p)
  double* hist;     // KP_HIST: ||r_k||^2 at [k], true residuals at
                    // [KP_HIST_MAX + k]; null when not recording
};

// The convergence state as the scalar steps publish it to coherent pinned
// host memory, so that the host follows a solve without stream round trips:
// one naturally aligned 64-bit word, written with a single store (so the
// host never sees a torn state, and no fence is needed: the store lands at
// the latest when the kernel ends).
//   bits  0-23  publication number p = 1, 2, ... (mod 2^24)
//   bits 24-47  iterations done
//   bits 48-51  state (RUNNING, CONVERGED, MAXIT, BREAKDOWN, PENDING)
//   bit  52     the residual norm met the tolerance (PENDING for a check)
//   bit  53     the last true residual may anchor the next one
//   bits 54-63  true-residual replacements (mod 2^10)
// The values the host reports at the end of a solve are written beside it;
// they are read only after the stream has drained.
struct CtrlMirror {
  unsigned long long word;
  double rr, true_rr, gamma0sq, tol2;
  int iter, pad_;
};
constexpr unsigned MIRROR_PUB_MASK = (1u << 24) - 1u;

// A true residual r_a at x_a anchors later ones, r = r_a - H (x - x_a) with
// FP32 matvecs on the step, once ||r_a|| <= ANCHOR_REL ||A^T b|| and
// ||r_a|| <= ANCHOR_TOL tol ||A^T b||.  The FP32-class matvecs err by up to
// about 1e-5 ||r_a|| (7e-6 measured on a reflexive FP16 solve at tol 2e-8),
// so the second bound keeps the anchored residual within a tenth of the
// tolerance; the first decides at loose tolerances.
constexpr double ANCHOR_REL = 1e-2;
constexpr double ANCHOR_TOL = 1e4;

// True residuals are formed as A^T u - lambda^2 x from u = b - A x (FP64).
// For tolerances >= TR_FAST_TOL the A^T u product runs on the FP32-class
// blur: its error is ~2e-8 ||A|| ||u||, below 1e-8 ||A^T b|| for data
// residuals ||u|| of a few per cent of ||b|| and below TR_FAST_TOL / 5 even
// at ||u|| = ||b||; tighter tolerances use the FP64 blur for it.
constexpr double TR_FAST_TOL = 1e-7;
// From these tolerances on, u = b - A x is formed on the fast blur as well
// (x rounded to FP32).  Its error reaches the residual as A^T du, smoothed by
// the blur, and x only through the Tikhonov filter (A^T A + lambda^2 I)^-1
// A^T, whose norm is at most 1 / (2 lambda) (the form c - H x would amplify
// by 1 / lambda^2).  Measured at 1024^2, K = 63: ||dr|| <= 6.5e-8 ||A^T b||
// on the MFMA blur, <= 1.4e-7 on the FP32 VALU blur; x moves by <= 1.7e-6
// and 5e-6 of its norm.
constexpr double TR_FASTU_TOL_MFMA = 1e-6;
constexpr double TR_FASTU_TOL_VALU = 1e-5;
// how a true residual forms u = b - A x and A^T u
enum TrMode : int { TR_FP64 = 0, TR_FAST_AT = 1, TR_FAST_ALL = 2 };

// ---------------------------------------------------------------------------
// reductions: deterministic two-stage sums (per-block FP64 partials, summed
// in a fixed order by whichever block finishes last)
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block; the result is valid in thread 0.
template <int NT>
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += sh[w];
  }
  return t;
}

// Write this block's partial sum(s) (valid in thread 0) for slots
// [slot, slot + nv).  A single-block scalar kernel sums them afterwards in a
// fixed order, so no atomics or fences are needed and the result is
// deterministic.
template <int NV>
__device__ inline void write_partials(const double (&v)[NV], double* partials, int slot,
                                      int bid) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) partials[(slot + k) * MAX_PARTIALS + bid] = v[k];
  }
}

// Power of two s with s * sqrt(rr) < 2^14 (keeps every FP16 intermediate of
// the preconditioner below 65504, since V is orthogonal).
__device__ inline float fp16_residual_scale(double rr) {
  if (!(rr > 0.0) || !isfinite(rr)) return 1.0f;
  int e;
  frexp(sqrt(rr), &e);
  int p = 14 - e;
  p = p > 126 ? 126 : (p < -126 ? -126 : p);
  return ldexpf(1.0f, p);
}

__device__ inline void set_scales(Ctrl* c, double rr) {
  const float s = (c->prec == KP_P16) ? fp16_residual_scale(rr) : 1.0f;
  c->pscale = s;
  c->zscale = (float)(1.0 / ((double)s * c->lam2));
}

// ---------------------------------------------------------------------------
// The iteration's scalar logic, shared by the one-block scalar step and by
// the kernels that fold a scalar step into their start: there every block
// sums the partials of the kernel before it, in the scalar step's order (so
// all blocks obtain the same value and take the same decision), and block 0
// alone writes the control block.  A kernel that folds a step reads no
// control-block field that its block 0 writes.  (A last-block reduction
// would need device-scope release/acquire fences, whose L2 write-backs
// measured far slower than a second launch.)
// ---------------------------------------------------------------------------
constexpr int FOLD_T = 256;            // threads that read partials, as the scalar step
constexpr int FOLD_W = FOLD_T / 64;    // ... and their waves

// Doubles of LDS scratch a fold in a block of NT threads needs (fold_slot2:
// twice as many).
template <int NT>
constexpr int fold_sh() {
  return (NT / 64 > FOLD_W ? NT / 64 : FOLD_W) + 1;
}

// Sum of the nb partials of `slot` in the scalar step's order, whatever the
// block size NT: FOLD_T virtual threads stride over the partials (virtual
// thread v sums partials v, v + FOLD_T, ... from zero), each virtual wave of
// 64 is reduced by one real wave (real wave w takes virtual waves w,
// w + NT/64, ...: a block of fewer than FOLD_T threads covers them all), and
// the FOLD_W wave totals are added in order.  Returned to every thread
// through sh[fold_sh<NT>()], which is free again on return (the first GEMM
// stages its operands into the same LDS).
template <int NT>
__device__ inline double fold_slot(const double* __restrict__ partials, int slot, int nb,
                                   double* sh) {
  constexpr int RW = NT / 64, PER = (FOLD_W + RW - 1) / RW;   // virtual waves per real wave
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int vw = wid + k * RW;
    double s = 0.0;
    if (vw < FOLD_W)
      for (int i = vw * 64 + lane; i < nb; i += FOLD_T) s += partials[slot * MAX_PARTIALS + i];
    v[k] = wave_sum(s);
  }
  __syncthreads();                     // sh may still be read by an earlier reduction
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (lane == 0 && wid + k * RW < FOLD_W) sh[wid + k * RW] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < FOLD_W; ++w) t += sh[w];
    sh[FOLD_W] = t;
  }
  __syncthreads();
  const double r = sh[FOLD_W];
  __syncthreads();                     // every thread has read it: the caller may reuse sh
  return r;
}

// Two slots at once (one round of partial loads, one block reduction),
// each summed exactly as fold_slot sums it.  sh: 2 fold_sh<NT>() doubles.
template <int NT>
__device__ inline double2 fold_slot2(const double* __restrict__ partials, int slot_a, int slot_b,
                                     int nb, double* sh) {
  constexpr int RW = NT / 64, PER = (FOLD_W + RW - 1) / RW;   // virtual waves per real wave
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double va[PER], vb[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int vw = wid + k * RW;
    double a = 0.0, b = 0.0;
    if (vw < FOLD_W)
      for (int i = vw * 64 + lane; i < nb; i += FOLD_T) {
        a += partials[slot_a * MAX_PARTIALS + i];
        b += partials[slot_b * MAX_PARTIALS + i];
      }
    va[k] = wave_sum(a);
    vb[k] = wave_sum(b);
  }
  __syncthreads();                     // sh may still be read by an earlier reduction
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (lane == 0 && wid + k * RW < FOLD_W) {
      sh[2 * (wid + k * RW)] = va[k];
      sh[2 * (wid + k * RW) + 1] = vb[k];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int w = 0; w < FOLD_W; ++w) {
      ta += sh[2 * w];
      tb += sh[2 * w + 1];
    }
    sh[2 * FOLD_W] = ta;
    sh[2 * FOLD_W + 1] = tb;
  }
  __syncthreads();
  const double2 r = make_double2(sh[2 * FOLD_W], sh[2 * FOLD_W + 1]);
  __syncthreads();                     // every thread has read it: the caller may reuse sh
  return r;
}

// r.z of the current direction: the last direction step's (PCG, FPCG) or
// ||r||^2 (CG)
__device__ inline double step_rho(const Ctrl* c) { return c->solver == KP_CG ? c->rho : c->rz; }

// After the step length (one thread): the direction step's r.z becomes the
// previous one, and the first-step and Fletcher-Reeves flags are spent.
// (The direction step itself writes none of these: its blocks read them.)
__device__ inline void commit_direction(Ctrl* c) {
  if (c->solver != KP_CG) {
    c->rho = c->rz;
    c->first = 0;
    c->fr_next = 0;
  }
}

// The state after an update with ||r||^2 = S (read-only: every block of a
// folding kernel evaluates it).
__device__ inline int rr_state(const Ctrl* c, double S) {
  if (!isfinite(S)) return BREAKDOWN;
  if (S <= c->tol2 || S <= c->repl2) return PENDING;
  return RUNNING;
}

// The residual-norm step after x += alpha p, r -= alpha w (one thread).
__device__ inline void apply_rr(Ctrl* c, double S) {
  c->rr = S;
  c->iter += 1;
  if (c->solver == KP_CG) {
    c->rho_prev = c->rho;
    c->beta = S / c->rho;
    c->rho = S;
  }
  set_scales(c, S);
  const int st = rr_state(c, S);
  if (st != RUNNING) c->done = st;
  // KP_HIST: the recurrence norm after each iteration
  if (c->hist != nullptr && c->iter >= 0 && c->iter < KP_HIST_MAX) c->hist[c->iter] = S;
}

// Whether a true residual with ||r||^2 = true_rr may anchor the next ones.
__device__ inline bool anchor_eligible(const Ctrl* c, double true_rr) {
  const double lim = fmin(ANCHOR_REL * ANCHOR_REL, ANCHOR_TOL * ANCHOR_TOL * c->tol_rel2);
  return true_rr <= lim * c->gamma0sq;
}

// The new state to the host mirror (one thread).
__device__ inline void publish_mirror(Ctrl* __restrict__ c, CtrlMirror* __restrict__ mirror) {
  const unsigned p = ((unsigned)c->pub + 1u) & MIRROR_PUB_MASK;
  c->pub = (int)p;
  const bool tol_hit = c->rr <= c->tol2;
  const bool anchor_ok = c->repl > 0 && anchor_eligible(c, c->true_rr);
  const unsigned long long w =
      (unsigned long long)p | ((unsigned long long)(c->iter & 0xffffff) << 24) |
      ((unsigned long long)(c->done & 0xf) << 48) | ((unsigned long long)tol_hit << 52) |
      ((unsigned long long)anchor_ok << 53) | ((unsigned long long)(c->repl & 0x3ff) << 54);
  volatile CtrlMirror* m = mirror;
  m->rr = c->rr;
  m->true_rr = c->true_rr;
  m->gamma0sq = c->gamma0sq;
  m->tol2 = c->tol2;
  m->iter = c->iter;
  m->word = w;
}

// beta of the direction step from r.z and z.Hp: Fletcher-Reeves rz / rho
// (PCG, and the step after a true-residual replacement), Polak-Ribiere
// -zw / delta (FPCG: equals -alpha (z.Hp) / rho), 0 for the first
// direction.  Read-only; *ok is false for a breakdown.
__device__ inline double beta_of(const Ctrl* c, double rz, double zw, bool* ok) {
  *ok = (rz > 0.0) && isfinite(rz) && isfinite(zw);
  if (!*ok) return 0.0;
  if (c->first) return 0.0;
  if (c->solver == KP_PCG || c->fr_next) return rz / c->rho;
  return -zw / c->delta;
}

// The control-block fields from which the folded scalar steps decide (the
// state after ||r||^2, the step length, beta), read by every workgroup at
// its kernel's start, before its first global loads.  Read after the fold,
// each would add a memory latency to every workgroup's path, since each read
// hangs on a branch over the one before.  A kernel that takes the snapshot
// uses only fields that none of its own workgroups writes (block 0's step
// writes others), so every workgroup sees what the kernels before it left.
struct StepIn {
  double tol2, repl2, rho, rz, delta;
  int solver, prec, first, fr_next;
};

__device__ inline StepIn step_in(const Ctrl* c) {
  StepIn k;
  k.tol2 = c->tol2;
  k.repl2 = c->repl2;
  k.rho = c->rho;
  k.rz = c->rz;
  k.delta = c->delta;
  k.solver = c->solver;
  k.prec = c->prec;
  k.first = c->first;
  k.fr_next = c->fr_next;
  return k;
}

// rr_state, beta_of and step_rho on a snapshot taken by step_in
__device__ inline int rr_state(const StepIn& k, double S) {
  if (!isfinite(S)) return BREAKDOWN;
  if (S <= k.tol2 || S <= k.repl2) return PENDING;
  return RUNNING;
}

__device__ inline double beta_of(const StepIn& k, double rz, double zw, bool* ok) {
  *ok = (rz > 0.0) && isfinite(rz) && isfinite(zw);
  if (!*ok) return 0.0;
  if (k.first) return 0.0;
  if (k.solver == KP_PCG || k.fr_next) return rz / k.rho;
  return -zw / k.delta;
}

__device__ inline double step_rho(const StepIn& k) { return k.solver == KP_CG ? k.rho : k.rz; }

// radices of the FFT form's transform length (three stages)
constexpr int FFT_MAX_RADICES = 3;

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct Plan {
  int n = 0, k = 0, kq = 0;       // kq: PSF row length padded to the tap chunk
  int bc = KP_BC_ZERO;            // boundary condition of A (KP_BC_ZERO / KP_BC_PERIODIC)
  bool refl_general = false;      // reflexive boundary with a PSF not symmetric in both
                                  // axes: A^T is not the blur, so H p, A^T b and the
                                  // true residuals' A^T go through the FFT form
  bool lowp = false;              // KP_SETUP_LOWP: factors rounded to FP16, FP32 SVDs
  bool owns = false;
  void* base = nullptr;
  size_t bytes = 0;

  // blur taps (row-major K x kq, zero padded): P for A^T, flipped P for A
  float* taps32 = nullptr;
  float* taps32_flip = nullptr;
  double* taps64 = nullptr;
  double* taps64_flip = nullptr;
  // MFMA fragments of the banded Toeplitz tap blocks (blur_mfma.hip): the
  // table for taps32, then the one for taps32_flip; taps scaled by 2^mfma_exq
  void* mfma_taps = nullptr;
  void* mfma32_taps = nullptr;   // tap fragments of the 32 x 32 x 16 MFMA blur
  int mfma_exq = 0;

  // KP-SVD factors
  double* sc = nullptr;          // singular values of A_c (descending)
  double* sr = nullptr;
  float* sc2 = nullptr;          // squares in FP32
  float* sr2 = nullptr;
  float* d0 = nullptr;           // exact KP-basis diagonal diag(V^T A^T A V), [n][n]
  float* d0t = nullptr;          // the same transposed, [j][i]
  const float* sprime_d0 = nullptr;  // the current solve's S' table: d0 with
                                     // KP_EXACT_DIAG, else nullptr (s_c^2 s_r^2)
  float* Vc32 = nullptr;         // row-major Vc[i][a]
  float* VcT32 = nullptr;        // row-major Vc^T
  float* Vr32 = nullptr;
  float* VrT32 = nullptr;
  __half* Vc16 = nullptr;
  __half* VcT16 = nullptr;
  __half* Vr16 = nullptr;
  __half* VrT16 = nullptr;
  uint8_t* Vc8 = nullptr;        // e4m3 codes, row-major, + block exponents
  uint8_t* VcT8 = nullptr;
  uint8_t* Vr8 = nullptr;
  uint8_t* VrT8 = nullptr;
  uint8_t* Vc8s = nullptr;       // E8M0 exponents, [rows][n/32]
  uint8_t* VcT8s = nullptr;
  uint8_t* Vr8s = nullptr;
  uint8_t* VrT8s = nullptr;
  float* UcT32 = nullptr;        // row-major Uc^T
  float* UrT32 = nullptr;        // row-major Ur^T

  // solver vectors
  float *r = nullptr, *p = nullptr, *q = nullptr, *w = nullptr, *z = nullptr;
  double* y64 = nullptr;         // FP64 scratch (b - A x of the FP64 true residual)
  double* x64 = nullptr;         // FP64 solution accumulator
  double* xa64 = nullptr;        // anchor: x and its true residual (FP64)
  double* ra64 = nullptr;
  // preconditioner intermediates (sized for FP32)
  void *t1 = nullptr, *t2 = nullptr, *t3 = nullptr;
  uint8_t *t1s = nullptr, *t2s = nullptr, *t3s = nullptr, *rs = nullptr;  // FP8 block exponents
  uint8_t* r8 = nullptr;                                                 // FP8 residual codes
  double* spec = nullptr;        // spectral scratch (GCV)
  Ctrl* ctrl = nullptr;
  double* partials = nullptr;
  double* hist = nullptr;        // residual history (2 KP_HIST_MAX FP64)
  int hist_count = 0;            // entries recorded by the last solve
  double hist_gamma0sq = 0.0;    // its ||A^T b||^2
  hipEvent_t ev_last = nullptr;   // recorded after the plan's last enqueued work
  hipEvent_t ev_start = nullptr;  // pcg_solve timing (created on first use)
  hipEvent_t ev_end = nullptr;
  Ctrl* host_ctrl = nullptr;     // pinned
  CtrlMirror* mirror = nullptr;  // coherent pinned host memory (host address)
  CtrlMirror* mirror_dev = nullptr;  // its device address

  // FFT form of the normal operator (fft.hip): length L, its radices, the
  // twiddle table, the PSF spectrum (transposed, scaled by 1/L^2) and two
  // n x (L/2 + 1) complex work arrays
  int fft_L = 0, fft_nrad = 0;
  int fft_rad[FFT_MAX_RADICES] = {};
  void* fft_tw = nullptr;
  void* fft_Ht = nullptr;
  void* fft_S = nullptr;
  void* fft_T = nullptr;
  int normal_op = 0;             // H p by the direct blurs (0) or the FFTs (1)
  float normal_times[2] = {};    // autotuner time of each form (ms)

  int blur_cfg = 0;              // blur kernel (autotuned; BLUR_CFG_MFMA = MFMA)
  int blur_cfg_valu = 0;         // fastest FP32-VALU tile shape (batched path)
  float blur_times[8] = {};      // autotuner timings (ms) per candidate

  // properties
  double kp_err = 0.0;
  int terms = 0;
  double sc_max = 0, sc_min = 0, sr_max = 0, sr_min = 0;
};

// ---------------------------------------------------------------------------
// launchers (return hipError_t)
// ---------------------------------------------------------------------------
hipError_t launch_blur_f32(const Plan& P, const float* src, float* dst, bool transpose,
                           hipStream_t s, const Ctrl* ctrl);
// w = A^T q + lambda^2 p with the partials of p.w; *nb receives their count
hipError_t launch_blur_normal(const Plan& P, const float* q, const float* p, float* w,
                              float lam2, hipStream_t s, int* nb);
// r = c = A^T b on the plan's blur, ||c||^2 (the SC_RHS scalar step); also
// p = w = 0 and, with zero_x, x = 0
hipError_t launch_rhs(const Plan& P, const float* b, bool zero_x, hipStream_t s);
// the control block set to `c` by a kernel (stream-ordered, no host sync)
hipError_t launch_init_ctrl(const Plan& P, const Ctrl& c, hipStream_t s);
hipError_t autotune_blur(Plan& P, hipStream_t s, float* times_ms);
// r = r_a - H (x - x_a) from the anchor (x_a, r_a) of the last true residual,
// with the FP32 blur kernels on the difference and FP64 epilogue arithmetic;
// moves the anchor to x
hipError_t launch_anchor_residual(const Plan& P, double lam2, bool fin, hipStream_t s);
hipError_t launch_diff32(const Plan& P, float* d, hipStream_t s);
// r = A^T (b - A x) - lam2 x with u = b - A x and A^T u on the FP64 blur or
// the plan's fast blur as TrMode says; records the anchor (x, r)
hipError_t launch_true_residual(const Plan& P, const float* b, const double* x64, double lam2,
                                bool fin, int trmode, hipStream_t s);
hipError_t launch_normal_fp64(const Plan& P, const float* x, double lam2, double* y,
                              hipStream_t s);

// x += alpha p, r -= alpha w with the partials of ||r||^2; with rr_step the
// residual-norm scalar step follows as a launch of its own, else the
// preconditioner's first GEMM folds it in (launch_precond's fold_rr)
hipError_t launch_update(const Plan& P, bool rr_step, hipStream_t s);
// alpha = rho / p.Hp from the normal blur's nbd partials, then the update
hipError_t launch_update_alpha(const Plan& P, int nbd, bool rr_step, hipStream_t s);
int update_partials(const Plan& P);     // partials of ||r||^2 an update writes
// p = z + beta p with beta from the nbz partials of r.z and z.Hp of the
// preconditioner's last GEMM (the direction step folded in; publishes)
hipError_t launch_pupdate_fold(const Plan& P, const float* z, int nbz, hipStream_t s);
hipError_t launch_convert_x(const Plan& P, float* x, bool to_f32, hipStream_t s);
hipError_t launch_pupdate(const Plan& P, hipStream_t s);
hipError_t launch_norm_scale(const Plan& P, const float* v, hipStream_t s);

// single-block kernels that turn per-block partials into the iteration's
// scalars (see scalar_kernel in vec.hip)
enum ScalarKind : int {
  SC_ALPHA = 0,    // delta = p.Hp -> alpha, breakdown test
  SC_RR = 1,       // ||r||^2 -> convergence / replacement test, FP16 scale, CG beta
  SC_BETA = 2,     // r.z, z.Hp -> beta (batched solves; pcg_solve folds it into
                   // the direction update, launch_pupdate_fold)
  SC_RHS = 3,      // ||A^T b||^2 -> tolerances
  SC_TRUE = 4,     // true residual ||c - Hx||^2 -> converged / continue
  SC_TRUE_INFO = 5,// true residual for reporting only
  SC_NORM = 6,     // ||r||^2 -> preconditioner scales only
};
hipError_t launch_scalar(const Plan& P, int kind, int nb, hipStream_t s);
hipError_t launch_fill_f64(double* a, int count, double v, hipStream_t s);
hipError_t launch_init_ctrl(const Plan& P, const Ctrl& host, hipStream_t s);

// z = M^{-1} r.  finalize: the solver's tail (kernels skip a finished
// solve; the last GEMM writes the partials of r.z and z.w, which
// launch_pupdate_fold consumes: precond_partials of them).  fold_rr > 0:
// the first GEMM folds in the residual-norm step of the update before it,
// summing that update's fold_rr partials of ||r||^2 (and publishes).
hipError_t launch_precond(const Plan& P, const float* r, float* z, const float* w,
                          int prec, bool finalize, float lam2, hipStream_t s,
                          int fold_rr = 0);
hipError_t launch_precond_fp8(const Plan& P, const float* r, float* z, const float* w,
                              bool finalize, float lam2, hipStream_t s, int fold_rr = 0);
int precond_partials(const Plan& P, int prec);
int precond_partials_fp8(const Plan& P);
bool fp8_supported_size(int n);   // the FP8 chain needs n to be a multiple of 128

// Non-blocking streams of the current device, created once per device and
// slot and kept for the process: the getters' copies run on AUX_COPY, the
// batched solver (whose iterations are captured into a graph; the caller's
// stream may be the legacy default stream, which cannot be captured) on
// AUX_BATCH.  NULL on error.
enum AuxSlot : int { AUX_COPY = 0, AUX_BATCH = 1 };
hipStream_t aux_stream(int slot);

// The batched solve.  With need_out set, stores the workspace bytes the
// batch needs there and, if ws is NULL, returns without launching anything.
int batched_solve(Plan* const* plans, const int* plan_of_item, int nitems, int mode,
                  double tol, int maxit, const float* const* b, const double* lambdas,
                  float* const* x, kp_info_t* infos, void* ws, size_t ws_bytes,
                  size_t* need_out, hipStream_t user_stream);
hipError_t launch_spectral_gemms(const Plan& P, const float* b, float* out, hipStream_t s);

// MFMA blur (blur_mfma.hip): chunks per tap row, table entries per
// orientation (16 bytes each), workgroups per launch, table construction
int mfma_nch(int K);
size_t mfma_taps_count(int K);
size_t mfma32_taps_count(int K);      // the same for the 32 x 32 x 16 kernel
int mfma_blocks(int n);
hipError_t build_mfma_taps(const Plan& P, hipStream_t s);

// FFT form of w = A^T A p + lam2 p with the partials of p.w (fft.hip); the
// plan's FFT length and radices, and the twiddle / PSF-spectrum tables
// (g_scratch: K (L/2 + 1) complex FP64).  The lengths come from a fixed
// menu; -1: no menu length is long enough (no FFT form for the plan).
int fft_length(int n, int k);
int fft_radices(int L, int* rad);
// the longer of the two boundaries' lengths that exist (the size of the FFT
// tables and work arrays), 0 when neither does
int fft_table_length(int n, int k);
hipError_t build_fft_tables(const Plan& P, const double* psf_dev, void* g_scratch,
                            hipStream_t s);
hipError_t launch_fft_normal(const Plan& P, const float* p, float* w, float lam2, hipStream_t s,
                             int* nb, const Ctrl* ctrl, bool with_partials = true);
// the same with the direction step p = z + beta p folded into its first pass
// (zero boundary; beta from nbz partials of r.z, z.Hp; publishes)
hipError_t launch_fft_normal_dir(const Plan& P, float lam2, int nbz, hipStream_t s, int* nb);
// A^T u alone by FFTs into out (the reflexive boundary's A^T for any PSF)
hipError_t launch_fft_at(const Plan& P, const float* u, float* out, hipStream_t s);
// the right-hand side, the true residual from u = b - A x in P.q, and the
// anchored true residual with their A^T (or A^T A) by FFTs (plans whose A^T
// is not a blur: refl_general)
hipError_t launch_fft_rhs(const Plan& P, const float* b, bool zero_x, hipStream_t s);
hipError_t launch_fft_true_res(const Plan& P, double lam2, bool fin, hipStream_t s);
hipError_t launch_fft_anchor_residual(const Plan& P, double lam2, bool fin, hipStream_t s);
int fft_length_reflexive(int n, int k);
// w = A^T A p + lam2 p on the plan's direct blurs (A p into P.q)
hipError_t launch_normal_direct(const Plan& P, const float* p, float* w, float lam2,
                                hipStream_t s, int* nb);
// time both forms of H p on this plan and keep the faster (P.normal_op)
hipError_t autotune_normal(Plan& P, hipStream_t s);
hipError_t launch_spectrum(const Plan& P, const float* b, hipStream_t s);
hipError_t launch_spectral_scores(const Plan& P, const double* grid_dev, int ngrid,
                                  double omega, double noise2, int kind, double* out_dev,
                                  hipStream_t s, const float* xhat = nullptr);
hipError_t launch_vbasis_gemms(const Plan& P, const float* b, float* out, hipStream_t s);
// 128 features of b (see spectral.hip) into out (device, 128 floats)
hipError_t launch_features(const Plan& P, const float* b, float* out, hipStream_t s);

}  // namespace kpcg
