// C ABI of libkpcg: plans, the (P)CG driver and the parameter-choice calls.
//
// The driver keeps all iteration scalars on the device (see Ctrl in
// common.h).  It enqueues blocks of iterations whose kernels turn into
// no-ops once the device marks the solve finished, and synchronises only at
// block boundaries to read the small control block.
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "blur_core.h"
#include "capi_internal.h"

using namespace kpcg;

namespace kpcg {
int build_factors(Plan& P, const double* psf_host, char* scratch, hipStream_t s);
size_t setup_scratch_bytes(int n, int k);
hipError_t launch_pupdate_from(const Plan& P, const float* z, hipStream_t s);
}

namespace {

constexpr int TAP_CHUNK = 16;
constexpr size_t ALIGN = 256;

struct Bump {
  char* base;
  size_t cur = 0;
  template <typename T>
  T* take(size_t count) {
    cur = (cur + ALIGN - 1) / ALIGN * ALIGN;
    T* p = base ? reinterpret_cast<T*>(base + cur) : nullptr;
    cur += count * sizeof(T);
    return p;
  }
};

// The plan's workspace: the persistent part (taps, factors, control block,
// partial sums, history), then one transient region shared by the solver's
// vectors and, during kp_setup only, the construction's scratch (its size is
// the larger of the two).  Returns the total bytes, 0 if the construction's
// scratch size cannot be determined; *scratch receives the region's start.
size_t layout(int n, int k, char* base, Plan* P, char** scratch = nullptr) {
  Bump b{base};
  const size_t nn = (size_t)n * n;
  const int kq = (k + TAP_CHUNK - 1) / TAP_CHUNK * TAP_CHUNK;
  const size_t nsc = (size_t)n * ((n + 31) / 32);
  Plan tmp;
  Plan& Q = P ? *P : tmp;
  Q.taps32 = b.take<float>((size_t)k * kq);
  Q.taps32_flip = b.take<float>((size_t)k * kq);
  Q.taps64 = b.take<double>((size_t)k * kq);
  Q.taps64_flip = b.take<double>((size_t)k * kq);
  Q.mfma_taps = b.take<uint8_t>(2 * mfma_taps_count(k) * 16);
  Q.mfma32_taps = b.take<uint8_t>(2 * mfma32_taps_count(k) * 16);
  Q.sc = b.take<double>(n);
  Q.sr = b.take<double>(n);
  Q.sc2 = b.take<float>(n);
  Q.sr2 = b.take<float>(n);
  Q.d0 = b.take<float>(nn);
  Q.d0t = b.take<float>(nn);
  Q.Vc32 = b.take<float>(nn);
  Q.VcT32 = b.take<float>(nn);
  Q.Vr32 = b.take<float>(nn);
  Q.VrT32 = b.take<float>(nn);
  Q.Vc16 = b.take<__half>(nn);
  Q.VcT16 = b.take<__half>(nn);
  Q.Vr16 = b.take<__half>(nn);
  Q.VrT16 = b.take<__half>(nn);
  Q.Vc8 = b.take<uint8_t>(nn);
  Q.VcT8 = b.take<uint8_t>(nn);
  Q.Vr8 = b.take<uint8_t>(nn);
  Q.VrT8 = b.take<uint8_t>(nn);
  Q.Vc8s = b.take<uint8_t>(nsc);
  Q.VcT8s = b.take<uint8_t>(nsc);
  Q.Vr8s = b.take<uint8_t>(nsc);
  Q.VrT8s = b.take<uint8_t>(nsc);
  Q.UcT32 = b.take<float>(nn);
  Q.UrT32 = b.take<float>(nn);
  // FFT tables and work arrays sized for the longer of the two lengths (none
  // where the menu has no length for either); the zero boundary's length is
  // the default, kp_setup sets the plan's own
  const int fL = fft_length(n, k);
  const int fLm = fft_table_length(n, k), fFm = fLm > 0 ? fLm / 2 + 1 : 0;
  const int hh = (k - 1) / 2;
  Q.fft_L = fL;
  Q.fft_nrad = fL > 0 ? fft_radices(fL, Q.fft_rad) : 0;
  Q.fft_tw = b.take<float2>((size_t)fLm);
  Q.fft_Ht = b.take<float2>((size_t)fFm * fLm);
  Q.spec = b.take<double>((((nn * sizeof(float)) + ALIGN - 1) / ALIGN * ALIGN) / sizeof(double) +
                          128 + 2 * 64 * 256);
  Q.ctrl = b.take<Ctrl>(1);
  Q.partials = b.take<double>((size_t)NSLOTS * MAX_PARTIALS);
  Q.hist = b.take<double>(2 * (size_t)KP_HIST_MAX);
  // transient region
  b.cur = (b.cur + ALIGN - 1) / ALIGN * ALIGN;
  const size_t region = b.cur;
  if (scratch) *scratch = base ? base + region : nullptr;
  Q.r = b.take<float>(nn);
  Q.p = b.take<float>(nn);
  Q.q = b.take<float>(nn);
  Q.w = b.take<float>(nn);
  Q.z = b.take<float>(nn);
  Q.y64 = b.take<double>(nn);
  Q.x64 = b.take<double>(nn);
  Q.xa64 = b.take<double>(nn);
  Q.ra64 = b.take<double>(nn);
  Q.t1 = b.take<float>(nn);
  Q.t2 = b.take<float>(nn);
  Q.t3 = b.take<float>(nn);
  Q.t1s = b.take<uint8_t>(nsc);
  Q.t2s = b.take<uint8_t>(nsc);
  Q.t3s = b.take<uint8_t>(nsc);
  Q.rs = b.take<uint8_t>(nsc);
  Q.r8 = b.take<uint8_t>(nn);
  Q.fft_S = b.take<float2>((size_t)(n + 2 * hh) * fFm);   // n + 2h row slots (reflexive)
  Q.fft_T = b.take<float2>((size_t)n * fFm);
  (void)Q;
  const size_t vec_end = (b.cur + ALIGN - 1) / ALIGN * ALIGN;
  const size_t scr = setup_scratch_bytes(n, k);
  if (scr == 0) return 0;
  const size_t scr_end = region + scr;
  return vec_end > scr_end ? vec_end : scr_end;
}

bool valid_sizes(int n, int k) {
  return n >= 1 && n <= 2048 && k >= 1 && (k & 1) == 1 && k <= 2 * n - 1;
}



int read_ctrl(Plan& P, hipStream_t s, Ctrl& out) {
  HIPCHK(hipMemcpyAsync(P.host_ctrl, P.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::memcpy(&out, P.host_ctrl, sizeof(Ctrl));
  return KP_OK;
}

int write_ctrl(Plan& P, hipStream_t s, const Ctrl& c) {
  HIPCHK(launch_init_ctrl(P, c, s));
  return KP_OK;
}

// The second half of an iteration: preconditioner and direction (CG: the
// direction only).  With fold_rr the preconditioner's first GEMM also takes
// the residual-norm step of the update before it (fold_rr > 0 partials);
// without, that step ran already (the right-hand side, a true residual).
// The direction step is folded into p = z + beta p.  Publishes twice with
// fold_rr (||r||, then r.z), else once; CG publishes nothing here.
// PCG and FPCG on the FFT form of a zero-boundary plan take the direction
// step in the first pass of the next H p instead (enqueue_matvec_half); the
// tail is then the preconditioner alone and publishes only with fold_rr.
bool dir_in_matvec(const Plan& P, int solver) {
  return solver != KP_CG && P.normal_op == KP_NORMAL_FFT && P.bc == KP_BC_ZERO;
}

hipError_t enqueue_tail(Plan& P, int solver, int prec, float lam2, hipStream_t s,
                        int fold_rr = 0) {
  hipError_t e;
  if (solver == KP_CG) return launch_pupdate_from(P, P.r, s);
  e = launch_precond(P, P.r, P.z, P.w, prec, true, lam2, s, fold_rr);
  if (e != hipSuccess || dir_in_matvec(P, solver)) return e;
  return launch_pupdate_fold(P, P.z, precond_partials(P, prec), s);
}

// The first half of an iteration: matvecs, step length, update.  With
// rr_step the residual-norm step follows as a launch of its own (CG, and the
// last iteration of a solve, where no preconditioner follows to fold it in)
// and publishes.  With dir_in_matvec the first FFT pass takes the direction
// step of the tail before it and publishes r.z.
hipError_t enqueue_matvec_half(Plan& P, int solver, int prec, float lam2, hipStream_t s,
                               bool rr_step = true) {
  hipError_t e;
  int nbd = 0;
  if (P.normal_op == KP_NORMAL_FFT) {
    // w = H p, p.w (FFTs); first p = z + beta p
    e = dir_in_matvec(P, solver) ? launch_fft_normal_dir(P, lam2, precond_partials(P, prec), s, &nbd)
                                 : launch_fft_normal(P, P.p, P.w, lam2, s, &nbd, P.ctrl);
    if (e != hipSuccess) return e;
  } else {
    e = launch_blur_f32(P, P.p, P.q, false, s, P.ctrl);         // q = A p
    if (e != hipSuccess) return e;
    e = launch_blur_normal(P, P.q, P.p, P.w, lam2, s, &nbd);    // w = A^T q + l^2 p, p.w
    if (e != hipSuccess) return e;
  }
  return launch_update_alpha(P, nbd, rr_step, s);               // alpha; x, r, ||r||
}

hipError_t enqueue_iteration(Plan& P, int solver, int prec, float lam2, hipStream_t s) {
  hipError_t e = enqueue_matvec_half(P, solver, prec, lam2, s, true);
  if (e != hipSuccess) return e;
  return enqueue_tail(P, solver, prec, lam2, s);
}

// The host mirror's latest publication, unpacked.
struct Snap {
  unsigned pub;
  int iter, done, repl;
  bool tol_hit, anchor_ok;
};

Snap read_mirror(const CtrlMirror* mirror) {
  const unsigned long long w = *reinterpret_cast<const volatile unsigned long long*>(&mirror->word);
  Snap out;
  out.pub = (unsigned)(w & MIRROR_PUB_MASK);
  out.iter = (int)((w >> 24) & 0xffffff);
  out.done = (int)((w >> 48) & 0xf);
  out.tol_hit = ((w >> 52) & 1) != 0;
  out.anchor_ok = ((w >> 53) & 1) != 0;
  out.repl = (int)((w >> 54) & 0x3ff);
  return out;
}

// Wait for a publication other than `after` (numbers wrap at 2^24, far more
// than one solve publishes between two reads).  Once no publication has come
// for QUERY_AFTER, the stream is queried (and again every QUERY_AFTER): an
// error ends the wait, and so does a drained stream with nothing new
// published (nothing more can come).  A stream query between kernel
// launches costs the device a few microseconds of idle time before the next
// launch, so during normal progress (one unit well under QUERY_AFTER, FP64
// true residuals of the largest images aside) the stream is never queried.
constexpr std::chrono::microseconds QUERY_AFTER{1000};

int wait_mirror(const Plan& P, hipStream_t s, unsigned after, Snap& out) {
  using clock = std::chrono::steady_clock;
  clock::time_point next_query = clock::now() + QUERY_AFTER;
  for (unsigned spins = 1;; ++spins) {
    out = read_mirror(P.mirror);
    if (out.pub != after) return KP_OK;
    if ((spins & 63u) == 0u && clock::now() >= next_query) {
      const hipError_t q = hipStreamQuery(s);
      if (q == hipSuccess) {
        out = read_mirror(P.mirror);
        return out.pub != after ? KP_OK : KP_ERR_HIP;
      }
      if (q != hipErrorNotReady) return KP_ERR_HIP;
      next_query = clock::now() + QUERY_AFTER;
    }
  }
}

}  // namespace

extern "C" {

size_t kp_workspace_size(int n, int k, int modes) {
  (void)modes;
  if (!valid_sizes(n, k)) return 0;
  return layout(n, k, nullptr, nullptr);
}

int kp_setup(const double* psf, int k, int n, int bc_flags, void* workspace, size_t ws_bytes,
             void* stream, kp_plan_t* plan) {
  const int bc = bc_flags & ~KP_SETUP_LOWP;
  if (plan == nullptr) return KP_ERR_ARG;
  *plan = nullptr;
  if (psf == nullptr || !valid_sizes(n, k)) {
    if (psf != nullptr && n >= 1 && k >= 1 && (k & 1) && k <= 2 * n - 1 && n > 2048)
      return KP_ERR_UNSUPPORTED;
    return KP_ERR_ARG;
  }
  if (bc != KP_BC_ZERO && bc != KP_BC_PERIODIC && bc != KP_BC_REFLEXIVE)
    return KP_ERR_UNSUPPORTED;
  if (k > KP_MAX_PSF) return KP_ERR_UNSUPPORTED;
  // periodic: the PSF would wrap onto itself; reflexive: one reflection
  // must cover every index
  if (bc != KP_BC_ZERO && k > n) return KP_ERR_ARG;
  bool refl_general = false;
  if (bc == KP_BC_REFLEXIVE) {
    // A^T = A (and the blur of A^T equals that of A) for PSFs symmetric in
    // both axes; for the others A^T is applied by the FFT form
    double mx = 0.0, asym = 0.0;
    for (int i = 0; i < k * k; ++i) mx = std::fmax(mx, std::fabs(psf[i]));
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) {
        asym = std::fmax(asym, std::fabs(psf[a * k + b] - psf[(k - 1 - a) * k + b]));
        asym = std::fmax(asym, std::fabs(psf[a * k + b] - psf[a * k + (k - 1 - b)]));
      }
    refl_general = asym > 1e-12 * mx;
    // such a plan's A^T exists only in the FFT form
    if (refl_general && fft_length_reflexive(n, k) <= 0) return KP_ERR_UNSUPPORTED;
  }
  for (int i = 0; i < k * k; ++i)
    if (!std::isfinite(psf[i])) return KP_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  kp_plan_s* h = new (std::nothrow) kp_plan_s();
  if (!h) return KP_ERR_ARG;
  Plan& P = h->P;
  P.n = n;
  P.k = k;
  P.bc = bc;
  P.lowp = (bc_flags & KP_SETUP_LOWP) != 0;
  P.refl_general = refl_general;
  P.kq = (k + TAP_CHUNK - 1) / TAP_CHUNK * TAP_CHUNK;
  const size_t need = layout(n, k, nullptr, nullptr);
  if (need == 0) {
    delete h;
    return KP_ERR_SOLVER;
  }
  char* base = nullptr;
  if (workspace != nullptr) {
    if (ws_bytes < need || !aligned16(workspace)) {
      delete h;
      return KP_ERR_WORKSPACE;
    }
    base = reinterpret_cast<char*>(workspace);
    P.owns = false;
  } else {
    if (hipMalloc(&base, need) != hipSuccess) {
      delete h;
      return KP_ERR_HIP;
    }
    P.owns = true;
  }
  P.base = base;
  P.bytes = need;
  char* scratch = nullptr;
  layout(n, k, base, &P, &scratch);
  if (bc == KP_BC_REFLEXIVE) {
    // the reflexive FFT form transforms the image extended by h per side
    P.fft_L = fft_length_reflexive(n, k);
    P.fft_nrad = P.fft_L > 0 ? fft_radices(P.fft_L, P.fft_rad) : 0;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&P.host_ctrl), 2 * sizeof(Ctrl)) != hipSuccess) {
    if (P.owns) hipFree(base);
    delete h;
    return KP_ERR_HIP;
  }
  std::memset(P.host_ctrl, 0, 2 * sizeof(Ctrl));
  if (hipHostMalloc(reinterpret_cast<void**>(&P.mirror), sizeof(CtrlMirror),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&P.mirror_dev), P.mirror, 0) !=
          hipSuccess) {
    if (P.mirror) hipHostFree(P.mirror);
    hipHostFree(P.host_ctrl);
    if (P.owns) hipFree(base);
    delete h;
    return KP_ERR_HIP;
  }
  std::memset(P.mirror, 0, sizeof(CtrlMirror));
  int rc = KP_OK;
  if (hipMemsetAsync(P.ctrl, 0, sizeof(Ctrl), s) != hipSuccess) rc = KP_ERR_HIP;
  if (rc == KP_OK && hipEventCreateWithFlags(&P.ev_last, hipEventDisableTiming) != hipSuccess)
    rc = KP_ERR_HIP;
  if (rc == KP_OK) rc = build_factors(P, psf, scratch, s);
  if (rc == KP_OK && autotune_blur(P, s, P.blur_times) != hipSuccess) rc = KP_ERR_HIP;
  if (rc == KP_OK && autotune_normal(P, s) != hipSuccess) rc = KP_ERR_HIP;
  if (rc == KP_OK && hipEventRecord(P.ev_last, s) != hipSuccess) rc = KP_ERR_HIP;
  if (rc == KP_OK && hipStreamSynchronize(s) != hipSuccess) rc = KP_ERR_HIP;
  if (rc != KP_OK) {
    hipStreamSynchronize(s);
    if (P.ev_last) hipEventDestroy(P.ev_last);
    hipHostFree(P.mirror);
    hipHostFree(P.host_ctrl);
    if (P.owns) hipFree(base);
    delete h;
    return rc;
  }
  *plan = h;
  return KP_OK;
}

int kp_plan_query(kp_plan_t plan, kp_plan_info_t* out) {
  if (!plan || !out) return KP_ERR_ARG;
  const Plan& P = plan->P;
  out->n = P.n;
  out->k = P.k;
  out->kron_terms = P.terms;
  out->normal_op = P.normal_op;
  out->kp_rel_error = P.kp_err;
  out->sigma_c_max = P.sc_max;
  out->sigma_c_min = P.sc_min;
  out->sigma_r_max = P.sr_max;
  out->sigma_r_min = P.sr_min;
  out->device_bytes = P.bytes;
  out->blur_config = P.blur_cfg;
  for (int i = 0; i < 8; ++i) out->blur_config_ms[i] = P.blur_times[i];
  out->fft_length = P.fft_L > 0 ? P.fft_L : 0;
  out->normal_op_ms[0] = P.normal_times[0];
  out->normal_op_ms[1] = P.normal_times[1];
  return KP_OK;
}

int kp_destroy(kp_plan_t plan) {
  if (!plan) return KP_ERR_ARG;
  Plan& P = plan->P;
  // the plan's last enqueued work (recorded on the stream it ran on) must
  // finish before its memory goes; other streams are left alone
  if (P.ev_last) hipEventSynchronize(P.ev_last);
  if (P.ev_last) hipEventDestroy(P.ev_last);
  if (P.mirror) hipHostFree(P.mirror);
  if (P.host_ctrl) hipHostFree(P.host_ctrl);
  if (P.ev_start) hipEventDestroy(P.ev_start);
  if (P.ev_end) hipEventDestroy(P.ev_end);
  if (P.owns && P.base) hipFree(P.base);
  delete plan;
  return KP_OK;
}

const char* kp_strerror(int status) {
  switch (status) {
    case KP_OK: return "success (solve: true relative residual <= tol)";
    case KP_MAXIT: return "maximum number of iterations reached";
    case KP_BREAKDOWN: return "breakdown: non-positive curvature or non-finite scalar";
    case KP_OK_FALLBACK:
      return "success after restarting with the FP32 preconditioner";
    case KP_ERR_ARG: return "invalid argument";
    case KP_ERR_UNSUPPORTED: return "unsupported configuration";
    case KP_ERR_HIP: return "HIP runtime error";
    case KP_ERR_SOLVER: return "FP64 factor SVD failed";
    case KP_ERR_WORKSPACE: return "workspace too small or misaligned";
    default: return "unknown status";
  }
}

}  // extern "C"

namespace {

int solve_once(kp_plan_t plan, const float* b, double lambda, double tol, int maxit, int mode,
               float* x, kp_info_t* info, void* stream) {
  const int solver = mode & KP_SOLVER_MASK;
  const int prec = mode & KP_PREC_MASK;
  if (solver == 3 || prec == KP_PREC_MASK) return KP_ERR_ARG;
  if (!aligned16(b) || !aligned16(x)) return KP_ERR_ARG;
  if (solver != KP_CG && prec == KP_P8 && !fp8_supported_size(plan->P.n))
    return KP_ERR_UNSUPPORTED;
  Plan& P = plan->P;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t N = (size_t)P.n * P.n;
  P.sprime_d0 = (mode & KP_EXACT_DIAG) ? P.d0 : nullptr;
  const double lam2d = lambda * lambda;
  const float lam2 = (float)lam2d;

  Ctrl c;
  std::memset(&c, 0, sizeof(c));
  c.tol_rel2 = tol * tol;
  c.lam2 = lam2d;
  c.maxit = maxit;
  c.solver = solver;
  c.prec = prec;
  c.first = 1;
  c.done = RUNNING;
  c.pscale = 1.0f;
  c.zscale = (float)(1.0 / lam2d);
  const bool hist = (mode & KP_HIST) != 0;
  c.hist = hist ? P.hist : nullptr;
  P.hist_count = 0;
  // nothing of this plan may still be publishing when the mirror is reset
  // (a no-op wait when the stream is idle, as after the previous solve)
  HIPCHK(hipStreamSynchronize(s));
  std::memset(P.mirror, 0, sizeof(CtrlMirror));
  if (hist) HIPCHK(launch_fill_f64(P.hist, 2 * KP_HIST_MAX, std::nan(""), s));
  int rc = write_ctrl(P, s, c);
  if (rc != KP_OK) return rc;
  if (mode & KP_WARM) HIPCHK(launch_convert_x(P, x, false, s));

  int replacements = 0;
  // A true residual is A^T (b - A x) - lambda^2 x.  u = b - A x is formed on
  // the fast blur for loose tolerances (TR_FASTU_TOL_*), else in FP64; A^T u
  // on the fast blur from TR_FAST_TOL on, else in FP64.
  // After one at x_a (residual r_a), later ones are computed as
  // r_a - H (x - x_a) with FP32 matvecs on the small step x - x_a: exact in
  // exact arithmetic, with an error of up to ~1e-5 ||r_a||.  Used once
  // ||r_a|| <= min(ANCHOR_REL, ANCHOR_TOL tol) ||A^T b||, so the error stays
  // below a tenth of the tolerance.
  const int trmode =
      tol >= (blur_cfg_is_mfma(P.blur_cfg) ? TR_FASTU_TOL_MFMA : TR_FASTU_TOL_VALU) ? TR_FAST_ALL
      : tol >= TR_FAST_TOL                                                        ? TR_FAST_AT
                                                                                  : TR_FP64;
  bool anchor_ok = false;        // the last true residual may anchor the next
  auto true_residual = [&](bool fin) -> hipError_t {
    if (anchor_ok) return launch_anchor_residual(P, lam2d, fin, s);
    return launch_true_residual(P, b, P.x64, lam2d, fin, trmode, s);
  };

  // The host follows the device through the word the scalar steps publish,
  // and keeps at most LOOKAHEAD publications enqueued beyond the last one it
  // has read.  For PCG and FPCG an iteration is the matvec half (A p, A^T q,
  // step, update) and the tail (preconditioner, whose first GEMM takes the
  // update's residual-norm step and publishes ||r||; direction: publishes
  // r.z); the matvec half of the last iteration, which no tail follows,
  // launches its own residual-norm step.  With dir_in_matvec the direction
  // step (and its r.z) moves into the next matvec half: every matvec half
  // follows a tail.  For CG an iteration publishes once (||r||).  Kernels
  // enqueued after the device has marked the solve PENDING or finished exit
  // at once and publish nothing.
  // With the direction step in the first FFT pass the two publications of
  // an iteration come at the start of each half, so one publication ahead
  // is half an iteration of queued work (~50 us at 1024^2), more than the
  // host needs to react; two kept up to ten kernels queued beyond a
  // publication that marks the solve PENDING, all of which then ran as
  // no-ops before the true residual (seeds 0-7 of the large workload:
  // 1.147-1.169 ms median with one, 1.177-1.185 ms with two, 1.179-1.186 ms
  // with three, same box).  Otherwise a publication ends a unit (CG's
  // residual-norm step, the direction update), and with one ahead the queue
  // would run dry at every publication: two.
  const bool dir = dir_in_matvec(P, solver);
  const unsigned LOOKAHEAD = dir ? 1u : 2u;
  Snap m{};
  unsigned seen = 0;             // the last publication read (mod 2^24)
  unsigned enq = 0;              // publications enqueued, if every unit runs
  auto inflight = [&]() { return (enq - seen) & MIRROR_PUB_MASK; };
  auto bump = [&]() { enq = (enq + 1u) & MIRROR_PUB_MASK; };
  int its = 0;                   // iterations enqueued (matvec halves)
  bool mv_next = true;           // the next unit is a matvec half
  bool fold_next = false;        // the next tail folds in the update's ||r|| step
  HIPCHK(launch_rhs(P, b, !(mode & KP_WARM), s));   // r = c = A^T b, ||c||; p = w (= x) = 0
  bump();
  if (mode & KP_WARM) {
    HIPCHK(launch_true_residual(P, b, P.x64, lam2d, true, trmode, s));    // r = c - H x0
    bump();
    ++replacements;
  }
  // first direction p = z_0 (CG: p = r_0)
  HIPCHK(enqueue_tail(P, solver, prec, lam2, s));
  if (solver != KP_CG && !dir) bump();
  auto top_up = [&]() -> hipError_t {
    while (inflight() < LOOKAHEAD && its < maxit) {
      hipError_t e;
      if (solver == KP_CG) {
        e = enqueue_iteration(P, solver, prec, lam2, s);
        ++its;
        bump();
      } else if (mv_next) {
        const bool last = its + 1 >= maxit;      // no tail will follow
        e = enqueue_matvec_half(P, solver, prec, lam2, s, last);
        ++its;
        mv_next = false;
        fold_next = !last;
        if (dir) bump();
        if (last) bump();
      } else {
        e = enqueue_tail(P, solver, prec, lam2, s, fold_next ? update_partials(P) : 0);
        if (fold_next) bump();
        if (!dir) bump();
        mv_next = true;
        fold_next = false;
      }
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  auto next = [&]() -> int {
    const int rc2 = wait_mirror(P, s, seen, m);
    if (rc2 != KP_OK) return rc2;
    seen = m.pub;
    anchor_ok = m.anchor_ok;
    return KP_OK;
  };

  int state = RUNNING;
  bool x_out = false;            // x holds the FP32 copy of the last true residual's x
  HIPCHK(top_up());
  if ((rc = next()) != KP_OK) return rc;
  for (;;) {
    if (m.done == PENDING) {
      // the recurrence residual met the tolerance or fell 1/REPLACE_DROP:
      // recompute it from b and x and continue from the true residual.
      // Everything enqueued after that publication was skipped.
      its = m.iter;
      HIPCHK(true_residual(true));
      ++replacements;
      enq = seen;
      bump();
      // a true residual that may end the solve: x in FP32 at once, so that
      // a converged solve needs no further launch (a solve that goes on
      // overwrites x later)
      x_out = m.tol_hit || its >= maxit;
      if (x_out) HIPCHK(launch_convert_x(P, x, true, s));
      if (m.tol_hit || its >= maxit) {
        // may have converged (or no budget left): see the outcome first
        if ((rc = next()) != KP_OK) return rc;
        if (m.done != RUNNING) { state = m.done; break; }
        if (its >= maxit) { state = MAXIT; break; }
      }
      // then the direction from the new residual: CG's p = r + beta p
      // (publishes nothing), else the preconditioner half as the next unit
      if (solver == KP_CG) HIPCHK(enqueue_tail(P, solver, prec, lam2, s));
      else mv_next = false;
      fold_next = false;                  // the true residual set ||r|| and the scales
    } else if (m.done != RUNNING) {
      state = m.done;
      break;
    } else if (m.iter >= maxit && inflight() == 0) {
      state = MAXIT;
      break;
    }
    HIPCHK(top_up());
    if ((rc = next()) != KP_OK) return rc;
  }

  // an unconverged solve reports its true residual; then x in FP32 (x_0 = 0
  // stays 0 for zero or non-finite data)
  if (state != CONVERGED) HIPCHK(true_residual(false));
  if (state != CONVERGED || !x_out) HIPCHK(launch_convert_x(P, x, true, s));
  HIPCHK(hipEventRecord(P.ev_end, s));
  HIPCHK(hipStreamSynchronize(s));
  const volatile CtrlMirror* fm = P.mirror;       // complete: the stream has drained
  const double gamma0sq = fm->gamma0sq, true_rr = fm->true_rr, rr = fm->rr, tol2 = fm->tol2;
  const int iters = fm->iter;
  if (hist && gamma0sq > 0.0 && std::isfinite(gamma0sq)) {
    P.hist_count = iters + 1 < KP_HIST_MAX ? iters + 1 : KP_HIST_MAX;
    P.hist_gamma0sq = gamma0sq;
  }
  if (!(gamma0sq > 0.0) || !std::isfinite(gamma0sq)) {
    // zero data: x = 0 is the solution; non-finite data: nothing to do
    const bool zero = gamma0sq == 0.0;
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = zero ? KP_OK : KP_BREAKDOWN;
      info->lambda = lambda;
    }
    return zero ? KP_OK : KP_BREAKDOWN;
  }
  int status;
  if (state == CONVERGED) status = KP_OK;
  else if (state == BREAKDOWN) status = KP_BREAKDOWN;
  else status = (true_rr <= tol2) ? KP_OK : KP_MAXIT;
  if (info) {
    info->iters = iters;
    info->status = status;
    info->replacements = replacements;
    info->fallback = 0;
    info->relres_rec = std::sqrt(rr / gamma0sq);
    info->relres_true = std::sqrt(true_rr / gamma0sq);
    info->lambda = lambda;
    info->rhs_norm = std::sqrt(gamma0sq);
    info->misfit = 0.0;
  }
  return status;
}

}  // namespace

extern "C" {

int pcg_solve(kp_plan_t plan, const float* b, double lambda, double tol, int maxit, int mode,
              float* x, kp_info_t* info, void* stream) {
  if (!plan || !b || !x) return KP_ERR_ARG;
  if (!(lambda > 0.0) || !std::isfinite(lambda) || !(tol > 0.0) || !std::isfinite(tol) ||
      maxit < 1)
    return KP_ERR_ARG;
  if ((mode & ~(KP_SOLVER_MASK | KP_PREC_MASK | KP_WARM | KP_NO_FALLBACK | KP_EXACT_DIAG |
                KP_HIST)) != 0)
    return KP_ERR_ARG;
  Plan& P = plan->P;
  // with a PSF that is not symmetric under the reflexive boundary, A^T runs
  // by FFTs in FP32 only: no FP64 true residual for the tightest tolerances
  if (P.refl_general && tol < TR_FAST_TOL) return KP_ERR_UNSUPPORTED;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!P.ev_start) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return KP_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
      hipEventDestroy(e0);
      return KP_ERR_HIP;
    }
    P.ev_start = e0;
    P.ev_end = e1;
  }
  HIPCHK(hipEventRecord(P.ev_start, s));
  // device time from the start event to the end event of the last run
  // (solve_once records the end event before its closing synchronisation)
  auto elapsed = [&]() -> float {
    float ms = 0.0f;
    return hipEventElapsedTime(&ms, P.ev_start, P.ev_end) == hipSuccess ? ms : 0.0f;
  };
  kp_info_t first{};
  const int st = solve_once(plan, b, lambda, tol, maxit, mode & ~KP_NO_FALLBACK, x, &first,
                            stream);
  HIPCHK(hipEventRecord(P.ev_last, s));
  if (st < 0) return st;
  first.ms = elapsed();
  const int solver = mode & KP_SOLVER_MASK, prec = mode & KP_PREC_MASK;
  const bool retry = (st == KP_MAXIT || st == KP_BREAKDOWN) && solver != KP_CG &&
                     prec != KP_P32 && !(mode & KP_NO_FALLBACK) &&
                     std::isfinite(first.relres_true);
  if (!retry) {
    if (info) *info = first;
    return st;
  }
  // reduced-precision preconditioner did not reach tol: restart from the last
  // iterate with the FP32 preconditioner (its own budget of maxit iterations)
  kp_info_t second{};
  const int st2 = solve_once(plan, b, lambda, tol, maxit,
                             (mode & (KP_SOLVER_MASK | KP_NO_FALLBACK | KP_EXACT_DIAG | KP_HIST)) |
                                 KP_P32 | KP_WARM,
                             x,
                             &second, stream);
  HIPCHK(hipEventRecord(P.ev_last, s));
  if (st2 < 0) return st2;
  if (info) {
    *info = second;
    info->iters = first.iters + second.iters;
    info->replacements = first.replacements + second.replacements;
    info->fallback = 1;
    info->status = st2 == KP_OK ? KP_OK_FALLBACK : st2;
    info->ms = elapsed();
  }
  return st2 == KP_OK ? KP_OK_FALLBACK : st2;
}

int kp_get_history(kp_plan_t plan, double* relres_rec, double* relres_true, int cap, int* count,
                   void* stream) {
  if (!plan || !count || cap < 0) return KP_ERR_ARG;
  Plan& P = plan->P;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  *count = P.hist_count;
  const int m = cap < P.hist_count ? cap : P.hist_count;
  if (m == 0 || (!relres_rec && !relres_true)) return KP_OK;
  std::vector<double> h(2 * (size_t)m);
  HIPCHK(hipMemcpyAsync(h.data(), P.hist, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(h.data() + m, P.hist + KP_HIST_MAX, sizeof(double) * m,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < m; ++k) {
    if (relres_rec) relres_rec[k] = std::sqrt(h[k] / P.hist_gamma0sq);
    if (relres_true) relres_true[k] = std::sqrt(h[m + k] / P.hist_gamma0sq);
  }
  return KP_OK;
}

// argument checks shared by pcg_solve_batched and its workspace query
static int batched_args(const kp_plan_t* plans, int nplans, const int* plan_of_item, int nitems,
                        int mode, std::vector<Plan*>& ps) {
  if (!plans || nplans < 1 || !plan_of_item || nitems < 1) return KP_ERR_ARG;
  if ((mode & ~(KP_SOLVER_MASK | KP_PREC_MASK | KP_WARM | KP_BATCH_EAGER | KP_EXACT_DIAG)) != 0)
    return KP_ERR_ARG;
  if ((mode & KP_SOLVER_MASK) == 3 || (mode & KP_PREC_MASK) == KP_PREC_MASK) return KP_ERR_ARG;
  ps.resize(nplans);
  for (int i = 0; i < nplans; ++i) {
    if (!plans[i]) return KP_ERR_ARG;
    ps[i] = &plans[i]->P;
  }
  // the batched matvecs are direct blurs: A^T must be one
  for (int i = 0; i < nplans; ++i)
    if (ps[i]->refl_general) return KP_ERR_UNSUPPORTED;
  for (int i = 0; i < nitems; ++i)
    if (plan_of_item[i] < 0 || plan_of_item[i] >= nplans) return KP_ERR_ARG;
  return KP_OK;
}

size_t pcg_solve_batched_workspace_size(const kp_plan_t* plans, int nplans,
                                        const int* plan_of_item, int nitems, int mode) {
  std::vector<Plan*> ps;
  if (batched_args(plans, nplans, plan_of_item, nitems, mode, ps) != KP_OK) return 0;
  size_t need = 0;
  if (batched_solve(ps.data(), plan_of_item, nitems, mode, 0.0, 0, nullptr, nullptr, nullptr,
                    nullptr, nullptr, 0, &need, nullptr) != KP_OK)
    return 0;
  return need;
}

int pcg_solve_batched(const kp_plan_t* plans, int nplans, const float* const* b,
                      const double* lambdas, const int* plan_of_item, int nitems, double tol,
                      int maxit, int mode, float* const* x, kp_info_t* infos, void* workspace,
                      size_t ws_bytes, void* stream) {
  std::vector<Plan*> ps;
  int rc = batched_args(plans, nplans, plan_of_item, nitems, mode, ps);
  if (rc != KP_OK) return rc;
  {
    // the sizing pass refuses unsupported item shapes before anything else
    size_t need = 0;
    rc = batched_solve(ps.data(), plan_of_item, nitems, mode, 0.0, 0, nullptr, nullptr, nullptr,
                       nullptr, nullptr, 0, &need, nullptr);
    if (rc != KP_OK) return rc;
  }
  if (!b || !lambdas || !x || !infos || !workspace) return KP_ERR_ARG;
  if (!(tol > 0.0) || !std::isfinite(tol) || maxit < 1) return KP_ERR_ARG;
  for (int i = 0; i < nitems; ++i) {
    if (!b[i] || !x[i] || !aligned16(b[i]) || !aligned16(x[i])) return KP_ERR_ARG;
    if (!(lambdas[i] > 0.0) || !std::isfinite(lambdas[i])) return KP_ERR_ARG;
  }
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return KP_ERR_WORKSPACE;
  // every plan's own solve state must be idle: the batch only reads factors
  rc = batched_solve(ps.data(), plan_of_item, nitems, mode, tol, maxit, b, lambdas, x, infos,
                     workspace, ws_bytes, nullptr, reinterpret_cast<hipStream_t>(stream));
  if (rc != KP_OK) return rc;
  int worst = KP_OK;
  for (int i = 0; i < nitems; ++i)
    if (infos[i].status > worst) worst = infos[i].status;
  return worst;
}

}  // extern "C"

namespace kpcg {

hipStream_t aux_stream(int slot) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, hipStream_t> streams;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(dev, slot);
  auto it = streams.find(key);
  if (it != streams.end()) return it->second;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
  streams[key] = st;
  return st;
}

int spectral_call(kp_plan_t plan, const float* b, const double* grid, int ngrid, double omega,
                  double noise2, int kind, double* scores_host, void* stream,
                  const float* x_true) {
  Plan& P = plan->P;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t N = (size_t)P.n * P.n;
  char* spec = reinterpret_cast<char*>(P.spec);
  double* grid_dev = reinterpret_cast<double*>(spec + ((N * sizeof(float) + 255) / 256) * 256);
  double* out_dev = grid_dev + 64;
  float* xhat = nullptr;
  HIPCHK(hipMemcpyAsync(grid_dev, grid, sizeof(double) * ngrid, hipMemcpyHostToDevice, s));
  if (kind == 2) {
    xhat = reinterpret_cast<float*>(P.t2);
    HIPCHK(launch_vbasis_gemms(P, x_true, xhat, s));
  }
  HIPCHK(launch_spectrum(P, b, s));
  HIPCHK(launch_spectral_scores(P, grid_dev, ngrid, omega, noise2, kind, out_dev, s, xhat));
  HIPCHK(hipMemcpyAsync(scores_host, out_dev, sizeof(double) * ngrid, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return KP_OK;
}

bool valid_grid(const double* grid, int ngrid, int max_points) {
  if (!grid || ngrid < 1 || ngrid > max_points) return false;
  for (int g = 0; g < ngrid; ++g)
    if (!(grid[g] > 0.0) || !std::isfinite(grid[g])) return false;
  return true;
}

}  // namespace kpcg

extern "C" {

int gcv_lambda(kp_plan_t plan, const float* b, const double* grid, int ngrid, double omega,
               double* lambda_out, double* scores_out, void* stream) {
  if (!plan || !b || !lambda_out || !valid_grid(grid, ngrid) || !std::isfinite(omega))
    return KP_ERR_ARG;
  if (!aligned16(b)) return KP_ERR_ARG;
  double sc[64];
  int rc = spectral_call(plan, b, grid, ngrid, omega, 0.0, 0, sc, stream);
  if (rc != KP_OK) return rc;
  int best = 0;
  for (int g = 1; g < ngrid; ++g)
    if (sc[g] < sc[best]) best = g;
  *lambda_out = grid[best];
  if (scores_out) std::memcpy(scores_out, sc, sizeof(double) * ngrid);
  return KP_OK;
}

int discrepancy_lambda(kp_plan_t plan, const float* b, const double* grid, int ngrid,
                       double noise_norm, double eta, double* lambda_out, double* values_out,
                       void* stream) {
  if (!plan || !b || !lambda_out || !valid_grid(grid, ngrid) || !(noise_norm >= 0.0) ||
      !(eta > 0.0) || !std::isfinite(noise_norm * eta))
    return KP_ERR_ARG;
  if (!aligned16(b)) return KP_ERR_ARG;
  double d[64];
  const double eps = eta * noise_norm;
  int rc = spectral_call(plan, b, grid, ngrid, 1.0, eps * eps, 1, d, stream);
  if (rc != KP_OK) return rc;
  int pick = -1;
  for (int g = 0; g < ngrid; ++g)
    if (d[g] <= 0.0) pick = g;
  *lambda_out = grid[pick < 0 ? 0 : pick];
  if (values_out) std::memcpy(values_out, d, sizeof(double) * ngrid);
  return KP_OK;
}

int kp_blur(kp_plan_t plan, const float* x, float* y, int transpose, void* stream) {
  if (!plan || !x || !y || x == y) return KP_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(launch_blur_f32(plan->P, x, y, transpose != 0, s, nullptr));
  HIPCHK(hipEventRecord(plan->P.ev_last, s));
  HIPCHK(hipStreamSynchronize(s));
  return KP_OK;
}

int kp_normal_fp64(kp_plan_t plan, const float* x, double lambda, double* y, void* stream) {
  if (!plan || !x || !y || !(lambda >= 0.0) || !std::isfinite(lambda)) return KP_ERR_ARG;
  if (plan->P.refl_general) return KP_ERR_UNSUPPORTED;     // its A^T is no FP64 blur
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(launch_normal_fp64(plan->P, x, lambda * lambda, y, s));
  HIPCHK(hipEventRecord(plan->P.ev_last, s));
  HIPCHK(hipStreamSynchronize(s));
  return KP_OK;
}

int kp_precond(kp_plan_t plan, const float* r, double lambda, int mode, float* z,
               void* stream) {
  if (!plan || !r || !z || r == z || !(lambda > 0.0) || !std::isfinite(lambda))
    return KP_ERR_ARG;
  const int prec = mode & KP_PREC_MASK;
  if (prec == KP_PREC_MASK) return KP_ERR_ARG;
  if (prec == KP_P8 && !fp8_supported_size(plan->P.n)) return KP_ERR_UNSUPPORTED;
  if (!aligned16(r) || !aligned16(z)) return KP_ERR_ARG;
  Plan& P = plan->P;
  P.sprime_d0 = (mode & KP_EXACT_DIAG) ? P.d0 : nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Ctrl c;
  std::memset(&c, 0, sizeof(c));
  c.lam2 = lambda * lambda;
  c.prec = prec;
  c.done = RUNNING;
  int rc = write_ctrl(P, s, c);
  if (rc != KP_OK) return rc;
  HIPCHK(launch_norm_scale(P, r, s));
  HIPCHK(launch_precond(P, r, z, nullptr, prec, false, (float)(lambda * lambda), s));
  HIPCHK(hipStreamSynchronize(s));
  return KP_OK;
}

int kp_time_blur(kp_plan_t plan, const float* x, float* y, int transpose, int reps,
                 float* avg_ms, void* stream) {
  if (!plan || !x || !y || x == y || reps < 1 || !avg_ms) return KP_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int rc = KP_OK;
  if (hipEventRecord(e0, s) != hipSuccess) rc = KP_ERR_HIP;
  for (int i = 0; i < reps && rc == KP_OK; ++i)
    if (launch_blur_f32(plan->P, x, y, transpose != 0, s, nullptr) != hipSuccess)
      rc = KP_ERR_HIP;
  if (rc == KP_OK && hipEventRecord(e1, s) != hipSuccess) rc = KP_ERR_HIP;
  if (rc == KP_OK && hipEventSynchronize(e1) != hipSuccess) rc = KP_ERR_HIP;
  float ms = 0.f;
  if (rc == KP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = KP_ERR_HIP;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *avg_ms = ms / reps;
  return rc;
}

int kp_time_precond(kp_plan_t plan, const float* r, double lambda, int mode, float* z,
                    int reps, float* avg_ms, void* stream) {
  if (!plan || !r || !z || r == z || reps < 1 || !avg_ms || !(lambda > 0.0)) return KP_ERR_ARG;
  const int prec = mode & KP_PREC_MASK;
  if (prec == KP_PREC_MASK) return KP_ERR_ARG;
  if (prec == KP_P8 && !fp8_supported_size(plan->P.n)) return KP_ERR_UNSUPPORTED;
  Plan& P = plan->P;
  P.sprime_d0 = (mode & KP_EXACT_DIAG) ? P.d0 : nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Ctrl c;
  std::memset(&c, 0, sizeof(c));
  c.lam2 = lambda * lambda;
  c.prec = prec;
  c.done = RUNNING;
  int rc = write_ctrl(P, s, c);
  if (rc != KP_OK) return rc;
  HIPCHK(launch_norm_scale(P, r, s));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  if (hipEventRecord(e0, s) != hipSuccess) rc = KP_ERR_HIP;
  for (int i = 0; i < reps && rc == KP_OK; ++i)
    if (launch_precond(P, r, z, nullptr, prec, false, (float)(lambda * lambda), s) != hipSuccess)
      rc = KP_ERR_HIP;
  if (rc == KP_OK && hipEventRecord(e1, s) != hipSuccess) rc = KP_ERR_HIP;
  if (rc == KP_OK && hipEventSynchronize(e1) != hipSuccess) rc = KP_ERR_HIP;
  float ms = 0.f;
  if (rc == KP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = KP_ERR_HIP;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *avg_ms = ms / reps;
  return rc;
}

int kp_set_blur_config(kp_plan_t plan, int cfg, int* prev) {
  if (!plan || cfg < 0 || cfg > BLUR_CFG_MFMA32) return KP_ERR_ARG;
  if (prev) *prev = plan->P.blur_cfg;
  plan->P.blur_cfg = cfg;
  return KP_OK;
}

// The factors and D0 are final once kp_setup has returned (it synchronises
// its stream), so the getters wait for nothing else: they copy on the
// device's auxiliary stream (non-blocking, so the copies neither wait for
// nor hold up other streams) and wait for those copies only.
// The forms of H p a plan can use: the FFT form for the zero and reflexive
// boundaries; the direct blurs unless A^T is not a blur (refl_general).
static bool normal_op_valid(const Plan& P, int op) {
  if (op == KP_NORMAL_FFT) return P.fft_L > 0 && (P.bc == KP_BC_ZERO || P.bc == KP_BC_REFLEXIVE);
  return !P.refl_general;
}

int kp_set_normal_op(kp_plan_t plan, int op, int* prev) {
  if (!plan || (op != KP_NORMAL_DIRECT && op != KP_NORMAL_FFT)) return KP_ERR_ARG;
  if (!normal_op_valid(plan->P, op)) return KP_ERR_UNSUPPORTED;
  if (prev) *prev = plan->P.normal_op;
  plan->P.normal_op = op;
  return KP_OK;
}

static hipError_t normal_op_launch(Plan& P, const float* x, float* y, float lam2, int op,
                                   hipStream_t s) {
  int nb;
  return op == KP_NORMAL_FFT ? launch_fft_normal(P, x, y, lam2, s, &nb, nullptr)
                             : launch_normal_direct(P, x, y, lam2, s, &nb);
}

static bool valid_normal_op(int op) {
  return op == KP_NORMAL_PLAN || op == KP_NORMAL_DIRECT || op == KP_NORMAL_FFT;
}

int kp_normal(kp_plan_t plan, const float* x, double lambda, float* y, int op, void* stream) {
  if (!plan || !x || !y || x == y || !(lambda >= 0.0) || !std::isfinite(lambda) ||
      !valid_normal_op(op))
    return KP_ERR_ARG;
  Plan& P = plan->P;
  if (x == P.q || y == P.q) return KP_ERR_ARG;
  if (!normal_op_valid(P, op == KP_NORMAL_PLAN ? P.normal_op : op)) return KP_ERR_UNSUPPORTED;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(normal_op_launch(P, x, y, (float)(lambda * lambda),
                          op == KP_NORMAL_PLAN ? P.normal_op : op, s));
  HIPCHK(hipEventRecord(P.ev_last, s));
  HIPCHK(hipStreamSynchronize(s));
  return KP_OK;
}

int kp_time_normal(kp_plan_t plan, const float* x, float* y, int op, int reps, float* avg_ms,
                   void* stream) {
  if (!plan || !x || !y || x == y || reps < 1 || !avg_ms || !valid_normal_op(op))
    return KP_ERR_ARG;
  Plan& P = plan->P;
  const int which = op == KP_NORMAL_PLAN ? P.normal_op : op;
  if (!normal_op_valid(P, which)) return KP_ERR_UNSUPPORTED;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return KP_ERR_HIP;
  }
  int rc = KP_OK;
  if (hipEventRecord(e0, s) != hipSuccess) rc = KP_ERR_HIP;
  for (int i = 0; i < reps && rc == KP_OK; ++i)
    if (normal_op_launch(P, x, y, 1e-4f, which, s) != hipSuccess) rc = KP_ERR_HIP;
  if (rc == KP_OK && hipEventRecord(e1, s) != hipSuccess) rc = KP_ERR_HIP;
  if (rc == KP_OK && hipEventSynchronize(e1) != hipSuccess) rc = KP_ERR_HIP;
  float ms = 0.f;
  if (rc == KP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = KP_ERR_HIP;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *avg_ms = ms / reps;
  return rc;
}

int kp_get_diag(kp_plan_t plan, float* d0) {
  if (!plan || !d0) return KP_ERR_ARG;
  Plan& P = plan->P;
  hipStream_t a = aux_stream(AUX_COPY);
  if (!a) return KP_ERR_HIP;
  HIPCHK(hipMemcpyAsync(d0, P.d0, sizeof(float) * P.n * P.n, hipMemcpyDeviceToHost, a));
  HIPCHK(hipStreamSynchronize(a));
  return KP_OK;
}

int kp_get_factors(kp_plan_t plan, double* sc, double* sr, double* vc, double* vr) {
  if (!plan || !sc || !sr) return KP_ERR_ARG;
  Plan& P = plan->P;
  const int n = P.n;
  hipStream_t a = aux_stream(AUX_COPY);
  if (!a) return KP_ERR_HIP;
  HIPCHK(hipMemcpyAsync(sc, P.sc, sizeof(double) * n, hipMemcpyDeviceToHost, a));
  HIPCHK(hipMemcpyAsync(sr, P.sr, sizeof(double) * n, hipMemcpyDeviceToHost, a));
  HIPCHK(hipStreamSynchronize(a));
  if (vc || vr) {
    const size_t nn = (size_t)n * n;
    float* tmp = new (std::nothrow) float[nn];
    if (!tmp) return KP_ERR_ARG;
    int rc = KP_OK;
    if (vc) {
      if (hipMemcpyAsync(tmp, P.Vc32, sizeof(float) * nn, hipMemcpyDeviceToHost, a) !=
              hipSuccess || hipStreamSynchronize(a) != hipSuccess)
        rc = KP_ERR_HIP;
      else
        for (size_t i = 0; i < nn; ++i) vc[i] = tmp[i];
    }
    if (vr && rc == KP_OK) {
      if (hipMemcpyAsync(tmp, P.Vr32, sizeof(float) * nn, hipMemcpyDeviceToHost, a) !=
              hipSuccess || hipStreamSynchronize(a) != hipSuccess)
        rc = KP_ERR_HIP;
      else
        for (size_t i = 0; i < nn; ++i) vr[i] = tmp[i];
    }
    delete[] tmp;
    return rc;
  }
  return KP_OK;
}

}  // extern "C"
