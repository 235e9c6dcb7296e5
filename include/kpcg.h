/*
 * kpcg.h -- C ABI of the MI355X (gfx950) library for Tikhonov image
 * deblurring with CG, PCG and flexible PCG preconditioned by a one-term
 * Kronecker-product SVD approximation of the blur.
 *
 * Method: Chen, Ji & Nagy, "Half-Precision Kronecker Product SVD
 * Preconditioner for Structured Inverse Problems" (arXiv:2311.15393).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - An image is an n x n float32 array, row-major and contiguous (element
 *    (i, j) at i*n + j; i is the vertical index).  Images passed as `const
 *    float *` / `float *` are DEVICE pointers owned by the caller.
 *  - A PSF is a K x K float64 HOST array, row-major, K odd, centre (h, h),
 *    h = (K-1)/2.  The library normalises nothing.  The blur A is the
 *    zero-boundary true convolution
 *        (A X)[i, j] = sum_{u,v=-h..h} P[h+u, h+v] X[i-u, j-v],
 *    and A^T is the matching correlation (the paper does not state its
 *    boundary condition or PSF centre; this is the reading taken).
 *  - `stream` is a hipStream_t (NULL = default stream).  All device work is
 *    enqueued on it.  Entry points that return scalars synchronise it.
 *  - Every function returns an int status (0 = success / converged, > 0 a
 *    solver outcome, < 0 an error; see KP_ERR_*), never throws, and leaves
 *    no HIP error pending on success.
 *  - A plan is not thread safe: use one plan per host thread / stream.
 */
#ifndef KPCG_H
#define KPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define KP_OK               0   /* success; for solves: converged, the TRUE
                                   relative residual (FP64) is <= tol      */
#define KP_MAXIT            1   /* maxit iterations without convergence    */
#define KP_BREAKDOWN        2   /* p.Hp <= 0, r.z <= 0 or a non-finite
                                   scalar; x holds the last iterate        */
#define KP_OK_FALLBACK      3   /* converged after the automatic restart
                                   with the FP32 preconditioner (pcg_solve
                                   with KP_P16 / KP_P8 only)               */
#define KP_ERR_ARG         -1   /* null pointer, n < 1, K even, K > 2n-1,
                                   lambda <= 0, tol <= 0, maxit < 1, a
                                   non-finite argument, bad mode bits      */
#define KP_ERR_UNSUPPORTED -2   /* unknown boundary condition, K above
                                   KP_MAX_PSF, or a call the plan's
                                   operator cannot serve (see
                                   KP_BC_REFLEXIVE)                        */
#define KP_ERR_HIP         -3   /* a HIP runtime call failed               */
#define KP_ERR_WORKSPACE   -4   /* caller workspace smaller than required,
                                   or misaligned                           */
#define KP_ERR_SOLVER      -5   /* the FP64 factor SVD (rocSOLVER) failed,
                                   or its workspace size query did         */

#define KP_MAX_PSF 63           /* largest supported PSF support K          */
#define KP_BC_ZERO      0       /* image zero outside [0, n)^2 (BTTB A)     */
#define KP_BC_PERIODIC  1       /* image extended periodically (BCCB A,
                                   K <= n); one-term KP with circulant
                                   factors                                 */
#define KP_BC_REFLEXIVE 2       /* image extended by half-sample
                                   reflection, K <= n; reflexive
                                   (Toeplitz-plus-Hankel) factors.  For a
                                   PSF symmetric in both axes A^T = A is the
                                   same blur; for any other A^T is the
                                   correlation over [-h, n+h) folded back
                                   onto the image, applied by FFTs only:
                                   such a plan's solves use KP_NORMAL_FFT
                                   and tol >= 1e-7, and the FP64 normal
                                   operator, the direct normal form and
                                   batched solves give KP_ERR_UNSUPPORTED  */
#define KP_SETUP_LOWP   0x100   /* flag OR-ed into kp_setup's bc: reduced-
                                   precision construction of S, V_r, V_c
                                   (Section 3 leaves computing them in half
                                   precision to future work): each factor
                                   is scaled by a power of two, rounded to
                                   FP16, and factorised by FP32 rocSOLVER */

/* ---- mode bits for pcg_solve / pcg_solve_batched --------------------- */
#define KP_CG        0x000      /* no preconditioner                        */
#define KP_PCG       0x001      /* PCG, Fletcher-Reeves beta (Section 3)    */
#define KP_FPCG      0x002      /* flexible PCG, Polak-Ribiere beta
                                   (Section 3, last paragraph)             */
#define KP_SOLVER_MASK 0x003
#define KP_P32       0x000      /* preconditioner factors and products FP32 */
#define KP_P16       0x010      /* FP16 factors, FP16 MFMA, FP32 accumulate */
#define KP_P8        0x020      /* FP8 e4m3 with 32-entry block scales      */
#define KP_PREC_MASK 0x030
#define KP_WARM      0x100      /* x holds the initial guess on entry       */
#define KP_BATCH_EAGER 0x200    /* pcg_solve_batched: launch every iteration
                                   eagerly instead of replaying a hipGraph */
#define KP_NO_FALLBACK 0x400    /* pcg_solve: no FP32 restart on failure    */
#define KP_EXACT_DIAG 0x800     /* preconditioner S = 1 / (D0 + lambda^2) with
                                   D0 = diag(V^T A^T A V), the exact diagonal
                                   of A^T A in the one-term KP basis V =
                                   V_r (x) V_c, built from every term of eq.
                                   (KronSumDecomp) (Section 5), in place of
                                   1 / (s_c^2 s_r^2 + lambda^2) (eq.
                                   (PreconSolve)).  Same V, same kernels and
                                   cost per iteration; equal to the default
                                   for separable PSFs.  An extension of the
                                   paper's preconditioner.                 */
#define KP_HIST 0x1000          /* pcg_solve: record the residual history
                                   of the solve in the plan (kp_get_history) */
#define KP_HIST_MAX 16384       /* history entries kept: iterations 0 ..
                                   KP_HIST_MAX - 1                         */

typedef struct kp_plan_s *kp_plan_t;   /* opaque */

/* Result of one solve. */
typedef struct kp_info_s {
    int32_t iters;          /* H_lambda applications (A, A^T pairs) in the
                               iteration, as the paper counts iterations   */
    int32_t status;         /* KP_OK, KP_MAXIT or KP_BREAKDOWN             */
    int32_t replacements;   /* true-residual recomputations                 */
    int32_t fallback;       /* 1 if pcg_solve restarted with the FP32
                               preconditioner                              */
    double  relres_rec;     /* recurrence ||r|| / ||A^T b|| at exit        */
    double  relres_true;    /* true ||A^T(b - A x) - lambda^2 x|| / ||A^T b||
                               at exit (b - A x accumulated in FP64)       */
    double  lambda;
    double  rhs_norm;       /* ||A^T b||_2                                 */
    double  misfit;         /* ||A x - b||_2 (pcg_solve_batched only; 0 for
                               pcg_solve)                                 */
    float   ms;             /* pcg_solve: device time in milliseconds
                               between HIP events recorded on `stream`
                               around all the work it enqueued (the FP32
                               restart included); 0 for pcg_solve_batched */
    int32_t reserved;
} kp_info_t;

/* Properties of a plan (the Kronecker approximation it holds). */
typedef struct kp_plan_info_s {
    int32_t n, k;
    int32_t kron_terms;     /* numerical rank of the weighted PSF: the
                               number of Kronecker terms needed to
                               represent A exactly (Table 1's k)          */
    int32_t normal_op;      /* form of H p the solver uses: KP_NORMAL_DIRECT
                               or KP_NORMAL_FFT (autotuned at setup)      */
    double  kp_rel_error;   /* ||A - A_r (x) A_c||_F / ||A||_F (Table 1)   */
    double  sigma_c_max, sigma_c_min, sigma_r_max, sigma_r_min;
    size_t  device_bytes;   /* device memory held by the plan              */
    int32_t blur_config;    /* blur tile shape picked by the setup-time
                               autotuner (index into its candidate list)  */
    float   blur_config_ms[8]; /* autotuner time per candidate (ms)       */
    int32_t fft_length;     /* L of the FFT form (zero-padded L x L grid),
                               0: no FFT form at this size                 */
    float   normal_op_ms[2];   /* autotuner time of H p: direct, FFT (ms)  */
} kp_plan_info_t;

/*
 * kp_workspace_size -- device bytes a plan for an n x n image and a K x K
 * PSF needs on the current device: the plan's data (factors, taps, tables,
 * the solver's vectors and control block) and, overlapping the solver's
 * vectors, the scratch of the construction in kp_setup, rocSOLVER's own
 * workspace included (found by rocBLAS's device-memory size query; the
 * first call on a device creates the library's rocBLAS handle for it, which
 * is kept for the process).  `modes` is reserved (pass 0).  Returns 0 for
 * invalid sizes or when the query fails (no device).
 */
size_t kp_workspace_size(int n, int k, int modes);

/*
 * kp_setup -- build the one-term Kronecker approximation and its SVD.
 *
 * Section 3, eq. (AKronSVD) and Section 5, eq. (KronSumDecomp): A is
 * approximated by the Frobenius-optimal Kronecker product A_r (x) A_c
 * (built from the leading singular triple of the PSF weighted by
 * sqrt(n - |k - h|) on both sides: banded Toeplitz factors for the zero
 * boundary; for the periodic and reflexive boundaries every weight is n,
 * i.e. the plain PSF SVD, and the factors are circulant or reflexive
 * Toeplitz-plus-Hankel), and A_r, A_c are factorised by
 * FP64 SVDs on the device.  The paper states no boundary condition; both
 * keep its PSF centre (h, h) and true convolution for A.  V_r, V_c are stored in FP32, FP16 and FP8 (with
 * block scales), U_r, U_c in FP32, singular values in FP64 and FP32.
 *
 *   psf        host, K*K float64, row-major
 *   k, n       PSF support (odd, <= KP_MAX_PSF, <= 2n-1; <= n for the
 *              periodic boundary), image size
 *   bc         KP_BC_ZERO, KP_BC_PERIODIC or KP_BC_REFLEXIVE, optionally
 *              | KP_SETUP_LOWP
 *              (other values: KP_ERR_UNSUPPORTED)
 *   workspace  device buffer of >= kp_workspace_size(n, k, 0) bytes,
 *              16-byte aligned, that holds all of the plan's device data
 *              and the construction's scratch (rocSOLVER's workspace is
 *              handed to rocBLAS from it): with a workspace kp_setup and
 *              every later call on the plan allocate no device memory.  The
 *              caller keeps ownership and keeps it alive until kp_destroy.
 *              NULL lets the plan allocate (hipMalloc) and own its memory.
 *   ws_bytes   size of `workspace` (ignored if workspace is NULL)
 *   plan       out: the new plan (NULL on error)
 * Errors: KP_ERR_ARG, KP_ERR_UNSUPPORTED, KP_ERR_WORKSPACE (too small or
 * misaligned), KP_ERR_HIP, KP_ERR_SOLVER.  Constructions on one device are
 * serialised (they share the device's rocBLAS handle).  Synchronises
 * `stream`.
 */
int kp_setup(const double *psf, int k, int n, int bc, void *workspace,
             size_t ws_bytes, void *stream, kp_plan_t *plan);

/* kp_plan_query -- fill `out` with the plan's properties (host only). */
int kp_plan_query(kp_plan_t plan, kp_plan_info_t *out);

/*
 * pcg_solve -- solve (A^T A + lambda^2 I) x = A^T b (eq. (tik:normal2)).
 *
 * Solver (mode & KP_SOLVER_MASK): CG, PCG with M = A_hat^T A_hat +
 * lambda^2 I applied as Z = V_c (S .* (V_c^T R V_r)) V_r^T (eq.
 * (PreconSolve)), or flexible PCG (Polak-Ribiere beta, Section 3; the one
 * direction update after a true-residual replacement takes the
 * Fletcher-Reeves beta, since the replacement breaks the recurrence the
 * Polak-Ribiere form relies on).  The same lambda is used in M and in the
 * problem (Section 5.3).  Preconditioner precision: mode & KP_PREC_MASK.
 * Vectors are FP32, matvecs FP32; the solution is accumulated in FP64 on
 * the device and the scalars alpha, beta, ||r|| are accumulated and kept in
 * FP64.  The true residual A^T (b - A x) - lambda^2 x (= c - H x) is
 * recomputed whenever the recurrence residual has fallen 1000x since the
 * last recomputation and before convergence is declared, and replaces the
 * recurrence residual: b - A x is accumulated in FP64, A^T of it on the
 * FP32-class blur for tol >= 1e-7 and in FP64 below (a reflexive plan whose
 * PSF is not symmetric: by FFTs, tol < 1e-7 gives KP_ERR_UNSUPPORTED).
 * Later recomputations
 * subtract H (x - x_a) from the last true residual r_a at x_a (FP32 matvecs
 * on the step, FP64 sums) once ||r_a|| is below min(1e-2, 1e4 tol) ||A^T b||
 * (those matvecs err by up to about 1e-5 ||r_a||).
 *
 *   b       device, n*n float32 data
 *   lambda  > 0, tol > 0 (relative to ||A^T b||), maxit >= 1
 *   x       device, n*n float32, not aliasing b: initial guess if
 *           mode & KP_WARM, else ignored (x_0 = 0); on return the last
 *           iterate (written in FP32 while the solve runs: b is read by
 *           every true residual)
 *   info    out (may be NULL)
 * If a solve with the FP16 or FP8 preconditioner ends in KP_MAXIT or
 * KP_BREAKDOWN (with a finite iterate), it is restarted from its last
 * iterate with the FP32 preconditioner and its own budget of maxit
 * iterations (info->iters counts both runs, info->fallback = 1); mode bit
 * KP_NO_FALLBACK turns this off (the restart keeps KP_EXACT_DIAG and
 * KP_HIST).  With KP_HIST the residual after every iteration is recorded
 * in the plan for kp_get_history (one FP64 store per scalar step).
 * Returns KP_OK (true relative residual <= tol), KP_OK_FALLBACK, KP_MAXIT,
 * KP_BREAKDOWN or an error.  Synchronises `stream` (it reads back the
 * convergence state).
 */
int pcg_solve(kp_plan_t plan, const float *b, double lambda, double tol,
              int maxit, int mode, float *x, kp_info_t *info, void *stream);

/*
 * gcv_lambda -- choose lambda on a grid with (weighted) GCV in the KP-SVD
 * basis (Section 2.2, eqs. (GCVTikSVD) and (wGCVTikSVD), evaluated with the
 * Kronecker approximation's SVD as in Section 5.1):
 *   b_hat = U_c^T B U_r,  s_ij = s_c[i] s_r[j],
 *   G_w(l) = N sum (l^2 b_hat/(s^2+l^2))^2 / (sum ((1-w) s^2 + l^2)/(s^2+l^2))^2
 * omega = 1 gives GCV.  For omega > 1 the trace term (the denominator
 * before squaring) increases with l and is negative for small l, where G_w
 * would fall back towards 0: those grid points score +inf, so the choice is
 * made on the branch continuous with large l (the paper minimises on a
 * bracket).  lambda_out = the grid value with the smallest score (ties:
 * smallest index).  scores_out: ngrid FP64 scores (host, may be NULL).
 * grid: host array of ngrid > 0 positive values.  Synchronises.
 */
int gcv_lambda(kp_plan_t plan, const float *b, const double *grid, int ngrid,
               double omega, double *lambda_out, double *scores_out,
               void *stream);

/*
 * discrepancy_lambda -- the discrepancy principle in the KP-SVD basis
 * (eq. (DSCTikSVD)): D(l) = sum (l^2 b_hat/(s^2+l^2))^2 - (eta*noise)^2.
 * lambda_out = the largest grid value with D <= 0 (D grows with l), else
 * grid[0].  values_out: ngrid FP64 values of D (may be NULL).
 */
int discrepancy_lambda(kp_plan_t plan, const float *b, const double *grid,
                       int ngrid, double noise_norm, double eta,
                       double *lambda_out, double *values_out, void *stream);

/*
 * pcg_solve_batched -- many solves of eq. (tik:normal2) in one set of
 * launches: item i solves with plan plans[plan_of_item[i]] (its PSF and
 * image size), data b[i], parameter lambdas[i], writing x[i].  All items
 * share tol, maxit and mode (solver and preconditioner bits and
 * KP_EXACT_DIAG as pcg_solve; with KP_P8 every item's n must be a multiple
 * of 128, else KP_ERR_UNSUPPORTED, and there is no FP32 restart of items
 * that fail, which end with KP_MAXIT; with KP_WARM
 * every x[i] holds its item's initial guess, whose residual is a full FP64
 * true residual, e.g. the solution at the neighbouring lambda of a sweep;
 * KP_BATCH_EAGER launches the
 * iterations eagerly instead of replaying a captured hipGraph).  Uneven
 * image sizes and PSF supports are allowed.  Each phase of an iteration is
 * one launch over the tiles of all items still iterating; each item stops
 * on its own (converged, maxit, breakdown).  infos[i] receives item i's
 * outcome, including its data misfit ||A x - b||.  Plans of every boundary
 * condition may be mixed; a reflexive plan whose PSF is not symmetric gives
 * KP_ERR_UNSUPPORTED (the batched matvecs are direct blurs).
 *
 *   plans, nplans   array of plan handles and its length
 *   b, x            arrays of nitems device pointers (FP32 n_i x n_i, 16-byte
 *                   aligned); lambdas: host array of nitems values > 0
 *   plan_of_item    host array of nitems indices into plans
 *   workspace       device buffer of >= pcg_solve_batched_workspace_size
 *                   bytes, 256-byte aligned, owned by the caller: the items'
 *                   vectors (about 56 n_i^2 bytes each), control blocks and
 *                   tile tables.  The library allocates no device memory.
 * The iterations run on a non-blocking stream of the library's (one per
 * device, created on first use), ordered after `stream` by an event and
 * before the return; batched calls are serialised per process.
 * Synchronises `stream`.  Returns KP_OK if every item converged, KP_MAXIT /
 * KP_BREAKDOWN if some did not (see infos), KP_ERR_WORKSPACE, or an error.
 */
int pcg_solve_batched(const kp_plan_t *plans, int nplans, const float *const *b,
                      const double *lambdas, const int *plan_of_item, int nitems,
                      double tol, int maxit, int mode, float *const *x,
                      kp_info_t *infos, void *workspace, size_t ws_bytes,
                      void *stream);

/* pcg_solve_batched_workspace_size -- device bytes pcg_solve_batched needs
   for these plans, items and mode (0 for invalid arguments). */
size_t pcg_solve_batched_workspace_size(const kp_plan_t *plans, int nplans,
                                        const int *plan_of_item, int nitems,
                                        int mode);

/*
 * opt_lambda -- the optimal-error rule in the KP-SVD basis, eq. (OptTikSVD):
 *   x_hat = V_c^T X_true V_r,  O(l) = sum (s b_hat/(s^2+l^2) - x_hat)^2,
 * which needs the true image (synthetic problems only: the targets the
 * lambda network is trained on).  x_true: device FP32 n x n.  lambda_out =
 * grid argmin (ties: smallest index); scores_out: ngrid values (may be
 * NULL).  grid: host, 1..64 positive values.  Synchronises.
 */
int opt_lambda(kp_plan_t plan, const float *b, const float *x_true,
               const double *grid, int ngrid, double *lambda_out,
               double *scores_out, void *stream);

/* kp_destroy -- release the plan (and its memory if it allocated it).
   Waits for the plan's last enqueued work (an event recorded on the stream
   of the last call that used it), not for other streams or the device. */
int kp_destroy(kp_plan_t plan);

/* ---- learned choice of lambda ------------------------------------------
 *
 * The paper picks lambda by GCV, weighted GCV or the discrepancy principle
 * in the KP-SVD basis (Section 2.2, Section 5.1) and leaves a systematic
 * choice of these parameters open (Section 5.1, Section 6).  These entry
 * points are the library's extension for that: a network maps KP-SVD
 * spectral features of b to log10(lambda), and GCV judges its answer.
 *
 * Features (kp_features): with c = V_c^T B V_r and s_ij = s_c[i] s_r[j],
 * 64 bins of log10(s) over [-8, 0) (s < 1e-8 -> bin 0, s >= 1 -> bin 63);
 *   f[k]      = log10(max(mean of c^2 over bin k, 1e-30))  (empty: 1e-30)
 *   f[64 + k] = log10(count of bin k / n^2 + 1e-12).
 * Network: 128 -> 256 -> 256 -> 256 -> 1, exact GELU z Phi(z) after each
 * hidden layer, linear output, on features standardised by the model's
 * per-feature mean and scale.  Hidden layers: FP16 weights and activations
 * on MFMA with FP32 accumulation; output layer, backward pass and Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on FP32 master weights.
 * Loss: mean over the batch of (y - t)^2 (t = log10 lambda target).
 *
 * Parameters are one flat FP32 array of KP_MLP_NPARAM values, weights
 * [out][in] row-major: W1 (256x128), b1 (256), W2 (256x256), b2, W3
 * (256x256), b3, W4 (1x256), b4 (1).
 * A model is not thread safe: one host thread / stream at a time.
 */
#define KP_MLP_NFEAT   128
#define KP_MLP_HIDDEN  256
#define KP_MLP_NPARAM  164865

typedef struct kp_mlp_s *kp_mlp_t;   /* opaque */

/* Outcome of kp_lambda_learned. */
typedef struct kp_lambda_info_s {
    double  lambda;        /* the choice: lambda_pred, or lambda_gcv on
                              fallback                                     */
    double  lambda_pred;   /* 10^(network output), clipped to the grid's
                              range                                        */
    double  lambda_gcv;    /* GCV grid argmin                              */
    double  gcv_ratio;     /* G(lambda_pred) / min_grid G - 1              */
    int32_t fell_back;     /* 1 if gcv_ratio > tau                         */
    int32_t reserved;
} kp_lambda_info_t;

/* kp_features -- the 128 features of b (device FP32 n x n) into
   features_out (device, 128 floats). */
int kp_features(kp_plan_t plan, const float *b, float *features_out,
                void *stream);

/* mlp_workspace_size -- device bytes of a model for batches of at most
   max_batch rows (1 <= max_batch <= 65536); 0 if out of range. */
size_t mlp_workspace_size(int max_batch);

/* mlp_create -- a model in `workspace` (device, >= mlp_workspace_size
   bytes, 16-byte aligned; NULL: the library allocates).  Parameters start
   at zero and the normaliser at mean 0, scale 1: set both before use. */
int mlp_create(int max_batch, void *workspace, size_t ws_bytes, void *stream,
               kp_mlp_t *mlp);

/* mlp_set_params / mlp_get_params -- copy the KP_MLP_NPARAM FP32 master
   parameters from / to a host array.  Setting them resets Adam's moments
   and step count.  Synchronise. */
int mlp_set_params(kp_mlp_t mlp, const float *params, void *stream);
int mlp_get_params(kp_mlp_t mlp, float *params, void *stream);

/* mlp_set_normalizer / mlp_get_normalizer -- the per-feature mean and
   scale (host arrays of 128; scales must be finite and > 0).  Synchronise. */
int mlp_set_normalizer(kp_mlp_t mlp, const float *mean, const float *scale,
                       void *stream);
int mlp_get_normalizer(kp_mlp_t mlp, float *mean, float *scale, void *stream);

/* mlp_fit_normalizer -- set the normaliser to the per-feature mean and
   population standard deviation of nb rows (device, nb x 128 FP32); a
   feature with deviation below 1e-6 gets scale 1. */
int mlp_fit_normalizer(kp_mlp_t mlp, const float *features, int nb,
                       void *stream);

/* lambda_predict -- network outputs (log10 lambda) of nb feature rows
   (device, nb x 128 FP32) into log10_lambda (device, nb FP64).  Any nb >= 1
   (processed max_batch rows at a time).  Does not synchronise. */
int lambda_predict(kp_mlp_t mlp, const float *features, int nb,
                   double *log10_lambda, void *stream);

/* lambda_predict_noalloc -- lambda_predict for callers that cannot
   allocate device memory (code under HIP graph capture, serving loops,
   harnesses that forbid hipMalloc): the same kernels and results, with the
   network's activations in a static device array of the library
   (KP_PREDICT_NOALLOC_BYTES, about 10.5 MiB per GPU, held until the
   process ends) instead of the model's workspace.  1 <= nb <=
   KP_PREDICT_NOALLOC_MAX_ROWS (larger nb: KP_ERR_WORKSPACE; call again per
   chunk).  Calls no allocating routine: the array's device address is
   looked up once per device, with that device current, by mlp_create (or
   by the first call on a device where no model was created).
   Every call on one GPU shares the array: calls that overlap on a GPU (two
   streams, two threads) race and must be serialised by the caller.
   Nothing in the array needs to start at zero (the forward writes every
   activation of rows 0..nb-1 before reading it).  Does not synchronise. */
#define KP_PREDICT_NOALLOC_MAX_ROWS 2048
#define KP_PREDICT_NOALLOC_BYTES 11026432   /* 10.5 MiB + 16 KiB */
int lambda_predict_noalloc(kp_mlp_t mlp, const float *features, int nb,
                           double *log10_lambda, void *stream);

/* mlp_train_step -- one Adam step on the minibatch rows[0..nb) (host
   array of indices into the nrows feature rows / targets; NULL: rows
   0..nb-1) of features (device, nrows x 128) and targets (device, nrows
   FP32 log10 lambda), with learning rate lr > 0.  1 <= nb <= max_batch.
   loss_out (host, may be NULL): the minibatch loss before the step;
   giving it synchronises. */
int mlp_train_step(kp_mlp_t mlp, const float *features, const float *targets,
                   int nrows, const int *rows, int nb, float lr,
                   double *loss_out, void *stream);

/* mlp_gradients -- loss and the gradient of the loss (host array of
   KP_MLP_NPARAM FP32, same layout as the parameters) on rows 0..nb-1,
   without updating.  Synchronises. */
int mlp_gradients(kp_mlp_t mlp, const float *features, const float *targets,
                  int nb, float *grads, double *loss_out, void *stream);

/* mlp_destroy -- release the model. */
int mlp_destroy(kp_mlp_t mlp);

/*
 * kp_lambda_learned -- lambda for b from the network, judged by GCV:
 * features of b -> network -> lambda_pred (clipped to [min grid, max grid]);
 * G (eq. (GCVTikSVD) in the KP-SVD basis) on the grid and at lambda_pred;
 * if G(lambda_pred) / min_grid G - 1 > tau the GCV grid argmin is used.
 * grid: host, 1..63 positive values; tau >= 0.  Synchronises.
 */
int kp_lambda_learned(kp_plan_t plan, kp_mlp_t mlp, const float *b,
                      const double *grid, int ngrid, double tau,
                      kp_lambda_info_t *info, void *stream);

/* kp_strerror -- static description of a status code. */
const char *kp_strerror(int status);

/* ---- operator-level entry points (used by the parity tests) ---------- */

/* y = A x (transpose = 0) or y = A^T x (transpose = 1); FP32 in and out,
   FP32 accumulation (A^T of a reflexive plan whose PSF is not symmetric:
   the folded correlation by FFTs, as KP_NORMAL_FFT's last passes).  x and y
   must not alias. */
int kp_blur(kp_plan_t plan, const float *x, float *y, int transpose,
            void *stream);

/* y = (A^T A + lambda^2 I) x with FP64 accumulation; y is FP64 (device).
   KP_ERR_UNSUPPORTED for a reflexive plan whose PSF is not symmetric. */
int kp_normal_fp64(kp_plan_t plan, const float *x, double lambda, double *y,
                   void *stream);

/* z = M^{-1} r with the mode's preconditioner precision (mode &
   KP_PREC_MASK) and S table (KP_EXACT_DIAG), using the same kernels as the
   solver.  r, z device FP32, must not alias. */
int kp_precond(kp_plan_t plan, const float *r, double lambda, int mode,
               float *z, void *stream);

/* Timing helpers for the benchmark: launch the blur kernel of kp_blur (or
   the preconditioner chain of kp_precond) `reps` times back to back on
   `stream`, bracketed by HIP events, and return the mean time per launch
   (per chain for kp_time_precond) in *avg_ms.  Synchronises. */
int kp_time_blur(kp_plan_t plan, const float *x, float *y, int transpose,
                 int reps, float *avg_ms, void *stream);
int kp_time_precond(kp_plan_t plan, const float *r, double lambda, int mode,
                    float *z, int reps, float *avg_ms, void *stream);

/* Blur kernel used by pcg_solve and kp_blur: 0..5 are FP32-VALU tile shapes,
   6 the FP16-split MFMA kernel on 16x16x32 instructions, 7 the same on
   32x32x16 instructions; kp_setup's autotuner picks the fastest.
   kp_set_blur_config overrides the choice (cfg in 0..7; *prev, if not NULL,
   receives the previous one). */
#define KP_BLUR_MFMA 6
#define KP_BLUR_MFMA32 7
int kp_set_blur_config(kp_plan_t plan, int cfg, int *prev);

/*
 * The normal operator H p = A^T A p + lambda^2 p in two forms, both FP32:
 *  - KP_NORMAL_DIRECT: A p then A^T (A p) on the plan's direct blur (the
 *    kernel kp_set_blur_config selects);
 *  - KP_NORMAL_FFT: zero-padded FFTs (Section 2.3 names FFTs for
 *    structured A; Section 5.2's cost model assumes cheap matvecs): with L
 *    the smallest length >= n + (K-1)/2 in a fixed menu of 28 products of
 *    three radices (64 .. 2160, enough for n <= 2048, K <= 63) and Hc the L x L
 *    DFT of the PSF wrapped around the origin, A p = crop(IDFT(Hc .*
 *    DFT(pad p))) and A^T q = crop(IDFT(conj(Hc) .* DFT(pad q))) on the
 *    n x n window (exact: every wrapped tap lands in the zero pad).  For
 *    the reflexive boundary p is first extended by h = (K-1)/2 reflected
 *    rows and columns per side (L >= n + K - 1), and A^T q is the
 *    correlation over [-h, n+h)^2 with the outer h-wide frame folded back
 *    onto its mirror images.  Five passes of one-workgroup-per-line
 *    Stockham FFTs in LDS; FP32 with the PSF spectrum and twiddles
 *    computed in FP64.
 * kp_setup times both on the plan and the solver uses the faster.  The FFT
 * form is offered for KP_BC_ZERO and KP_BC_REFLEXIVE plans (periodic:
 * direct; forcing FFT gives KP_ERR_UNSUPPORTED); a reflexive plan whose
 * PSF is not symmetric has the FFT form only (forcing direct gives
 * KP_ERR_UNSUPPORTED).
 * kp_set_normal_op forces a form for pcg_solve's iterations (true residuals
 * stay on the blurs, but for the FFT A^T of a reflexive plan whose PSF is
 * not symmetric); kp_normal computes y = H x with the plan's form
 * (KP_NORMAL_PLAN) or a given one, into the FP32 device image y (x and y
 * must differ; the direct form uses the plan's scratch vector); it
 * synchronises.  kp_time_normal: mean time of `reps` back-to-back
 * applications between HIP events (synchronises).
 */
#define KP_NORMAL_PLAN   -1
#define KP_NORMAL_DIRECT  0
#define KP_NORMAL_FFT     1
int kp_set_normal_op(kp_plan_t plan, int op, int *prev);
int kp_normal(kp_plan_t plan, const float *x, double lambda, float *y, int op,
              void *stream);
int kp_time_normal(kp_plan_t plan, const float *x, float *y, int op, int reps,
                   float *avg_ms, void *stream);

/* Copy the exact KP-basis diagonal D0[i][j] = ||A (v_c,i v_r,j^T)||_F^2
   (the table KP_EXACT_DIAG uses; built by kp_setup from all Kronecker terms
   with FP64 arithmetic, stored FP32) to the host array d0 (n*n, row-major:
   i indexes the column factor's singular vectors, j the row factor's).
   The copy runs on a non-blocking stream of the library's and waits for
   nothing else (the table is final once kp_setup returns).  For a KP_BC_PERIODIC plan D0 comes from the
   circulant terms; its singular vectors are unique only up to rotations
   within pairs of equal singular values, and D0 is that of the stored V. */
int kp_get_diag(kp_plan_t plan, float *d0);

/* Copy the FP64 singular values s_c, s_r (host arrays of n) and, if not
   NULL, the stored FP32 copies of V_c, V_r widened to FP64 row-major n x n
   host arrays (V[i*n + a] = V(i,a)).  Copies as kp_get_diag does. */
int kp_get_factors(kp_plan_t plan, double *sc, double *sr, double *vc,
                   double *vr);

/*
 * kp_get_history -- the residual history of the plan's last pcg_solve run
 * with mode bit KP_HIST: the convergence curve of the iteration (the
 * quantity behind the relative-error-per-iteration figures of Section 5),
 * relative to ||A^T b||.
 *   relres_rec   host, cap doubles (or NULL): entry k is ||r_k|| / ||A^T b||
 *                of the recurrence residual after iteration k (k = 0: r_0 =
 *                A^T b, so 1.0), before any true-residual replacement at k
 *   relres_true  host, cap doubles (or NULL): entry k is ||c - H x_k|| /
 *                ||A^T b|| where a true residual was formed at iteration k
 *                (replacement, warm start, final check), else NaN
 *   cap          >= 0 entries to copy; count (out) receives the number
 *                recorded, min(iterations + 1, KP_HIST_MAX) (0 if the last
 *                solve ran without KP_HIST or had zero or non-finite data)
 * After the automatic FP32 restart the history is that of the restart.
 * Synchronises `stream`.  Returns KP_OK or KP_ERR_ARG (null plan or count,
 * cap < 0) / KP_ERR_HIP.
 */
int kp_get_history(kp_plan_t plan, double *relres_rec, double *relres_true,
                   int cap, int *count, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* KPCG_H */
