// H p = A^T A p + lambda^2 p by zero-padded FFTs (the FFT form of the matvec
// the paper's Section 2.3 names for structured A, and its Section 5.2 cost
// model: cheap matvecs when FFTs are available).
//
// With the zero boundary, A p is the n x n window of the linear convolution
// of p with the PSF.  On an L x L grid with L >= n + h the circular
// convolution with the PSF wrapped around the origin equals it on that
// window (every wrapped tap lands in the zero pad), and so does the circular
// correlation for A^T q.  So, with Hc the 2-D DFT of the wrapped PSF,
//     A p   = crop(IDFT(Hc .* DFT(pad(p)))),
//     A^T q = crop(IDFT(conj(Hc) .* DFT(pad(q)))).
// The reflexive boundary extends p by h reflected rows and columns per side
// first (L >= n + 2h), and its A^T folds the correlation over [-h, n+h) back
// onto the image.
//
// Five passes:
//   rows_fwd  two real rows of p packed as one complex line (x_a + i x_b),
//             one length-L transform, split into the two half spectra
//             (k = 0 .. L/2) -> S
//   cols      one column k of S: transform, times Hc[:, k] (1/L^2 folded
//             in), inverse transform, rows 0 .. n-1 kept -> T
//   rows_mid  two rows of T: Hermitian extension packed as one complex
//             spectrum, inverse transform (real part row a, imaginary part
//             row b: A p), columns 0 .. n-1 kept and re-padded, forward
//             transform, split -> S (the half spectra of A p)
//   cols      with conj(Hc) -> T
//   rows_out  inverse as rows_mid, w = result + lambda^2 p on the n x n
//             window, and the per-workgroup partial sums of p . w.
// S and T are stored by frequency: S[k][row], T[k][row] (row pitch spitch,
// tpitch), so the column passes read and write whole contiguous lines and
// a row pass's workgroup, which owns 2B consecutive rows, reads and writes
// 2B consecutive elements per frequency.
//
// Each length-L transform is a Stockham autosort FFT of three stages,
// L = R1 R2 R3 (radices from a fixed menu of lengths, all compile-time):
// stage s of radix R with Ns = the product of the earlier radices reads
// x[j + r L/R] (r < R) for each j < L/R, twiddles by W_{Ns R}^{(j mod Ns) r},
// transforms the R values in registers and writes them to
// (j / Ns) Ns R + (j mod Ns) + r Ns.  The in-register transforms are
// mixed-radix (8, 4, 2, 3, 5, 7) with the roots of unity as compile-time
// constants; W_L comes from an FP32 table built in FP64 and kept in LDS.  The
// first stage reads global memory and the last may write it; the others
// exchange through LDS.  A workgroup transforms B lines at once.
#include <cmath>
#include <type_traits>

#include "blur_core.h"

namespace kpcg {

struct FftGeom {
  int n, L, F;
  const float2* tw;                     // exp(-2 pi i t / L), t < L
  int refl, h;                          // reflexive boundary; PSF half-width
  int spitch, tpitch;                   // row pitch of S and T (elements)
};

// half-sample reflection of an index in [-n, 2n)
__device__ inline int refl_index(int q, int n) { return q < 0 ? -q - 1 : (q >= n ? 2 * n - 1 - q : q); }

__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ inline float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }   // -i a
__device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// ---------------------------------------------------------------------------
// compile-time roots of unity: W<N, M> = exp(-2 pi i M / N)
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

__host__ __device__ constexpr double ce_sin(double x) {      // |x| <= pi
  double t = x, s = x;
  for (int i = 1; i < 26; ++i) {
    t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}
__host__ __device__ constexpr double ce_cos(double x) {      // |x| <= pi
  double t = 1.0, s = 1.0;
  for (int i = 1; i < 26; ++i) {
    t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}
// the angle -2 pi M / N reduced to (-pi, pi]
__host__ __device__ constexpr double root_angle(int N, int M) {
  const int m = ((M % N) + N) % N;
  const int mm = 2 * m > N ? m - N : m;
  return -2.0 * kPi * (double)mm / (double)N;
}
template <int N, int M>
struct W {
  static constexpr float re = (float)ce_cos(root_angle(N, M));
  static constexpr float im = (float)ce_sin(root_angle(N, M));
};

template <int I, int E, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (I < E) {
    fn(std::integral_constant<int, I>{});
    static_for<I + 1, E>(fn);
  }
}

// ---------------------------------------------------------------------------
// forward DFTs of compile-time length in registers (W = exp(-2 pi i / N))
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dft2(float2* v) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
__device__ __forceinline__ void dft4(float2* v) {
  const float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]), a2 = cadd(v[1], v[3]),
               a3 = mul_mi(csub(v[1], v[3]));
  v[0] = cadd(a0, a2);
  v[1] = cadd(a1, a3);
  v[2] = csub(a0, a2);
  v[3] = csub(a1, a3);
}
__device__ __forceinline__ void dft8(float2* v) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e);
  dft4(o);
  constexpr float r = 0.70710678118654752f;
  // o_k *= exp(-i pi k / 4)
  o[1] = make_float2(r * (o[1].x + o[1].y), r * (o[1].y - o[1].x));
  o[2] = mul_mi(o[2]);
  o[3] = make_float2(r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}
// odd R: with A_k = v_k + v_{R-k}, B_k = v_k - v_{R-k} (k = 1 .. (R-1)/2),
// X_m = v_0 + sum_k cos(2 pi m k / R) A_k -/+ i sum_k sin(2 pi m k / R) B_k
// for m and R - m
template <int R>
__device__ __forceinline__ void dft_odd(float2* v) {
  constexpr int H = (R - 1) / 2;
  float2 A[H], B[H];
  static_for<1, H + 1>([&](auto k) {
    A[k - 1] = cadd(v[k], v[R - k]);
    B[k - 1] = csub(v[k], v[R - k]);
  });
  float2 out[R];
  float2 x0 = v[0];
  static_for<0, H>([&](auto k) { x0 = cadd(x0, A[k]); });
  out[0] = x0;
  static_for<1, H + 1>([&](auto m) {
    float2 re = v[0], im = make_float2(0.f, 0.f);
    static_for<1, H + 1>([&](auto k) {
      constexpr int e = (decltype(m)::value * decltype(k)::value) % R;
      constexpr float c = W<R, e>::re;     // cos(2 pi e / R)
      constexpr float s = -W<R, e>::im;    // sin(2 pi e / R)
      re.x = fmaf(c, A[k - 1].x, re.x);
      re.y = fmaf(c, A[k - 1].y, re.y);
      im.x = fmaf(s, B[k - 1].x, im.x);
      im.y = fmaf(s, B[k - 1].y, im.y);
    });
    out[m] = cadd(re, mul_mi(im));          // re - i im
    out[R - m] = csub(re, mul_mi(im));      // re + i im
  });
  static_for<0, R>([&](auto m) { v[m] = out[m]; });
}

template <int N>
constexpr int first_radix() {
  return (N % 8 == 0) ? 8 : (N % 4 == 0) ? 4 : (N % 2 == 0) ? 2 : (N % 3 == 0) ? 3
         : (N % 5 == 0) ? 5 : 7;
}

// v <- DFT_N(v); N a product of 2, 3, 5, 7 (decimation in time: N = R M,
// X[k + M q] = sum_r W_R^{rq} W_N^{rk} DFT_M(v[r + R m])[k])
template <int N>
__device__ __forceinline__ void dftr(float2 (&v)[N]) {
  if constexpr (N == 1) {
  } else if constexpr (N == 2) {
    dft2(v);
  } else if constexpr (N == 4) {
    dft4(v);
  } else if constexpr (N == 8) {
    dft8(v);
  } else if constexpr (N == 3 || N == 5 || N == 7) {
    dft_odd<N>(v);
  } else {
    constexpr int R = first_radix<N>(), M = N / R;
    static_assert(R * M == N && M > 1, "N must be 7-smooth");
    float2 d[R][M];
    static_for<0, R>([&](auto r) {
      static_for<0, M>([&](auto m) { d[r][m] = v[r + R * m]; });
      dftr<M>(d[r]);
    });
    static_for<1, R>([&](auto r) {
      static_for<1, M>([&](auto k) {
        constexpr int e = decltype(r)::value * decltype(k)::value;
        d[r][k] = cmul(d[r][k], make_float2(W<N, e>::re, W<N, e>::im));
      });
    });
    static_for<0, M>([&](auto k) {
      float2 t[R];
      static_for<0, R>([&](auto r) { t[r] = d[r][k]; });
      dftr<R>(t);
      static_for<0, R>([&](auto q) { v[k + M * q] = t[q]; });
    });
  }
}

// sum_t x[t] W^{-tk}: conj(DFT(conj x))
template <int N, bool INV>
__device__ __forceinline__ void dft_dir(float2 (&v)[N]) {
  if constexpr (INV) static_for<0, N>([&](auto i) { v[i].y = -v[i].y; });
  dftr<N>(v);
  if constexpr (INV) static_for<0, N>([&](auto i) { v[i].y = -v[i].y; });
}

// ---------------------------------------------------------------------------
// Stockham transforms of length L = R1 R2 R3 over B lines per workgroup
// ---------------------------------------------------------------------------
template <int A1, int A2, int A3>
struct Sh3 {
  static constexpr int R1 = A1, R2 = A2, R3 = A3;
  static constexpr int L = R1 * R2 * R3;
  static constexpr int F = L / 2 + 1;
#ifndef KPCG_FFT_B1_MIN
#define KPCG_FFT_B1_MIN 1536
#endif
  static constexpr int B = L >= KPCG_FFT_B1_MIN ? 1 : L >= 512 ? 2 : (L >= 192 ? 4 : 8);   // lines per workgroup
  static constexpr int RMIN = R1 < R2 ? (R1 < R3 ? R1 : R3) : (R2 < R3 ? R2 : R3);
  static constexpr int NTASK = B * (L / RMIN);                    // most tasks of a stage
  // one task per thread in every stage (a second round would double it)
  static constexpr int NT = ((NTASK + 63) / 64) * 64;
  static_assert(NT <= 1024, "too many tasks per stage");
  static constexpr int LP = L + 1;                                // line pitch in LDS
  static constexpr size_t LDS = (size_t)(L + 2 * B * LP) * sizeof(float2);
  static constexpr int TWN = (L + NT - 1) / NT;                  // twiddle loads per thread
  static constexpr int EPT = (B * L + NT - 1) / NT;              // elements per thread
};

__device__ inline bool fft_skip(const Ctrl* ctrl) { return ctrl != nullptr && ctrl->done != RUNNING; }

// Row passes: workgroup b runs on XCD b % 8 (the grid is a multiple of 8),
// and each XCD takes a contiguous range of the G line groups, so that the
// groups sharing cache lines of S and T (consecutive rows of one frequency)
// share one L2.  -1: no group (padding of the grid).
__device__ inline int xcd_line_group(int G) {
  const int per = gridDim.x / 8;
  const int g = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  return g < G ? g : -1;
}

// the twiddle table through registers (loads issued first) into LDS
template <int NT, int TWN>
struct TwLoad {
  float2 v[TWN];
  __device__ void load(const float2* __restrict__ tw, int L) {
#pragma unroll
    for (int e = 0; e < TWN; ++e) {
      const int t = threadIdx.x + e * NT;
      if (t < L) v[e] = tw[t];
    }
  }
  __device__ void store(float2* lds, int L) const {
#pragma unroll
    for (int e = 0; e < TWN; ++e) {
      const int t = threadIdx.x + e * NT;
      if (t < L) lds[t] = v[e];
    }
  }
};

// One radix-R stage over the workgroup's B lines: task (b, j), j < L/R,
// b fastest, reads src(b, j + r L/R) (r < R), multiplies by
// W_{Ns R}^{(j mod Ns) r}, transforms (INV: exponents negated) and writes
// dst(b, (j / Ns) Ns R + (j mod Ns) + r Ns).  After the stages with
// Ns = 1, R1, R1 R2 the lines hold their DFTs in natural order.
template <class C, int R, int Ns, bool INV, class Src, class Dst>
__device__ __forceinline__ void sh_stage(Src&& src, Dst&& dst, const float2* tw) {
  constexpr int J = C::L / R, TWS = C::L / (Ns * R);
  for (int q = threadIdx.x; q < C::B * J; q += C::NT) {
    const int b = q % C::B, j = q / C::B;
    const int k = j % Ns;
    float2 v[R];
    static_for<0, R>([&](auto r) { v[r] = src(b, j + decltype(r)::value * J); });
    if constexpr (Ns > 1) {
      static_for<1, R>([&](auto r) {
        float2 w = tw[k * decltype(r)::value * TWS];
        if constexpr (INV) w.y = -w.y;
        v[r] = cmul(v[r], w);
      });
    }
    dft_dir<R, INV>(v);
    const int base = (j / Ns) * Ns * R + k;
    static_for<0, R>([&](auto r) { dst(b, base + decltype(r)::value * Ns, v[r]); });
  }
}

struct NoStep {
  __device__ void operator()() const {}
};

// A whole transform: stage 1 from src into X, stage 2 from X into Y, stage
// 3 from Y into dst, with barriers between them.  src must not read X.
// after1 runs between stage 1 (which reads no twiddles) and its barrier: a
// pass stores its twiddle table to LDS there, so that waiting for the table
// does not hold back the issue of stage 1's global loads.
template <class C, bool INV, class Src, class Dst, class After1 = NoStep>
__device__ __forceinline__ void sh_transform(Src&& src, float2* X, float2* Y, Dst&& dst,
                                             const float2* tw, After1 after1 = {}) {
  sh_stage<C, C::R1, 1, INV>(src, [&](int b, int t, float2 v) { X[b * C::LP + t] = v; }, tw);
  after1();
  __syncthreads();
  sh_stage<C, C::R2, C::R1, INV>([&](int b, int t) { return X[b * C::LP + t]; },
                                 [&](int b, int t, float2 v) { Y[b * C::LP + t] = v; }, tw);
  __syncthreads();
  sh_stage<C, C::R3, C::R1 * C::R2, INV>([&](int b, int t) { return Y[b * C::LP + t]; }, dst, tw);
}

// Split the transforms Z (line b at Z + b LP) of x_a + i x_b into the half
// spectra of the two real rows, X_a = (Z_k + conj Z_{L-k}) / 2,
// X_b = (Z_k - conj Z_{L-k}) / (2 i), stored at S[k][sa], S[k][sb]; lines b
// fastest, so that the workgroup writes its 2B rows of one k together.
template <class C>
__device__ inline void split_store(const float2* Z, int line0, int nl, int rows,
                                   float2* __restrict__ S, int spitch) {
  for (int q = threadIdx.x; q < C::B * C::F; q += C::NT) {
    const int b = q % C::B, k = q / C::B, line = line0 + b;
    if (line >= nl) continue;
    const float2* zb = Z + b * C::LP;
    const float2 z = zb[k];
    const float2 zr = cconj(zb[k == 0 ? 0 : C::L - k]);
    const int sa = 2 * line, sb = sa + 1;
    S[(size_t)k * spitch + sa] = cscale(cadd(z, zr), 0.5f);
    if (sb < rows) S[(size_t)k * spitch + sb] = cscale(mul_mi(csub(z, zr)), 0.5f);
  }
}

// The Hermitian-extended spectrum of rows ra (real part, ra < 0: zero) and
// rb (imaginary part, rb < 0: zero) at frequency kap: Z = A + i B from the
// half spectra stored in T[k][row].  Only the loads sit under the guards:
// arithmetic on a loaded value inside its guard makes the compiler wait for
// that load before issuing the next, one memory latency per element.
template <class C>
__device__ inline float2 row_spectrum(const float2* __restrict__ T, int tpitch, int ra, int rb,
                                      int kap) {
  const bool low = kap < C::F;
  const int kk = low ? kap : C::L - kap;
  float2 A = make_float2(0.f, 0.f), Bv = A;
  if (ra >= 0) A = T[(size_t)kk * tpitch + ra];
  if (rb >= 0) Bv = T[(size_t)kk * tpitch + rb];
  const float ay = low ? A.y : -A.y, by = low ? Bv.y : -Bv.y;
  return make_float2(A.x - by, ay + Bv.x);
}

// ---------------------------------------------------------------------------
// pass kernels (LDS: the twiddle table, then line buffers A and Bf)
// ---------------------------------------------------------------------------

// Row pass of the forward transform.  Plain (ext = 0): rows 0 .. n-1 of p,
// zero-padded to L.  Extended (ext = 1, reflexive boundary): the image
// extended by half-sample reflection over the rows and columns [-h, n+h):
// row slot s holds image row refl(s - h), and a column index j in [-h, 0)
// sits at the circular position L + j.
template <class C>
__global__ __launch_bounds__(C::NT) void fft_rows_fwd_kernel(const float* __restrict__ p, FftGeom g,
                                                           int ext, float2* __restrict__ S,
                                                           const Ctrl* ctrl) {
  if (fft_skip(ctrl)) return;
  extern __shared__ float2 fft_lds[];
  float2* tw = fft_lds;
  float2* A = tw + C::L;
  float2* Bf = A + C::B * C::LP;
  const int n = g.n, h = ext ? g.h : 0;
  const int rows = n + 2 * h, nl = (rows + 1) / 2;
  const int grp = xcd_line_group((nl + C::B - 1) / C::B);
  if (grp < 0) return;
  const int line0 = grp * C::B;
  TwLoad<C::NT, C::TWN> ts;
  ts.load(g.tw, C::L);
  auto src = [&](int b, int t) -> float2 {
    float2 x = make_float2(0.f, 0.f);
    const int line = line0 + b;
    const int j = t >= C::L - h ? t - C::L : t;          // column of circular position t
    if (line >= nl || j < -h || j >= n + h) return x;
    const int jj = ext ? refl_index(j, n) : j;
    const int sa = 2 * line, sb = sa + 1;
    x.x = p[(size_t)(ext ? refl_index(sa - h, n) : sa) * n + jj];
    if (sb < rows) x.y = p[(size_t)(ext ? refl_index(sb - h, n) : sb) * n + jj];
    return x;
  };
  sh_transform<C, false>(src, A, Bf, [&](int b, int t, float2 v) { A[b * C::LP + t] = v; }, tw,
                         [&] { ts.store(tw, C::L); });
  __syncthreads();
  split_store<C>(A, line0, nl, rows, S, g.spitch);
}

// The first row pass with the direction step of the iteration before it
// folded in (zero boundary): every workgroup sums the nbz partials of r.z
// and z.Hp of the preconditioner's last GEMM in the scalar step's order
// and takes beta from them, forms p = z + beta p on its rows (each element
// read and written by one thread) and transforms the new p; workgroup 0
// stores r.z, z.Hp, beta (or the breakdown) and publishes.  The loads of z
// and the old p are issued before the partials are summed.
struct DirStep {
  const float* z;
  Ctrl* ctrl;
  const double* partials;
  int nbz;
  CtrlMirror* mirror;
};

template <class C>
__global__ __launch_bounds__(C::NT) void fft_rows_fwd_dir_kernel(float* __restrict__ p, FftGeom g,
                                                               float2* __restrict__ S, DirStep ds) {
  if (ds.ctrl->done != RUNNING) return;
  const StepIn kin = step_in(ds.ctrl);
  extern __shared__ float2 fft_lds[];
  __shared__ double sh[2 * fold_sh<C::NT>()];
  float2* tw = fft_lds;
  float2* A = tw + C::L;
  float2* Bf = A + C::B * C::LP;
  const int n = g.n, nl = (n + 1) / 2;
  const int grp = xcd_line_group((nl + C::B - 1) / C::B);
  if (grp < 0) return;                 // never workgroup 0
  const int line0 = grp * C::B;
  TwLoad<C::NT, C::TWN> ts;
  ts.load(g.tw, C::L);
  // this thread's task of stage 1 (one per thread): line b, positions
  // j + r L/R1; z and the old p of rows 2 line, 2 line + 1 there
  constexpr int R = C::R1, J = C::L / R;
  const int q = threadIdx.x, b = q % C::B, j = q / C::B, line = line0 + b;
  const bool task = q < C::B * J, rows_in = line < nl;
  const int sa = 2 * line, sb = sa + 1;
  float pa[R], pb[R], za[R], zb[R];
  static_for<0, R>([&](auto r) {
    const int t = j + decltype(r)::value * J;
    const bool in = task && rows_in && t < n;
    pa[r] = in ? p[(size_t)sa * n + t] : 0.f;
    za[r] = in ? ds.z[(size_t)sa * n + t] : 0.f;
    pb[r] = (in && sb < n) ? p[(size_t)sb * n + t] : 0.f;
    zb[r] = (in && sb < n) ? ds.z[(size_t)sb * n + t] : 0.f;
  });
  const double2 f = fold_slot2<C::NT>(ds.partials, SLOT_RZ, SLOT_ZW, ds.nbz, sh);
  const double rz = f.x, zw = f.y;
  bool ok;
  const double beta = beta_of(kin, rz, zw, &ok);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ds.ctrl->rz = rz;
    ds.ctrl->zw = zw;
    if (ok) ds.ctrl->beta = beta;
    else ds.ctrl->done = BREAKDOWN;
    if (ds.mirror != nullptr) publish_mirror(ds.ctrl, ds.mirror);
  }
  if (!ok) return;
  const float bt = (float)beta;
  ts.store(tw, C::L);
  if (task) {
    float2 v[R];
    static_for<0, R>([&](auto r) {
      const int t = j + decltype(r)::value * J;
      v[r] = make_float2(fmaf(bt, pa[r], za[r]), fmaf(bt, pb[r], zb[r]));
      if (rows_in && t < n) {
        p[(size_t)sa * n + t] = v[r].x;
        if (sb < n) p[(size_t)sb * n + t] = v[r].y;
      }
    });
    dft_dir<R, false>(v);
    static_for<0, R>([&](auto r) { A[b * C::LP + j * R + decltype(r)::value] = v[r]; });
  }
  __syncthreads();
  sh_stage<C, C::R2, C::R1, false>([&](int bb, int t) { return A[bb * C::LP + t]; },
                                   [&](int bb, int t, float2 v) { Bf[bb * C::LP + t] = v; }, tw);
  __syncthreads();
  sh_stage<C, C::R3, C::R1 * C::R2, false>([&](int bb, int t) { return Bf[bb * C::LP + t]; },
                                           [&](int bb, int t, float2 v) { A[bb * C::LP + t] = v; },
                                           tw);
  __syncthreads();
  split_store<C>(A, line0, nl, n, S, g.spitch);
}

// Column pass: column k of S (its in_rows row slots, slot s at the circular
// row position s - in_off, the rest zero), its transform times the PSF
// spectrum (or its conjugate), the inverse; rows 0 .. n-1 kept, or with fold
// (the correlation of the reflexive boundary's A^T) the rows [-h, n+h)
// folded onto the image by the reflection: row a gains rows -1-a (circular
// L-1-a, for a < h) and 2n-1-a (for a >= n-h).
template <class C>
__global__ __launch_bounds__(C::NT) void fft_cols_kernel(const float2* __restrict__ S, FftGeom g,
                                                       int in_rows, int in_off,
                                                       const float2* __restrict__ Ht, int conjH,
                                                       int fold, float2* __restrict__ T,
                                                       const Ctrl* ctrl) {
  if (fft_skip(ctrl)) return;
  extern __shared__ float2 fft_lds[];
  float2* tw = fft_lds;
  float2* A = tw + C::L;
  float2* Bf = A + C::B * C::LP;
  const int n = g.n, k0 = blockIdx.x * C::B;
  TwLoad<C::NT, C::TWN> ts;
  ts.load(g.tw, C::L);
  // the PSF spectrum of this thread's elements of the product below (only
  // the loads under the guard, conjugated at the product, so that the loads
  // are all in flight together)
  float2 hv[C::EPT];
#pragma unroll
  for (int i = 0; i < C::EPT; ++i) {
    const int q = threadIdx.x + i * C::NT, b = q % C::B, t = q / C::B, k = k0 + b;
    hv[i] = make_float2(0.f, 0.f);
    if (q < C::B * C::L && k < C::F) hv[i] = Ht[(size_t)k * C::L + t];
  }
  auto src = [&](int b, int t) -> float2 {
    const int k = k0 + b;
    const int sl = (t >= C::L - in_off ? t - C::L : t) + in_off;   // row slot of row t
    return (k < C::F && sl >= 0 && sl < in_rows) ? S[(size_t)k * g.spitch + sl]
                                                 : make_float2(0.f, 0.f);
  };
  sh_transform<C, false>(src, A, Bf, [&](int b, int t, float2 v) { A[b * C::LP + t] = v; }, tw,
                         [&] { ts.store(tw, C::L); });
  __syncthreads();
#pragma unroll
  for (int i = 0; i < C::EPT; ++i) {
    const int q = threadIdx.x + i * C::NT, b = q % C::B, t = q / C::B;
    float2 hq = hv[i];
    if (conjH) hq.y = -hq.y;
    if (q < C::B * C::L) A[b * C::LP + t] = cmul(A[b * C::LP + t], hq);
  }
  __syncthreads();
  auto srcA = [&](int b, int t) { return A[b * C::LP + t]; };
  if (!fold) {
    sh_transform<C, true>(srcA, Bf, A, [&](int b, int t, float2 v) {
      const int k = k0 + b;
      if (k < C::F && t < n) T[(size_t)k * g.tpitch + t] = v;
    }, tw);
    return;
  }
  sh_transform<C, true>(srcA, Bf, A, [&](int b, int t, float2 v) { Bf[b * C::LP + t] = v; }, tw);
  __syncthreads();
  const int hf = g.h;
  for (int q = threadIdx.x; q < C::B * n; q += C::NT) {
    const int b = q % C::B, i = q / C::B, k = k0 + b;
    if (k >= C::F) continue;
    const float2* zb = Bf + b * C::LP;
    float2 t = zb[i];
    if (i < hf) t = cadd(t, zb[C::L - 1 - i]);
    if (i >= n - hf) t = cadd(t, zb[2 * n - 1 - i]);
    T[(size_t)k * g.tpitch + i] = t;
  }
}

template <class C>
__global__ __launch_bounds__(C::NT) void fft_rows_mid_kernel(const float2* __restrict__ T,
                                                           FftGeom g, float2* __restrict__ S,
                                                           const Ctrl* ctrl) {
  if (fft_skip(ctrl)) return;
  extern __shared__ float2 fft_lds[];
  float2* tw = fft_lds;
  float2* A = tw + C::L;
  float2* Bf = A + C::B * C::LP;
  const int n = g.n, nl = (n + 1) / 2;
  const int grp = xcd_line_group((nl + C::B - 1) / C::B);
  if (grp < 0) return;
  const int line0 = grp * C::B;
  TwLoad<C::NT, C::TWN> ts;
  ts.load(g.tw, C::L);
  auto src = [&](int b, int kap) -> float2 {
    const int line = line0 + b, live = line < nl;
    const int ra = live ? 2 * line : -1, rb = live && 2 * line + 1 < n ? 2 * line + 1 : -1;
    return row_spectrum<C>(T, g.tpitch, ra, rb, kap);
  };
  // A p of the line's two rows (real, imaginary part) into A
  sh_transform<C, true>(src, A, Bf, [&](int b, int t, float2 v) { A[b * C::LP + t] = v; }, tw,
                        [&] { ts.store(tw, C::L); });
  __syncthreads();
  // columns >= n cut, re-padded; forward transform into Bf
  auto srcc = [&](int b, int t) -> float2 {
    const int line = line0 + b;
    float2 v = t < n ? A[b * C::LP + t] : make_float2(0.f, 0.f);
    if (2 * line + 1 >= n) v.y = 0.f;
    return v;
  };
  sh_transform<C, false>(srcc, Bf, A, [&](int b, int t, float2 v) { Bf[b * C::LP + t] = v; }, tw);
  __syncthreads();
  split_store<C>(Bf, line0, nl, n, S, g.spitch);
}

// Last row pass: the inverse transform of two rows, rows 0 .. n-1 of the
// result (with fold, the columns [-h, n+h) folded onto the image as in the
// column pass), plus lambda^2 p and the partials of p . w when p is given.
template <class C>
__global__ __launch_bounds__(C::NT) void fft_rows_out_kernel(
    const float2* __restrict__ T, FftGeom g, int fold, const float* __restrict__ p,
    float* __restrict__ w, float lam2, double* __restrict__ partials, const Ctrl* ctrl) {
  if (fft_skip(ctrl)) return;
  extern __shared__ float2 fft_lds[];
  __shared__ double sh[C::NT / 64];
  float2* tw = fft_lds;
  float2* A = tw + C::L;
  float2* Bf = A + C::B * C::LP;
  const int n = g.n, nl = (n + 1) / 2;
  const int grp = xcd_line_group((nl + C::B - 1) / C::B);
  if (grp < 0) return;
  const int line0 = grp * C::B;
  TwLoad<C::NT, C::TWN> ts;
  ts.load(g.tw, C::L);
  // the rows of p at this thread's outputs (element q: line q % B, column q / B)
  constexpr int OPT = (C::B * C::L + C::NT - 1) / C::NT;
  float pa[OPT], pb[OPT];
#pragma unroll
  for (int i = 0; i < OPT; ++i) {
    const int q = threadIdx.x + i * C::NT, b = q % C::B, j = q / C::B, line = line0 + b;
    const int ra = 2 * line, rb = ra + 1;
    const bool ok = p != nullptr && q < C::B * C::L && j < n && line < nl;
    pa[i] = ok ? p[(size_t)ra * n + j] : 0.f;
    pb[i] = (ok && rb < n) ? p[(size_t)rb * n + j] : 0.f;
  }
  auto src = [&](int b, int kap) -> float2 {
    const int line = line0 + b, live = line < nl;
    const int ra = live ? 2 * line : -1, rb = live && 2 * line + 1 < n ? 2 * line + 1 : -1;
    return row_spectrum<C>(T, g.tpitch, ra, rb, kap);
  };
  sh_transform<C, true>(src, A, Bf, [&](int b, int t, float2 v) { A[b * C::LP + t] = v; }, tw,
                        [&] { ts.store(tw, C::L); });
  __syncthreads();
  const int hf = fold ? g.h : 0;
  double dsum = 0.0;
#pragma unroll
  for (int i = 0; i < OPT; ++i) {
    const int q = threadIdx.x + i * C::NT, b = q % C::B, j = q / C::B, line = line0 + b;
    if (q >= C::B * C::L || j >= n || line >= nl) continue;
    const float2* zb = A + b * C::LP;
    float2 t = zb[j];
    if (j < hf) t = cadd(t, zb[C::L - 1 - j]);
    if (j >= n - hf) t = cadd(t, zb[2 * n - 1 - j]);
    const int ra = 2 * line, rb = ra + 1;
    const float wa = fmaf(lam2, pa[i], t.x);
    w[(size_t)ra * n + j] = wa;
    dsum += (double)pa[i] * (double)wa;
    if (rb < n) {
      const float wb = fmaf(lam2, pb[i], t.y);
      w[(size_t)rb * n + j] = wb;
      dsum += (double)pb[i] * (double)wb;
    }
  }
  const double tot = block_sum<C::NT>(dsum, sh);
  if (threadIdx.x == 0 && partials) partials[SLOT_DELTA * MAX_PARTIALS + grp] = tot;
}

// ---------------------------------------------------------------------------
// setup: twiddles and the PSF spectrum, in FP64
// ---------------------------------------------------------------------------
__global__ void fft_tw_kernel(int L, float2* __restrict__ tw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L) return;
  double s, c;
  sincospi(-2.0 * (double)t / (double)L, &s, &c);
  tw[t] = make_float2((float)c, (float)s);
}

// G[u][k] = sum_v P[h+u][h+v] exp(-2 pi i k v / L), u, v in [-h, h]
__global__ void fft_psf_rows_kernel(const double* __restrict__ psf, int K, int L, int F,
                                    double2* __restrict__ G) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * F) return;
  const int ui = idx / F, k = idx - ui * F, h = (K - 1) / 2;
  double re = 0.0, im = 0.0;
  for (int vi = 0; vi < K; ++vi) {
    const long t = ((long)k * (vi - h)) % L;
    double s, c;
    sincospi(-2.0 * (double)t / (double)L, &s, &c);
    const double pv = psf[ui * K + vi];
    re += pv * c;
    im += pv * s;
  }
  G[idx] = make_double2(re, im);
}

// Ht[k][m] = (1 / L^2) sum_u G[u][k] exp(-2 pi i m u / L)
__global__ void fft_psf_cols_kernel(const double2* __restrict__ G, int K, int L, int F,
                                    float2* __restrict__ Ht) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)F * L) return;
  const int k = (int)(idx / L), m = (int)(idx - (size_t)k * L), h = (K - 1) / 2;
  double re = 0.0, im = 0.0;
  for (int ui = 0; ui < K; ++ui) {
    const long t = ((long)m * (ui - h)) % L;
    double s, c;
    sincospi(-2.0 * (double)t / (double)L, &s, &c);
    const double2 gv = G[ui * F + k];
    re += gv.x * c - gv.y * s;
    im += gv.x * s + gv.y * c;
  }
  const double inv = 1.0 / ((double)L * (double)L);
  Ht[idx] = make_float2((float)(re * inv), (float)(im * inv));
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// the transform lengths L = R1 R2 R3 the kernels are built for (radices of
// the three Stockham stages), in increasing order; the largest covers the
// reflexive boundary's n + 2h at n = 2048, K = 63, and a plan that needs a
// longer one has no FFT form
#define KPCG_FFT_SIZES(X)                                                                      \
  X(4, 4, 4) X(4, 4, 6) X(4, 4, 8) X(4, 6, 6) X(4, 6, 8) X(4, 8, 8) X(4, 8, 10) X(6, 8, 8)    \
  X(6, 8, 10) X(6, 9, 10) X(7, 8, 10) X(8, 8, 9) X(7, 8, 12) X(8, 8, 12) X(7, 8, 16)          \
  X(8, 8, 15) X(8, 8, 16) X(7, 10, 15) X(8, 9, 15) X(8, 12, 12) X(9, 12, 12) X(10, 12, 12)    \
  X(10, 10, 16) X(12, 12, 12) X(10, 12, 16) X(12, 12, 14) X(10, 14, 15) X(12, 12, 15)

struct FftSize {
  int r1, r2, r3;
};
static constexpr FftSize kFftSizes[] = {
#define KPCG_FFT_ENTRY(a, b, c) {a, b, c},
    KPCG_FFT_SIZES(KPCG_FFT_ENTRY)
#undef KPCG_FFT_ENTRY
};

static int fft_menu_length(int need) {
  for (const FftSize& z : kFftSizes)
    if (z.r1 * z.r2 * z.r3 >= need) return z.r1 * z.r2 * z.r3;
  return -1;
}

// the zero boundary's length: every wrapped tap must land in the zero pad,
// L >= n + h
int fft_length(int n, int k) { return fft_menu_length(n + (k - 1) / 2); }

// the reflexive boundary's length: the image extended by h on each side
// convolved with the PSF must not wrap onto the image, L >= n + 2h
int fft_length_reflexive(int n, int k) { return fft_menu_length(n + 2 * ((k - 1) / 2)); }

int fft_table_length(int n, int k) {
  const int a = fft_length(n, k), b = fft_length_reflexive(n, k);
  const int m = a > b ? a : b;
  return m > 0 ? m : 0;
}

// the radices of L's three stages, or -1
int fft_radices(int L, int* rad) {
  for (const FftSize& z : kFftSizes)
    if (z.r1 * z.r2 * z.r3 == L) {
      rad[0] = z.r1;
      rad[1] = z.r2;
      rad[2] = z.r3;
      return 3;
    }
  return -1;
}

static FftGeom geom(const Plan& P) {
  FftGeom g;
  g.n = P.n;
  g.L = P.fft_L;
  g.F = P.fft_L / 2 + 1;
  g.tw = reinterpret_cast<const float2*>(P.fft_tw);
  g.refl = P.bc == KP_BC_REFLEXIVE ? 1 : 0;
  g.h = (P.k - 1) / 2;
  // S holds every row slot of the reflexive extension
  g.spitch = P.n + 2 * g.h;
  g.tpitch = P.n;
  return g;
}

hipError_t build_fft_tables(const Plan& P, const double* psf_dev, void* g_scratch,
                            hipStream_t s) {
  if (P.fft_L <= 0) return hipSuccess;     // no FFT form at this size
  const int L = P.fft_L, F = L / 2 + 1, K = P.k;
  hipLaunchKernelGGL(fft_tw_kernel, dim3((L + 255) / 256), dim3(256), 0, s, L,
                     reinterpret_cast<float2*>(P.fft_tw));
  double2* G = reinterpret_cast<double2*>(g_scratch);
  hipLaunchKernelGGL(fft_psf_rows_kernel, dim3((K * F + 255) / 256), dim3(256), 0, s, psf_dev,
                     K, L, F, G);
  const size_t tot = (size_t)F * L;
  hipLaunchKernelGGL(fft_psf_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     G, K, L, F, reinterpret_cast<float2*>(P.fft_Ht));
  return hipGetLastError();
}

// the dynamic LDS above 64 KB is granted once per kernel
template <class Kern>
static hipError_t grant_lds(Kern kern, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// mode 0: w = A^T A p + lam2 p (all five passes); mode 1: w = A^T p (the
// row pass of p, the column pass with conj Hc, the last row pass)
template <class C>
static hipError_t run_fft(const Plan& P, const FftGeom& g, int mode, const float* p, float* w,
                          float lam2, double* partials, const Ctrl* ctrl, int* nb,
                          const DirStep* dir, hipStream_t s) {
  static bool granted = false;
  if (!granted) {
    hipError_t e = grant_lds(fft_rows_fwd_kernel<C>, C::LDS);
    if (e == hipSuccess) e = grant_lds(fft_rows_fwd_dir_kernel<C>, C::LDS);
    if (e == hipSuccess) e = grant_lds(fft_cols_kernel<C>, C::LDS);
    if (e == hipSuccess) e = grant_lds(fft_rows_mid_kernel<C>, C::LDS);
    if (e == hipSuccess) e = grant_lds(fft_rows_out_kernel<C>, C::LDS);
    if (e != hipSuccess) return e;
    granted = true;
  }
  float2* S = reinterpret_cast<float2*>(P.fft_S);
  float2* T = reinterpret_cast<float2*>(P.fft_T);
  const float2* Ht = reinterpret_cast<const float2*>(P.fft_Ht);
  const int n = g.n;
  const int ext = (mode == 0 && g.refl) ? 1 : 0;
  const int rows_in = ext ? n + 2 * g.h : n;
  const int gr_in = ((rows_in + 1) / 2 + C::B - 1) / C::B;
  const int gr = ((n + 1) / 2 + C::B - 1) / C::B;
  auto pad8 = [](int v) { return (v + 7) / 8 * 8; };
  const int gc = (C::F + C::B - 1) / C::B;
  if (dir != nullptr)
    hipLaunchKernelGGL(fft_rows_fwd_dir_kernel<C>, dim3(pad8(gr_in)), dim3(C::NT), C::LDS, s,
                       const_cast<float*>(p), g, S, *dir);
  else
    hipLaunchKernelGGL(fft_rows_fwd_kernel<C>, dim3(pad8(gr_in)), dim3(C::NT), C::LDS, s, p, g,
                       ext, S, ctrl);
  if (mode == 0) {
    hipLaunchKernelGGL(fft_cols_kernel<C>, dim3(gc), dim3(C::NT), C::LDS, s, S, g, rows_in,
                       ext ? g.h : 0, Ht, 0, 0, T, ctrl);
    hipLaunchKernelGGL(fft_rows_mid_kernel<C>, dim3(pad8(gr)), dim3(C::NT), C::LDS, s, T, g, S, ctrl);
  }
  hipLaunchKernelGGL(fft_cols_kernel<C>, dim3(gc), dim3(C::NT), C::LDS, s, S, g, n, 0, Ht, 1,
                     g.refl, T, ctrl);
  hipLaunchKernelGGL(fft_rows_out_kernel<C>, dim3(pad8(gr)), dim3(C::NT), C::LDS, s, T, g, g.refl,
                     mode == 0 ? p : nullptr, w, lam2, partials, ctrl);
  if (nb) *nb = gr;
  return hipGetLastError();
}

static hipError_t dispatch_fft(const Plan& P, int mode, const float* p, float* w, float lam2,
                               double* partials, const Ctrl* ctrl, int* nb, const DirStep* dir,
                               hipStream_t s) {
  const FftGeom g = geom(P);
#define KPCG_FFT_CASE(a, b, c)                                                   \
  if (P.fft_rad[0] == a && P.fft_rad[1] == b && P.fft_rad[2] == c && g.L == a * b * c) \
    return run_fft<Sh3<a, b, c>>(P, g, mode, p, w, lam2, partials, ctrl, nb, dir, s);
  KPCG_FFT_SIZES(KPCG_FFT_CASE)
#undef KPCG_FFT_CASE
  return hipErrorInvalidValue;
}

// w = A^T A p + lam2 p with the partials of p . w (with_partials).  Zero
// boundary: the plain passes.  Reflexive boundary: the first row pass
// extends p by reflection (n + 2h row slots), the first column pass reads
// them, and the passes of A^T fold the correlation back onto the image.
hipError_t launch_fft_normal(const Plan& P, const float* p, float* w, float lam2, hipStream_t s,
                             int* nb, const Ctrl* ctrl, bool with_partials) {
  return dispatch_fft(P, 0, p, w, lam2, with_partials ? P.partials : nullptr, ctrl, nb, nullptr,
                      s);
}

// The iteration's matvec half with the direction step before it: p = z +
// beta p in the first row pass (beta from the nbz partials of r.z and z.Hp
// of the preconditioner's last GEMM; publishes), then w = A^T A p + lam2 p
// with the partials of p . w (zero boundary only: each element of p is read
// by one thread).
hipError_t launch_fft_normal_dir(const Plan& P, float lam2, int nbz, hipStream_t s, int* nb) {
  if (P.bc != KP_BC_ZERO || nbz > MAX_PARTIALS) return hipErrorInvalidValue;
  DirStep d;
  d.z = P.z;
  d.ctrl = P.ctrl;
  d.partials = P.partials;
  d.nbz = nbz;
  d.mirror = P.mirror_dev;
  return dispatch_fft(P, 0, P.p, P.w, lam2, P.partials, P.ctrl, nb, &d, s);
}

// out = A^T u alone; no control-block test, no partials.
hipError_t launch_fft_at(const Plan& P, const float* u, float* out, hipStream_t s) {
  return dispatch_fft(P, 1, u, out, 0.0f, nullptr, nullptr, nullptr, nullptr, s);
}

// ---------------------------------------------------------------------------
// A blur epilogue (blur_core.h) applied to a dense n x n result v, element
// by element, with the per-block partial sums of its reduction: the FFT
// forms of the right-hand side and of the true residuals use the blurs'
// epilogues unchanged.
// ---------------------------------------------------------------------------
constexpr int EPI_T = 256, EPI_MAXB = 1024;

template <class Epi>
__global__ __launch_bounds__(EPI_T) void epi_dense_kernel(const float* __restrict__ v, int n,
                                                          Epi epi, double* __restrict__ partials) {
  const int N = n * n;
  double d = 0.0;
  for (int o = blockIdx.x * EPI_T + threadIdx.x; o < N; o += gridDim.x * EPI_T) {
    const int i = o / n, j = o - i * n;
    const float val = v[o];
    epi.row(i, j, 1, &val, d);
  }
  if constexpr (Epi::kReduce) {
    __shared__ double sh[EPI_T / 64];
    const double t = block_sum<EPI_T>(d, sh);
    if (threadIdx.x == 0) partials[Epi::kSlot * MAX_PARTIALS + blockIdx.x] = t;
  }
}

template <class Epi>
static hipError_t epi_dense(const Plan& P, const float* v, Epi epi, hipStream_t s, int* nb) {
  const int N = P.n * P.n;
  int b = (N + EPI_T - 1) / EPI_T;
  b = b > EPI_MAXB ? EPI_MAXB : b;
  hipLaunchKernelGGL(epi_dense_kernel<Epi>, dim3(b), dim3(EPI_T), 0, s, v, P.n, epi, P.partials);
  *nb = b;
  return hipGetLastError();
}

// r = c = A^T b, ||c||^2 (the SC_RHS step); p = w (= x) = 0: launch_rhs by FFTs
hipError_t launch_fft_rhs(const Plan& P, const float* b, bool zero_x, hipStream_t s) {
  hipError_t e = launch_fft_at(P, b, P.q, s);
  if (e != hipSuccess) return e;
  int nb;
  e = epi_dense(P, P.q, EpiRhs{P.r, P.n, P.p, P.w, zero_x ? P.x64 : nullptr}, s, &nb);
  if (e != hipSuccess) return e;
  return launch_scalar(P, SC_RHS, nb, s);
}

// r = A^T u - lam2 x from u = b - A x already in P.q (FP32), with the anchor
// recorded; A^T u by FFTs into P.z
hipError_t launch_fft_true_res(const Plan& P, double lam2, bool fin, hipStream_t s) {
  hipError_t e = launch_fft_at(P, P.q, P.z, s);
  if (e != hipSuccess) return e;
  int nb;
  e = epi_dense(P, P.z, EpiTrueRes{P.x64, P.r, lam2, P.n, P.xa64, P.ra64}, s, &nb);
  if (e != hipSuccess) return e;
  return launch_scalar(P, fin ? SC_TRUE : SC_TRUE_INFO, nb, s);
}

// r = r_a - H (x - x_a) from the anchor, A^T A of fp32(x - x_a) by FFTs
hipError_t launch_fft_anchor_residual(const Plan& P, double lam2, bool fin, hipStream_t s) {
  hipError_t e = launch_diff32(P, P.q, s);
  if (e != hipSuccess) return e;
  e = launch_fft_normal(P, P.q, P.z, 0.0f, s, nullptr, nullptr, false);
  if (e != hipSuccess) return e;
  int nb;
  e = epi_dense(P, P.z, EpiAnchorRes{P.x64, P.xa64, P.ra64, P.r, lam2, P.n}, s, &nb);
  if (e != hipSuccess) return e;
  return launch_scalar(P, fin ? SC_TRUE : SC_TRUE_INFO, nb, s);
}

}  // namespace kpcg
