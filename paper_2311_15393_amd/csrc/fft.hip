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
// L is the smallest even size >= n + h whose prime factors are 2, 3, 5, 7.
//
// Five passes, each one workgroup per line with the line in LDS:
//   rows_fwd  two real rows of p packed as one complex row (x_a + i x_b),
//             one length-L transform, split into the two half spectra
//             (k = 0 .. L/2) -> S [n][F], F = L/2 + 1
//   cols      one column k of S: transform, times Hc[:, k] / L^2, inverse
//             transform, rows 0 .. n-1 kept -> T
//   rows_mid  two rows of T: Hermitian extension packed as one complex
//             spectrum, inverse transform (real part row a, imaginary part
//             row b: A p), columns 0 .. n-1 kept and re-padded, forward
//             transform, split -> S (the half spectra of A p)
//   cols      with conj(Hc) -> T
//   rows_out  inverse as rows_mid, w = result + lambda^2 p on the n x n
//             window, and the per-workgroup partial sum of p . w.
// The inverse transforms use IDFT(Y) = conj(DFT(conj(Y))) / L with the 1/L^2
// folded into the stored Hc.  Each 1-D transform is a Stockham autosort FFT
// in LDS (ping-pong buffers) over the radices 8, 4, 2, 3, 5, 7, with
// twiddles from an FP32 table of exp(-2 pi i t / L) built in FP64.
#include <cmath>

#include "blur_core.h"

namespace kpcg {

constexpr int FT = 256;                 // threads per FFT workgroup

struct FftGeom {
  int n, L, F, nrad;
  int rad[FFT_MAX_RADICES];
  const float2* tw;                     // exp(-2 pi i t / L), t < L
  int refl, h;                          // reflexive boundary; PSF half-width
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

// forward DFTs of length R (W = exp(-2 pi i / R)) in place
__device__ inline void dft2(float2* v) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
__device__ inline void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
  const float2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3),
               a3 = mul_mi(csub(v1, v3));
  v0 = cadd(a0, a2);
  v1 = cadd(a1, a3);
  v2 = csub(a0, a2);
  v3 = csub(a1, a3);
}
__device__ inline void dft8(float2* v) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  constexpr float r = 0.70710678118654752f;
  // o_k *= exp(-i pi k / 4)
  o1 = make_float2(r * (o1.x + o1.y), r * (o1.y - o1.x));
  o2 = mul_mi(o2);
  o3 = make_float2(r * (o3.y - o3.x), -r * (o3.x + o3.y));
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}
// odd R: with A_k = v_k + v_{R-k}, B_k = v_k - v_{R-k} (k = 1 .. (R-1)/2),
// X_m = v_0 + sum_k cos(2 pi m k / R) A_k -/+ i sum_k sin(2 pi m k / R) B_k
// for m and R - m
template <int R>
__device__ inline void dft_odd(float2* v, const float (*C)[4], const float (*S)[4]) {
  constexpr int H = (R - 1) / 2;
  float2 A[H], B[H];
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    A[k - 1] = cadd(v[k], v[R - k]);
    B[k - 1] = csub(v[k], v[R - k]);
  }
  float2 x0 = v[0];
#pragma unroll
  for (int k = 0; k < H; ++k) x0 = cadd(x0, A[k]);
  float2 out[R];
  out[0] = x0;
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    float2 re = v[0], im = make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      re.x = fmaf(C[m][k], A[k - 1].x, re.x);
      re.y = fmaf(C[m][k], A[k - 1].y, re.y);
      im.x = fmaf(S[m][k], B[k - 1].x, im.x);
      im.y = fmaf(S[m][k], B[k - 1].y, im.y);
    }
    out[m] = cadd(re, mul_mi(im));          // re - i im
    out[R - m] = csub(re, mul_mi(im));      // re + i im
  }
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = out[m];
}
// cos / sin (2 pi m k / R), indices [m][k], m, k <= 3
__constant__ float kC3[4][4] = {{1, 1, 1, 1}, {1, -0.5f, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
__constant__ float kS3[4][4] = {{0, 0, 0, 0}, {0, 0.86602540378443865f, 0, 0}, {0, 0, 0, 0},
                                {0, 0, 0, 0}};
__constant__ float kC5[4][4] = {{1, 1, 1, 1},
                                {1, 0.30901699437494742f, -0.80901699437494742f, 0},
                                {1, -0.80901699437494742f, 0.30901699437494742f, 0},
                                {0, 0, 0, 0}};
__constant__ float kS5[4][4] = {{0, 0, 0, 0},
                                {0, 0.95105651629515357f, 0.58778525229247313f, 0},
                                {0, 0.58778525229247313f, -0.95105651629515357f, 0},
                                {0, 0, 0, 0}};
__constant__ float kC7[4][4] = {
    {1, 1, 1, 1},
    {1, 0.62348980185873353f, -0.22252093395631440f, -0.90096886790241913f},
    {1, -0.22252093395631440f, -0.90096886790241913f, 0.62348980185873353f},
    {1, -0.90096886790241913f, 0.62348980185873353f, -0.22252093395631440f}};
__constant__ float kS7[4][4] = {
    {0, 0, 0, 0},
    {0, 0.78183148246802981f, 0.97492791218182361f, 0.43388373911755812f},
    {0, 0.97492791218182361f, -0.43388373911755812f, -0.78183148246802981f},
    {0, 0.43388373911755812f, -0.78183148246802981f, 0.97492791218182361f}};

// One radix-R Stockham stage over the whole line: in -> out (tw: the
// twiddle table in LDS).
template <int R>
__device__ inline void fft_stage(const float2* __restrict__ in, float2* __restrict__ out,
                                 const float2* __restrict__ tw, int L, int Ns) {
  const int Ls = L / R;
  const int step = L / (Ns * R);
  for (int j = threadIdx.x; j < Ls; j += FT) {
    const int k = j % Ns;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[j + r * Ls];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[k * r * step]);
    }
    if constexpr (R == 2) dft2(v);
    else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8(v);
    else if constexpr (R == 3) dft_odd<3>(v, kC3, kS3);
    else if constexpr (R == 5) dft_odd<5>(v, kC5, kS5);
    else dft_odd<7>(v, kC7, kS7);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[base + r * Ns] = v[r];
  }
}

// Forward DFT of the line in a (length g.L), b as the second buffer, with
// the twiddle table tw in LDS.  Returns the buffer holding the result.
// Ends with a barrier.
__device__ inline float2* fft_line(float2* a, float2* b, const float2* tw, const FftGeom& g) {
  int Ns = 1;
  for (int s = 0; s < g.nrad; ++s) {
    const int R = g.rad[s];
    switch (R) {
      case 8: fft_stage<8>(a, b, tw, g.L, Ns); break;
      case 4: fft_stage<4>(a, b, tw, g.L, Ns); break;
      case 2: fft_stage<2>(a, b, tw, g.L, Ns); break;
      case 3: fft_stage<3>(a, b, tw, g.L, Ns); break;
      case 5: fft_stage<5>(a, b, tw, g.L, Ns); break;
      default: fft_stage<7>(a, b, tw, g.L, Ns); break;
    }
    __syncthreads();
    float2* t = a; a = b; b = t;
    Ns *= R;
  }
  return a;
}

__device__ inline bool fft_skip(const Ctrl* ctrl) { return ctrl != nullptr && ctrl->done != RUNNING; }

// Split the transform Z of x_a + i x_b into the half spectra of the two real
// rows: X_a = (Z_k + conj Z_{L-k}) / 2, X_b = (Z_k - conj Z_{L-k}) / (2 i).
__device__ inline void split_store(const float2* Z, int L, int F, float2* Sa, float2* Sb) {
  for (int k = threadIdx.x; k < F; k += FT) {
    const float2 z = Z[k];
    const float2 zr = cconj(Z[k == 0 ? 0 : L - k]);
    Sa[k] = cscale(cadd(z, zr), 0.5f);
    if (Sb) Sb[k] = cscale(mul_mi(csub(z, zr)), 0.5f);
  }
}

// Every kernel issues all of its global loads (its line, the twiddle table,
// and the PSF spectrum column or the p rows it needs at the end) before it
// waits for any of them, then works in LDS: a line of L <= FFT_MAX_L points
// is FE elements per thread.
constexpr int FE = (FFT_MAX_L + FT - 1) / FT;

// the twiddle table into registers (issued), then into LDS (tw_lds)
struct TwStage {
  float2 v[FE];
  __device__ void load(const float2* __restrict__ tw, int L) {
#pragma unroll
    for (int e = 0; e < FE; ++e) {
      const int t = threadIdx.x + e * FT;
      if (t < L) v[e] = tw[t];
    }
  }
  __device__ void store(float2* tw_lds, int L) const {
#pragma unroll
    for (int e = 0; e < FE; ++e) {
      const int t = threadIdx.x + e * FT;
      if (t < L) tw_lds[t] = v[e];
    }
  }
};

// Row pass of the forward transform.  Plain (ext = 0): rows 0 .. n-1 of p,
// zero-padded to L.  Extended (ext = 1, reflexive boundary): the image
// extended by half-sample reflection over the rows and columns [-h, n+h):
// row slot s of S holds image row refl(s - h), and a column index j in
// [-h, 0) sits at the circular position L + j.
__global__ __launch_bounds__(FT) void fft_rows_fwd_kernel(const float* __restrict__ p, FftGeom g,
                                                          int ext, float2* __restrict__ S,
                                                          const Ctrl* ctrl) {
  if (fft_skip(ctrl)) return;
  extern __shared__ float2 fft_lds[];
  float2* a = fft_lds;
  float2* b = fft_lds + g.L;
  float2* tw = fft_lds + 2 * g.L;
  const int n = g.n, L = g.L, h = ext ? g.h : 0;
  const int rows = n + 2 * h, ra = 2 * blockIdx.x, rb = ra + 1;
  const int sa = ext ? refl_index(ra - h, n) : ra;
  const int sb = rb < rows ? (ext ? refl_index(rb - h, n) : rb) : -1;
  TwStage ts;
  ts.load(g.tw, L);
  float2 v[FE];
#pragma unroll
  for (int e = 0; e < FE; ++e) {
    const int c = threadIdx.x + e * FT;
    v[e] = make_float2(0.f, 0.f);
    const int j = c >= L - h ? c - L : c;          // column of circular position c
    if (c < L && j >= -h && j < n + h) {
      const int jj = ext ? refl_index(j, n) : j;
      v[e].x = p[(size_t)sa * n + jj];
      if (sb >= 0) v[e].y = p[(size_t)sb * n + jj];
    }
  }
  ts.store(tw, L);
#pragma unroll
  for (int e = 0; e < FE; ++e) {
    const int j = threadIdx.x + e * FT;
    if (j < L) a[j] = v[e];
  }
  __syncthreads();
  const float2* Z = fft_line(a, b, tw, g);
  split_store(Z, L, g.F, S + (size_t)ra * g.F, sb >= 0 ? S + (size_t)rb * g.F : nullptr);
}

// Columns: consecutive workgroups go to different XCDs (round robin), so the
// column index is chosen to give each XCD a contiguous range of columns:
// neighbouring columns share cache lines of S and T.
__device__ inline int xcd_column(int bid, int F) {
  const int per = (F + 7) / 8;
  const int k = (bid & 7) * per + (bid >> 3);
  return k;
}

// Column pass: the column k of S (its in_rows row slots, slot s at the
// circular row position s - in_off, the rest zero), its transform times the
// PSF spectrum (or its conjugate), the inverse; rows 0 .. n-1 kept, or with
// fold (the correlation of the reflexive boundary's A^T) the rows [-h, n+h)
// folded onto the image by the reflection: row a gains rows -1-a (circular
// L-1-a, for a < h) and 2n-1-a (for a >= n-h).
__global__ __launch_bounds__(FT) void fft_cols_kernel(const float2* __restrict__ S, FftGeom g,
                                                      int in_rows, int in_off,
                                                      const float2* __restrict__ Ht, int conjH,
                                                      int fold, float2* __restrict__ T,
                                                      const Ctrl* ctrl) {
  if (fft_skip(ctrl)) return;
  const int k = xcd_column(blockIdx.x, g.F);
  if (k >= g.F) return;
  extern __shared__ float2 fft_lds[];
  const int n = g.n, L = g.L, F = g.F;
  float2* a = fft_lds;
  float2* b = fft_lds + L;
  float2* tw = fft_lds + 2 * L;
  TwStage ts;
  ts.load(g.tw, L);
  // the column and the PSF spectrum column
  const float2* h = Ht + (size_t)k * L;
  float2 v[FE], hv[FE];
#pragma unroll
  for (int e = 0; e < FE; ++e) {
    const int c = threadIdx.x + e * FT;
    v[e] = make_float2(0.f, 0.f);
    const int sl = (c >= L - in_off ? c - L : c) + in_off;   // row slot of circular row c
    if (c < L && sl >= 0 && sl < in_rows) v[e] = S[(size_t)sl * F + k];
    if (c < L) hv[e] = h[c];
  }
  ts.store(tw, L);
#pragma unroll
  for (int e = 0; e < FE; ++e) {
    const int i = threadIdx.x + e * FT;
    if (i < L) a[i] = v[e];
  }
  __syncthreads();
  float2* Y = fft_line(a, b, tw, g);
  float2* other = Y == a ? b : a;
  // the spectrum times Hc (or conj Hc), conjugated for the inverse transform;
  // element m of Y belongs to the thread that loaded hv for m
#pragma unroll
  for (int e = 0; e < FE; ++e) {
    const int m = threadIdx.x + e * FT;
    if (m < L) {
      float2 hm = hv[e];
      if (conjH) hm.y = -hm.y;
      Y[m] = cconj(cmul(Y[m], hm));
    }
  }
  __syncthreads();
  const float2* y = fft_line(Y, other, tw, g);
  const int hf = fold ? g.h : 0;
  for (int i = threadIdx.x; i < n; i += FT) {
    float2 t = y[i];
    if (i < hf) t = cadd(t, y[L - 1 - i]);
    if (i >= n - hf) t = cadd(t, y[2 * n - 1 - i]);
    T[(size_t)i * F + k] = cconj(t);
  }
}

// conj of the full spectrum of x_a + i x_b from the half spectra held in
// registers (ta, tb: element j of thread t is k = t + j FT, k < F) into out
// (Hermitian extension), ready for IDFT(Z) = conj(DFT(conj Z)): out[k] for
// k < F and out[L - k] for 0 < k < L - F + 1... written by the owner of k.
__device__ inline void pack_conj_regs(const float2 (&ta)[FE], const float2 (&tb)[FE], bool has_b,
                                      int L, int F, float2* out) {
#pragma unroll
  for (int e = 0; e < FE; ++e) {
    const int k = threadIdx.x + e * FT;
    if (k < F) {
      const float2 a = ta[e], bb = has_b ? tb[e] : make_float2(0.f, 0.f);
      // Z_k = a + i b; conj(Z_k)
      out[k] = cconj(make_float2(a.x - bb.y, a.y + bb.x));
      // Z_{L-k} = conj a + i conj b (for 0 < k, L - k >= F)
      if (k > 0 && L - k >= F) out[L - k] = cconj(make_float2(a.x + bb.y, bb.x - a.y));
    }
  }
}

__device__ inline void load_half_rows(const float2* __restrict__ T, int ra, int rb, int n, int F,
                                      float2 (&ta)[FE], float2 (&tb)[FE]) {
#pragma unroll
  for (int e = 0; e < FE; ++e) {
    const int k = threadIdx.x + e * FT;
    if (k < F) {
      ta[e] = T[(size_t)ra * F + k];
      tb[e] = rb < n ? T[(size_t)rb * F + k] : make_float2(0.f, 0.f);
    }
  }
}

__global__ __launch_bounds__(FT) void fft_rows_mid_kernel(const float2* __restrict__ T,
                                                          FftGeom g, float2* __restrict__ S,
                                                          const Ctrl* ctrl) {
  if (fft_skip(ctrl)) return;
  extern __shared__ float2 fft_lds[];
  const int n = g.n, L = g.L, F = g.F, ra = 2 * blockIdx.x, rb = ra + 1;
  float2* a = fft_lds;
  float2* b = fft_lds + L;
  float2* tw = fft_lds + 2 * L;
  TwStage ts;
  ts.load(g.tw, L);
  float2 ta[FE], tb[FE];
  load_half_rows(T, ra, rb, n, F, ta, tb);
  ts.store(tw, L);
  pack_conj_regs(ta, tb, rb < n, L, F, a);
  __syncthreads();
  float2* z = fft_line(a, b, tw, g);
  // conj(z) = A p rows ra (real) and rb (imaginary); keep j < n, re-pad
  for (int j = threadIdx.x; j < L; j += FT) {
    float2 v = make_float2(0.f, 0.f);
    if (j < n) {
      v = cconj(z[j]);
      if (rb >= n) v.y = 0.f;
    }
    z[j] = v;
  }
  __syncthreads();
  float2* other = z == a ? b : a;
  const float2* Z = fft_line(z, other, tw, g);
  split_store(Z, L, F, S + (size_t)ra * F, rb < n ? S + (size_t)rb * F : nullptr);
}

// Last row pass: the inverse transform of two rows, rows 0 .. n-1 of the
// result (with fold, the columns [-h, n+h) folded onto the image as in the
// column pass), plus lambda^2 p and the partials of p . w when p is given.
__global__ __launch_bounds__(FT) void fft_rows_out_kernel(const float2* __restrict__ T, FftGeom g,
                                                          int fold, const float* __restrict__ p,
                                                          float* __restrict__ w, float lam2,
                                                          double* __restrict__ partials,
                                                          const Ctrl* ctrl) {
  if (fft_skip(ctrl)) return;
  extern __shared__ float2 fft_lds[];
  __shared__ double sh[FT / 64];
  const int n = g.n, L = g.L, F = g.F, ra = 2 * blockIdx.x, rb = ra + 1;
  float2* a = fft_lds;
  float2* b = fft_lds + L;
  float2* tw = fft_lds + 2 * L;
  TwStage ts;
  ts.load(g.tw, L);
  float2 ta[FE], tb[FE];
  load_half_rows(T, ra, rb, n, F, ta, tb);
  // the two rows of p for lambda^2 p and p . w
  float pa[FE], pb[FE];
#pragma unroll
  for (int e = 0; e < FE; ++e) {
    const int j = threadIdx.x + e * FT;
    pa[e] = 0.f;
    pb[e] = 0.f;
    if (p != nullptr && j < n) {
      pa[e] = p[(size_t)ra * n + j];
      pb[e] = rb < n ? p[(size_t)rb * n + j] : 0.f;
    }
  }
  ts.store(tw, L);
  pack_conj_regs(ta, tb, rb < n, L, F, a);
  __syncthreads();
  const float2* z = fft_line(a, b, tw, g);
  const int hf = fold ? g.h : 0;
  double d = 0.0;
#pragma unroll
  for (int e = 0; e < FE; ++e) {
    const int j = threadIdx.x + e * FT;
    if (j < n) {
      float2 zt = z[j];
      if (j < hf) zt = cadd(zt, z[L - 1 - j]);
      if (j >= n - hf) zt = cadd(zt, z[2 * n - 1 - j]);
      const float2 v = cconj(zt);
      const size_t oa = (size_t)ra * n + j;
      const float wa = fmaf(lam2, pa[e], v.x);
      w[oa] = wa;
      d += (double)pa[e] * (double)wa;
      if (rb < n) {
        const float wb = fmaf(lam2, pb[e], v.y);
        w[oa + n] = wb;
        d += (double)pb[e] * (double)wb;
      }
    }
  }
  const double tot = block_sum<FT>(d, sh);
  if (threadIdx.x == 0 && partials) partials[SLOT_DELTA * MAX_PARTIALS + blockIdx.x] = tot;
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
int fft_length(int n, int k) {
  const int h = (k - 1) / 2;
  for (int L = n + h + ((n + h) & 1);; L += 2) {
    int r = L;
    for (int f : {2, 3, 5, 7})
      while (r % f == 0) r /= f;
    if (r == 1) return L;
  }
}

// the reflexive boundary's length: the image extended by h on each side
// convolved with the PSF must not wrap onto the image, L >= n + 2h
int fft_length_reflexive(int n, int k) { return fft_length(n + (k - 1) / 2, k); }

int fft_radices(int L, int* rad) {
  int m = L, c = 0;
  while (m % 8 == 0) { rad[c++] = 8; m /= 8; }
  while (m % 4 == 0) { rad[c++] = 4; m /= 4; }
  while (m % 2 == 0) { rad[c++] = 2; m /= 2; }
  for (int f : {3, 5, 7})
    while (m % f == 0) { rad[c++] = f; m /= f; }
  return m == 1 ? c : -1;
}

static FftGeom geom(const Plan& P) {
  FftGeom g;
  g.n = P.n;
  g.L = P.fft_L;
  g.F = P.fft_L / 2 + 1;
  g.nrad = P.fft_nrad;
  for (int i = 0; i < FFT_MAX_RADICES; ++i) g.rad[i] = i < P.fft_nrad ? P.fft_rad[i] : 1;
  g.tw = reinterpret_cast<const float2*>(P.fft_tw);
  g.refl = P.bc == KP_BC_REFLEXIVE ? 1 : 0;
  g.h = (P.k - 1) / 2;
  return g;
}

hipError_t build_fft_tables(const Plan& P, const double* psf_dev, void* g_scratch,
                            hipStream_t s) {
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

size_t fft_lds_bytes(int L) { return (size_t)3 * L * sizeof(float2); }   // a, b, twiddles

// w = A^T A p + lam2 p with the partials of p . w (with_partials).  Zero
// boundary: the plain passes.  Reflexive boundary: the first row pass
// extends p by reflection (n + 2h row slots), the first column pass reads
// them, and the passes of A^T fold the correlation back onto the image.
hipError_t launch_fft_normal(const Plan& P, const float* p, float* w, float lam2, hipStream_t s,
                             int* nb, const Ctrl* ctrl, bool with_partials) {
  const FftGeom g = geom(P);
  const size_t lds = fft_lds_bytes(g.L);        // <= 3 * FFT_MAX_L * 8 B = 55.3 KB
  float2* S = reinterpret_cast<float2*>(P.fft_S);
  float2* T = reinterpret_cast<float2*>(P.fft_T);
  const float2* Ht = reinterpret_cast<const float2*>(P.fft_Ht);
  const int ext_rows = g.refl ? g.n + 2 * g.h : g.n;
  const int rows = (g.n + 1) / 2;
  const int cols = ((g.F + 7) / 8) * 8;
  hipLaunchKernelGGL(fft_rows_fwd_kernel, dim3((ext_rows + 1) / 2), dim3(FT), lds, s, p, g,
                     g.refl, S, ctrl);
  hipLaunchKernelGGL(fft_cols_kernel, dim3(cols), dim3(FT), lds, s, S, g, ext_rows,
                     g.refl ? g.h : 0, Ht, 0, 0, T, ctrl);
  hipLaunchKernelGGL(fft_rows_mid_kernel, dim3(rows), dim3(FT), lds, s, T, g, S, ctrl);
  hipLaunchKernelGGL(fft_cols_kernel, dim3(cols), dim3(FT), lds, s, S, g, g.n, 0, Ht, 1, g.refl,
                     T, ctrl);
  hipLaunchKernelGGL(fft_rows_out_kernel, dim3(rows), dim3(FT), lds, s, T, g, g.refl, p, w, lam2,
                     with_partials ? P.partials : nullptr, ctrl);
  if (nb) *nb = rows;
  return hipGetLastError();
}

// out = A^T u alone (the last three passes of the normal operator, the row
// pass on u zero-padded); no control-block test, no partials.
hipError_t launch_fft_at(const Plan& P, const float* u, float* out, hipStream_t s) {
  const FftGeom g = geom(P);
  const size_t lds = fft_lds_bytes(g.L);
  float2* S = reinterpret_cast<float2*>(P.fft_S);
  float2* T = reinterpret_cast<float2*>(P.fft_T);
  const float2* Ht = reinterpret_cast<const float2*>(P.fft_Ht);
  const int rows = (g.n + 1) / 2;
  const int cols = ((g.F + 7) / 8) * 8;
  hipLaunchKernelGGL(fft_rows_fwd_kernel, dim3(rows), dim3(FT), lds, s, u, g, 0, S,
                     (const Ctrl*)nullptr);
  hipLaunchKernelGGL(fft_cols_kernel, dim3(cols), dim3(FT), lds, s, S, g, g.n, 0, Ht, 1, g.refl,
                     T, (const Ctrl*)nullptr);
  hipLaunchKernelGGL(fft_rows_out_kernel, dim3(rows), dim3(FT), lds, s, T, g, g.refl,
                     (const float*)nullptr, out, 0.0f, (double*)nullptr, (const Ctrl*)nullptr);
  return hipGetLastError();
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
