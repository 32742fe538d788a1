// Extended-precision pipelines (double-double and quad-double) for 2D and 3D
// distance fields.
//
// The same zero-padded FFT convolution as the float32/float64 paths
// (Sec. 3, Table 1: splat the indicator, transform, multiply by the kernel
// spectrum, transform back, S = -tau log phi of eq. STilde), carried in an
// extended real type R so that the FFT's absolute error floor drops from
// about 2^-53 of the largest term to 2^-104 (R = dd, pairs of float64) or
// 2^-208 (R = qd, four float64 parts).  Sec. 3.2 observes that the float64
// convolution fails far from the sources for small tau and resorts to
// multiple-precision arithmetic; these pipelines play that role on the GPU.
// Every kernel below is a template over R; the exported launchers pick the
// instantiation from DDGeom::quad.
//
// Layout in the plan's workspace (x fastest, M = padded lengths; 2D):
//   twx, twy  M/2 complex twiddles exp(-2 pi i k / M) in R
//   tabs      C spectra, My x Mx values of R each, scaled by 1/(Mx My): the
//             real spectrum of f, then the imaginary parts of the gradient
//             kernels' (C = 3 when the gradient is prepared)
//   cnt       ny x nx float64 multiplicities (the indicator g)
//   G         My x Mx complex work grid in R (row spectra)
//   Gc        C x ny x Mx complex values in R (column-pass outputs)
// 3D plans add twz, take Mz x My x Mx spectra (C = 4 with the gradient) and
// run the y and z axes as strided line passes (dd_convolve_columns).
// The transforms are radix-2 in LDS (stages fused in pairs), one row or
// column per block:
// decimation in time (bit-reversed in, natural out) forward and decimation
// in frequency (natural in, bit-reversed out) inverse, so no permutation
// pass is needed between them.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dd.hpp"
#include "qd.hpp"
#include "dt_dd.hpp"
#include "epilogue.hpp"

namespace dt {
namespace {

using ddm::cplx;
using ddm::dd;
using ddm::qd;
using ddm::xp;

constexpr int kThreads = 256;
// Threads per block of the transform kernels (their launch bound): 256 for
// double-double; up to 512 for quad-double, whose 2048-point lines fill
// 128 KB of LDS (one block per CU) and whose kernels fit two waves per SIMD
// in registers, so the larger block doubles the waves that share a CU.
template <class R> constexpr int threads_of() { return sizeof(R) > 16 ? 512 : 256; }
// Threads of one launch whose blocks hold `elems` values: the larger block
// only where it has work for every thread (shorter blocks would leave half
// of it idle in each radix-4 stage).
template <class R> int block_threads(int elems) { return elems >= 2048 ? threads_of<R>() : kThreads; }

__device__ __forceinline__ int brev(int x, int logM) { return (int)(__builtin_bitreverse32((uint32_t)x) >> (32 - logM)); }

template <class R> __device__ __forceinline__ cplx<R> zero_c() { return {xp<R>::zero(), xp<R>::zero()}; }

// Channels and spectra of a plan: 0 f, 1 .. ndim the gradient kernels (odd:
// imaginary spectra), then the Hessian kernels in the order xx, xy, [xz,]
// yy, [yz,] zz (even or odd in two axes: real spectra).
__host__ __device__ __forceinline__ bool dd_imag_channel(int c, int ndim) { return c >= 1 && c <= ndim; }
__device__ __forceinline__ void dd_hess_pair(int ndim, int h, int& i, int& j) {
  if (ndim == 2) {
    i = h == 2 ? 1 : 0;
    j = h == 0 ? 0 : 1;
  } else {
    const int a[6] = {0, 0, 0, 1, 1, 2}, b[6] = {0, 1, 2, 1, 2, 2};
    i = a[h];
    j = b[h];
  }
}

template <class R> __device__ __forceinline__ cplx<R> twiddle(const cplx<R>* __restrict__ tw, int k, bool inv) {
  cplx<R> w = tw[k];
  if (inv) w.im = ddm::neg(w.im);
  return w;
}

// In-place radix-2 decimation in time over bit-reversed input; natural
// order out.  tw[k] = exp(-2 pi i k / M); INV conjugates it.  Stages s and
// s + 1 are taken together: a thread carries four elements through both in
// registers (the same butterflies as two radix-2 stages), which halves the
// LDS round trips and barriers; an odd last stage runs alone.  NL lines of
// M elements stored back to back are transformed together (the same
// arithmetic per line).
template <class R, bool INV, int NL = 1>
__device__ __forceinline__ void fft_dit(cplx<R>* buf, int M, int logM, const cplx<R>* __restrict__ tw) {
  int s = 1;
  for (; s + 1 <= logM; s += 2) {
    const int half = 1 << (s - 1);
    for (int qa = threadIdx.x; qa < NL * (M >> 2); qa += blockDim.x) {
      cplx<R>* b = NL == 1 ? buf : buf + ((qa >> (logM - 2)) << logM);   // line qa / (M / 4)
      const int q = NL == 1 ? qa : qa & ((M >> 2) - 1);
      const int j = q & (half - 1);
      const int i0 = ((q >> (s - 1)) << (s + 1)) + j;
      const cplx<R> wa = twiddle(tw, j * (M >> s), INV);
      const cplx<R> wb = twiddle(tw, j * (M >> (s + 1)), INV);
      const cplx<R> wc = twiddle(tw, (j + half) * (M >> (s + 1)), INV);
      const cplx<R> a0 = b[i0], a1 = b[i0 + half], a2 = b[i0 + 2 * half], a3 = b[i0 + 3 * half];
      const cplx<R> t1 = ddm::cmul(a1, wa), t3 = ddm::cmul(a3, wa);
      const cplx<R> x0 = ddm::cadd(a0, t1), x1 = ddm::csub(a0, t1);
      const cplx<R> x2 = ddm::cadd(a2, t3), x3 = ddm::csub(a2, t3);
      const cplx<R> u2 = ddm::cmul(x2, wb), u3 = ddm::cmul(x3, wc);
      b[i0] = ddm::cadd(x0, u2);
      b[i0 + 2 * half] = ddm::csub(x0, u2);
      b[i0 + half] = ddm::cadd(x1, u3);
      b[i0 + 3 * half] = ddm::csub(x1, u3);
    }
    __syncthreads();
  }
  if (s == logM) {
    const int half = 1 << (s - 1);
    for (int ba = threadIdx.x; ba < NL * (M >> 1); ba += blockDim.x) {
      cplx<R>* bu = NL == 1 ? buf : buf + ((ba >> (logM - 1)) << logM);
      const int bb = NL == 1 ? ba : ba & ((M >> 1) - 1);
      const int j = bb & (half - 1);
      const int i0 = ((bb >> (s - 1)) << s) + j;
      const cplx<R> v = ddm::cmul(bu[i0 + half], twiddle(tw, j * (M >> s), INV));
      const cplx<R> u = bu[i0];
      bu[i0] = ddm::cadd(u, v);
      bu[i0 + half] = ddm::csub(u, v);
    }
    __syncthreads();
  }
}

// In-place radix-2 decimation in frequency over natural-order input;
// bit-reversed order out.  An odd top stage runs alone, then stages t and
// t - 1 are taken together as in fft_dit; NL lines as in fft_dit.
template <class R, bool INV, int NL = 1>
__device__ __forceinline__ void fft_dif(cplx<R>* buf, int M, int logM, const cplx<R>* __restrict__ tw) {
  int t = logM;
  if (logM & 1) {
    const int half = 1 << (t - 1);
    for (int ba = threadIdx.x; ba < NL * (M >> 1); ba += blockDim.x) {
      cplx<R>* bu = NL == 1 ? buf : buf + ((ba >> (logM - 1)) << logM);
      const int bb = NL == 1 ? ba : ba & ((M >> 1) - 1);
      const int j = bb & (half - 1);
      const int i0 = ((bb >> (t - 1)) << t) + j;
      const cplx<R> u = bu[i0], v = bu[i0 + half];
      bu[i0] = ddm::cadd(u, v);
      bu[i0 + half] = ddm::cmul(ddm::csub(u, v), twiddle(tw, j * (M >> t), INV));
    }
    __syncthreads();
    --t;
  }
  for (; t >= 2; t -= 2) {
    const int s = t - 1;              // lower stage of the pair
    const int half = 1 << (s - 1);
    for (int qa = threadIdx.x; qa < NL * (M >> 2); qa += blockDim.x) {
      cplx<R>* b = NL == 1 ? buf : buf + ((qa >> (logM - 2)) << logM);
      const int q = NL == 1 ? qa : qa & ((M >> 2) - 1);
      const int j = q & (half - 1);
      const int i0 = ((q >> (s - 1)) << (s + 1)) + j;
      const cplx<R> wb = twiddle(tw, j * (M >> t), INV);
      const cplx<R> wc = twiddle(tw, (j + half) * (M >> t), INV);
      const cplx<R> wa = twiddle(tw, j * (M >> s), INV);
      const cplx<R> a0 = b[i0], a1 = b[i0 + half], a2 = b[i0 + 2 * half], a3 = b[i0 + 3 * half];
      const cplx<R> y0 = ddm::cadd(a0, a2), y2 = ddm::cmul(ddm::csub(a0, a2), wb);
      const cplx<R> y1 = ddm::cadd(a1, a3), y3 = ddm::cmul(ddm::csub(a1, a3), wc);
      b[i0] = ddm::cadd(y0, y1);
      b[i0 + half] = ddm::cmul(ddm::csub(y0, y1), wa);
      b[i0 + 2 * half] = ddm::cadd(y2, y3);
      b[i0 + 3 * half] = ddm::cmul(ddm::csub(y2, y3), wa);
    }
    __syncthreads();
  }
}

// exp(-2 pi i k / M) for 0 <= k < M/2, M a power of two >= 8: the angle is
// reduced to an octant so that the series sees |a| <= pi/4.
template <class R>
__global__ void k_dd_twiddles(cplx<R>* __restrict__ tw, int M) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M / 2) return;
  int j, oct;
  if (8 * k <= M) {
    j = k;
    oct = 0;
  } else if (4 * k <= M) {
    j = M / 4 - k;
    oct = 1;
  } else if (8 * k <= 3 * M) {
    j = k - M / 4;
    oct = 2;
  } else {
    j = M / 2 - k;
    oct = 3;
  }
  const R a = ddm::mul_d(xp<R>::two_pi(), (double)j / (double)M);
  R s, c;
  ddm::sincos_reduced(a, s, c);
  R cs, sn;
  switch (oct) {
    case 0: cs = c; sn = s; break;
    case 1: cs = s; sn = c; break;
    case 2: cs = ddm::neg(s); sn = c; break;
    default: cs = ddm::neg(c); sn = s; break;
  }
  tw[k] = {cs, ddm::neg(sn)};
}

// Kernel samples at every displacement d of the padded grid (minimum image;
// the Nyquist lines are set to 0 as in the other precisions): kind 0 is
// f = exp(-r / tau), kind 1 + a the gradient kernel (h_a d_a / r) f, 0 at
// r = 0 (eq. SxSyconv).  The displacement h d is an exact product (its
// float64 rounding error carried as the second part).
template <class R>
__global__ void k_dd_tab_sample(cplx<R>* __restrict__ G, DDGeom g, int kind) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)g.Mx * g.My * g.Mz) return;
  const int x = (int)(i % g.Mx), y = (int)((i / g.Mx) % g.My), z = (int)(i / ((int64_t)g.Mx * g.My));
  cplx<R> v = zero_c<R>();
  if (x != g.Mx / 2 && y != g.My / 2 && (g.ndim == 2 || z != g.Mz / 2)) {
    const int dx = x < g.Mx / 2 ? x : x - g.Mx;
    const int dy = y < g.My / 2 ? y : y - g.My;
    const int dz = z < g.Mz / 2 ? z : z - g.Mz;
    const R px = xp<R>::prod(g.hx, (double)dx), py = xp<R>::prod(g.hy, (double)dy);
    const R pz = g.ndim == 3 ? xp<R>::prod(g.hz, (double)dz) : xp<R>::zero();
    R r2 = ddm::add(ddm::mul(px, px), ddm::mul(py, py));
    if (g.ndim == 3) r2 = ddm::add(r2, ddm::mul(pz, pz));
    const R r = ddm::sqrt(r2);
    const R f = ddm::exp_nonpos(ddm::neg(ddm::div_d(r, g.tau)));
    const R p[3] = {px, py, pz};
    if (kind == 0) {
      v.re = f;
    } else if (kind == kDDKindRF) {
      v.re = ddm::mul(r, f);                     // r f (the adjoint's tau kernel), 0 at r = 0
    } else if (xp<R>::lead(r) > 0.0 && kind <= g.ndim) {
      v.re = ddm::mul(ddm::div(p[kind - 1], r), f);
    } else if (xp<R>::lead(r) > 0.0) {
      // Hessian kernel (-n_i n_j / tau + (delta_ij - n_i n_j) / r) f
      int a, b;
      dd_hess_pair(g.ndim, kind - 1 - g.ndim, a, b);
      const R nn = ddm::mul(ddm::div(p[a], r), ddm::div(p[b], r));
      const R t1 = ddm::neg(ddm::div_d(nn, g.tau));
      const R t2 = ddm::div(a == b ? ddm::sub(xp<R>::from(1.0), nn) : ddm::neg(nn), r);
      v.re = ddm::mul(ddm::add(t1, t2), f);
    }
  }
  G[i] = v;
}

// Strided lines of one axis: line l < n_lines is (o, i) = (l / n_inner,
// l % n_inner), its element j at o * outer + j * stride + i.
struct DDLines {
  int M, logM, n_inner, n_in, n_out;
  int64_t n_lines, in_outer, in_stride, out_outer, out_stride;
  int log_lb;   // a block takes 2^log_lb adjacent lines (n_inner a multiple of that)
};

// Forward transform of each line (input elements j >= n_in are zero).
// MODE 0: complex spectrum to out; 1 / 2: its real / imaginary part times
// 2^scale_e to tab.  A block takes LB = 2^log_lb adjacent lines (the inner
// index is the fastest in memory, so element j of the LB lines is one
// contiguous run) and reads them whole before writing, so in and out may be
// the same array.
template <class R, int MODE, int LB>
__global__ __launch_bounds__(threads_of<R>()) void k_dd_line_fwd(const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                          R* __restrict__ tab, const cplx<R>* __restrict__ tw,
                                                          DDLines L, int scale_e) {
  extern __shared__ __align__(16) char smem[];
  cplx<R>* buf = (cplx<R>*)smem;
  constexpr int lb = LB;
  const int64_t l = (int64_t)blockIdx.x << L.log_lb;
  const int64_t o = l / L.n_inner, i = l % L.n_inner;
  const cplx<R>* src = in + o * L.in_outer + i;
  for (int u = threadIdx.x; u < (L.M << L.log_lb); u += blockDim.x) {
    const int t = u & (lb - 1), j = u >> L.log_lb;
    buf[(t << L.logM) + brev(j, L.logM)] = j < L.n_in ? src[(int64_t)j * L.in_stride + t] : zero_c<R>();
  }
  __syncthreads();
  fft_dit<R, false, LB>(buf, L.M, L.logM, tw);
  if (MODE == 0) {
    cplx<R>* dst = out + o * L.out_outer + i;
    for (int u = threadIdx.x; u < (L.M << L.log_lb); u += blockDim.x) {
      const int t = u & (lb - 1), k = u >> L.log_lb;
      dst[(int64_t)k * L.out_stride + t] = buf[(t << L.logM) + k];
    }
  } else {
    R* dst = tab + o * L.out_outer + i;
    for (int u = threadIdx.x; u < (L.M << L.log_lb); u += blockDim.x) {
      const int t = u & (lb - 1), k = u >> L.log_lb;
      const cplx<R> v = buf[(t << L.logM) + k];
      dst[(int64_t)k * L.out_stride + t] = ddm::scale2(MODE == 2 ? v.im : v.re, scale_e);
    }
  }
}

// Inverse (unnormalised) transform of each line from its natural-order
// spectrum; the first n_out samples are kept.  LB adjacent lines per block.
template <class R, int LB>
__global__ __launch_bounds__(threads_of<R>()) void k_dd_line_inv(const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                          const cplx<R>* __restrict__ tw, DDLines L) {
  extern __shared__ __align__(16) char smem[];
  cplx<R>* buf = (cplx<R>*)smem;
  constexpr int lb = LB;
  const int64_t l = (int64_t)blockIdx.x << L.log_lb;
  const int64_t o = l / L.n_inner, i = l % L.n_inner;
  const cplx<R>* src = in + o * L.in_outer + i;
  for (int u = threadIdx.x; u < (L.M << L.log_lb); u += blockDim.x) {
    const int t = u & (lb - 1), k = u >> L.log_lb;
    buf[(t << L.logM) + k] = src[(int64_t)k * L.in_stride + t];
  }
  __syncthreads();
  fft_dif<R, true, LB>(buf, L.M, L.logM, tw);
  cplx<R>* dst = out + o * L.out_outer + i;
  for (int u = threadIdx.x; u < (L.n_out << L.log_lb); u += blockDim.x) {
    const int t = u & (lb - 1), y = u >> L.log_lb;
    dst[(int64_t)y * L.out_stride + t] = buf[(t << L.logM) + brev(y, L.logM)];
  }
}

// Forward transform of rows.  REAL_IN: row y of the ny x nx multiplicities,
// zero-padded to Mx; else row y of G in place.
template <class R, bool REAL_IN>
__global__ __launch_bounds__(threads_of<R>()) void k_dd_row_fwd(const double* __restrict__ cnt, cplx<R>* __restrict__ G,
                                                         const cplx<R>* __restrict__ tw, DDGeom g) {
  extern __shared__ __align__(16) char smem[];
  cplx<R>* buf = (cplx<R>*)smem;
  const int y = blockIdx.x;
  const int M = g.Mx;
  for (int x = threadIdx.x; x < M; x += blockDim.x) {
    cplx<R> v;
    if (REAL_IN) {
      v = zero_c<R>();
      if (x < g.nx) v.re = xp<R>::from(cnt[(int64_t)y * g.nx + x]);
    } else {
      v = G[(int64_t)y * M + x];
    }
    buf[brev(x, g.logMx)] = v;
  }
  __syncthreads();
  fft_dit<R, false>(buf, M, g.logMx, tw);
  for (int x = threadIdx.x; x < M; x += blockDim.x) G[(int64_t)y * M + x] = buf[x];
}

// Table mode (plan time): column kx of the row-transformed samples in G,
// forward transform, and the real (IMAG = false) or imaginary part of the
// spectrum, scaled by 1/(Mx My), into tab.
template <class R, bool IMAG>
__global__ __launch_bounds__(threads_of<R>()) void k_dd_col_table(const cplx<R>* __restrict__ G, R* __restrict__ tab,
                                                           const cplx<R>* __restrict__ tw, DDGeom g) {
  extern __shared__ __align__(16) char smem[];
  cplx<R>* buf = (cplx<R>*)smem;
  const int kx = blockIdx.x;
  const int M = g.My;
  for (int y = threadIdx.x; y < M; y += blockDim.x) buf[brev(y, g.logMy)] = G[(int64_t)y * g.Mx + kx];
  __syncthreads();
  fft_dit<R, false>(buf, M, g.logMy, tw);
  const int e = -(g.logMx + g.logMy);
  for (int ky = threadIdx.x; ky < M; ky += blockDim.x)
    tab[(int64_t)ky * g.Mx + kx] = ddm::scale2(IMAG ? buf[ky].im : buf[ky].re, e);
}

// Column kx, for each channel c < C: forward transform of rows [0, ny) of
// Gin (zero above), product with spectrum c (channel 0 real: f; channels
// 1.. imaginary: the odd gradient kernels, i v), inverse transform, rows
// [0, ny) into channel c of Gout (ny x Mx each).  With several channels
// (MULTI) each thread keeps its bins of the forward spectrum in registers
// (My <= kSpecPerThread * blockDim.x), so the forward transform runs once.
constexpr int kSpecPerThread = 8;

// The last axis of a plan: transform length M, a line every `stride`
// elements (2D: Mx, line kx; 3D: My Mx, line ky Mx + kx), n rows present and
// kept, output channels `plane` apart, spectra `tab_chan` apart.
struct DDFused {
  int M, logM, n;
  int64_t stride, plane, tab_chan;
  DDChannels ch;
  int log_lb;   // a block takes 2^log_lb adjacent lines
};

template <class R, bool MULTI, int LB, int SPT = kSpecPerThread>
__global__ __launch_bounds__(threads_of<R>()) void k_dd_col_fused(const cplx<R>* __restrict__ Gin, cplx<R>* __restrict__ Gout,
                                                           const R* __restrict__ tabs, const cplx<R>* __restrict__ tw,
                                                           DDFused F, int C) {
  extern __shared__ __align__(16) char smem[];
  cplx<R>* buf = (cplx<R>*)smem;
  constexpr int lb = LB;
  const int64_t kx = (int64_t)blockIdx.x << F.log_lb;   // the block's first line
  const int M = F.M;
  const int ML = M << F.log_lb;   // elements of the block's lines; element u: line u mod LB, row u / LB
  const int64_t npad = F.tab_chan, plane = F.plane;
  for (int u = threadIdx.x; u < ML; u += blockDim.x) {
    const int t = u & (lb - 1), y = u >> F.log_lb;
    buf[(t << F.logM) + brev(y, F.logM)] = y < F.n ? Gin[(int64_t)y * F.stride + kx + t] : zero_c<R>();
  }
  __syncthreads();
  fft_dit<R, false, LB>(buf, M, F.logM, tw);
  cplx<R> sp[MULTI ? SPT : 1];
  if (MULTI) {
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      const int u = threadIdx.x + k * blockDim.x;
      if (u < ML) sp[k] = buf[((u & (lb - 1)) << F.logM) + (u >> F.log_lb)];
    }
  }
  for (int c = 0; c < C; ++c) {
    const R* tab = tabs + F.ch.tab_of[c] * npad;
    if (MULTI) __syncthreads();   // every thread has read its spectrum bins (or its last outputs)
    // (a.re + i a.im) t, or (a.re + i a.im) (i t) = -a.im t + i a.re t; each
    // thread rewrites only the slots whose spectrum it holds
    const bool imag = (F.ch.imag >> c) & 1u;
    auto product = [&](int u, const cplx<R>& a) {
      const int t = u & (lb - 1), ky = u >> F.log_lb;
      const R tv = tab[(int64_t)ky * F.stride + kx + t];
      buf[(t << F.logM) + ky] = !imag ? ddm::cmul_real(a, tv) : cplx<R>{ddm::neg(ddm::mul(a.im, tv)), ddm::mul(a.re, tv)};
    };
    if (MULTI) {
#pragma unroll
      for (int k = 0; k < SPT; ++k) {
        const int u = threadIdx.x + k * blockDim.x;
        if (u < ML) product(u, sp[k]);
      }
    } else {
      for (int u = threadIdx.x; u < ML; u += blockDim.x)
        product(u, buf[((u & (lb - 1)) << F.logM) + (u >> F.log_lb)]);
    }
    __syncthreads();
    fft_dif<R, true, LB>(buf, M, F.logM, tw);
    for (int u = threadIdx.x; u < (F.n << F.log_lb); u += blockDim.x) {
      const int t = u & (lb - 1), y = u >> F.log_lb;
      Gout[c * plane + (int64_t)y * F.stride + kx + t] = buf[(t << F.logM) + brev(y, F.logM)];
    }
    if (!MULTI) __syncthreads();
  }
}

// Inverse transforms of row y and the epilogue: phi = Re of channel 0,
// S = -tau log phi where phi >= Theta, else S_max (scal[0] = Theta,
// scal[1] = S_max); with the gradient channels also grad_a S = psi_a / phi
// (eq. SxSyconv), and with the Hessian channels H_ij = chi_ij / phi +
// S_i S_j / tau (eqs. Sxx, Syy, Sxy), all 0 where phi < Theta, and from those
// the curvatures (mean, Gaussian, k1, k2; the same formulas as the other
// precisions).  S, grad, hess or curv may be null.  phi, grad S and H stay in
// registers (nx <= kMaxPerThread * blockDim.x) while the later channels are
// transformed.
constexpr int kMaxPerThread = 4;

template <class R>
__global__ __launch_bounds__(threads_of<R>()) void k_dd_row_inv_epi(const cplx<R>* __restrict__ Gc, const cplx<R>* __restrict__ tw,
                                                             double* __restrict__ S, double* __restrict__ grad,
                                                             double* __restrict__ hess, double* __restrict__ curv,
                                                             const double* __restrict__ scal, DDGeom g, int C) {
  extern __shared__ __align__(16) char smem[];
  cplx<R>* buf = (cplx<R>*)smem;
  const int y = blockIdx.x;
  const int M = g.Mx;
  const int64_t plane = (int64_t)g.ny * M, nodes = (int64_t)g.nx * g.ny;
  const double theta = scal[0], smax = scal[1];
  double phi[kMaxPerThread], gs[kMaxPerThread][3], hs[kMaxPerThread][6];
  for (int c = 0; c < C; ++c) {
    for (int x = threadIdx.x; x < M; x += blockDim.x) buf[x] = Gc[c * plane + (int64_t)y * M + x];
    __syncthreads();
    fft_dif<R, true>(buf, M, g.logMx, tw);
#pragma unroll
    for (int k = 0; k < kMaxPerThread; ++k) {
      const int x = threadIdx.x + k * blockDim.x;
      if (x >= g.nx) break;
      const R v = buf[brev(x, g.logMx)].re;
      const double vh = xp<R>::lead(v), vl = xp<R>::next(v);
      if (c == 0) {
        phi[k] = vh;
        if (S) {
          // log(hi + lo) = log(hi) + lo / hi to float64 accuracy
          const bool ok0 = vh > 0.0 && vh >= theta;
          S[(int64_t)y * g.nx + x] = ok0 ? -g.tau * (log(vh) + vl / vh) : smax;
        }
      } else {
        const bool ok = phi[k] > 0.0 && phi[k] >= theta;
        if (c <= g.ndim) {
          const double gv = ok ? vh / phi[k] : 0.0;
          gs[k][c - 1] = gv;
          if (grad) grad[(c - 1) * nodes + (int64_t)y * g.nx + x] = gv;
        } else {
          const int hh = c - 1 - g.ndim;
          int a, b;
          dd_hess_pair(g.ndim, hh, a, b);
          const double hv = ok ? vh / phi[k] + gs[k][a] * gs[k][b] / g.tau : 0.0;
          hs[k][hh] = hv;
          if (hess) hess[hh * nodes + (int64_t)y * g.nx + x] = hv;
        }
      }
    }
    __syncthreads();
  }
  if (curv) {
#pragma unroll
    for (int k = 0; k < kMaxPerThread; ++k) {
      const int x = threadIdx.x + k * blockDim.x;
      if (x >= g.nx) break;
      double cv[4];
      if (g.ndim == 2) curvature_graph(gs[k], hs[k], cv);
      else curvature_level_set(gs[k], hs[k], cv);
      for (int q = 0; q < 4; ++q) curv[q * nodes + (int64_t)y * g.nx + x] = cv[q];
    }
  }
}

// Inverse transforms of row y of C channels into plain fields (the float64
// leading part of the real part), out[c][row][x] for x < nx (the adjoint's
// convolutions w * u_a and w * r f).
template <class R>
__global__ __launch_bounds__(threads_of<R>()) void k_dd_row_inv_plain(const cplx<R>* __restrict__ Gc, const cplx<R>* __restrict__ tw,
                                                               double* __restrict__ out, DDGeom g, int C) {
  extern __shared__ __align__(16) char smem[];
  cplx<R>* buf = (cplx<R>*)smem;
  const int y = blockIdx.x;
  const int M = g.Mx;
  const int64_t plane = (int64_t)g.ny * M, nodes = (int64_t)g.nx * g.ny;
  for (int c = 0; c < C; ++c) {
    for (int x = threadIdx.x; x < M; x += blockDim.x) buf[x] = Gc[c * plane + (int64_t)y * M + x];
    __syncthreads();
    fft_dif<R, true>(buf, M, g.logMx, tw);
    for (int x = threadIdx.x; x < g.nx; x += blockDim.x) out[c * nodes + (int64_t)y * g.nx + x] = xp<R>::lead(buf[brev(x, g.logMx)].re);
    __syncthreads();
  }
}

// The adjoint at the sources: dL/dY_k = (w * u_a)(Y_k) / p2 from the channel
// fields (a < ndim), and per-block sums of (w * r f)(Y_k) / p2 for dL/dtau
// (scal[3] = p2, the power of two that scaled w).  Sources outside the grid
// get 0 (the forward call has already raised the sticky range error).
__global__ __launch_bounds__(256) void k_dd_gather(const float* __restrict__ Y, int64_t K,
                                                   const double* __restrict__ fields, const double* __restrict__ scal,
                                                   float* __restrict__ dY, double* __restrict__ partials, DDGeom g) {
  __shared__ double red[256];
  const int D = g.ndim;
  const int64_t nodes = (int64_t)g.nx * g.ny * g.nz;
  const double inv_p2 = 1.0 / scal[3];
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
    const double y0 = Y[D * k], y1 = Y[D * k + 1], y2 = D == 3 ? Y[D * k + 2] : 0.0;
    const double fx = __builtin_floor((y0 - g.ox) / g.hx), fy = __builtin_floor((y1 - g.oy) / g.hy);
    const double fz = D == 3 ? __builtin_floor((y2 - g.oz) / g.hz) : 0.0;
    const bool in = fx >= 0.0 && fx < (double)g.nx && fy >= 0.0 && fy < (double)g.ny && fz >= 0.0 &&
                    fz < (double)g.nz;
    const int64_t node = in ? ((int64_t)fz * g.ny + (int64_t)fy) * g.nx + (int64_t)fx : 0;
    for (int a = 0; a < D; ++a) dY[D * k + a] = in ? (float)(fields[a * nodes + node] * inv_p2) : 0.0f;
    if (in) acc += fields[D * nodes + node] * inv_p2;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if ((int)threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// Node assignment idx = floor((y - o) / h) in float64; multiplicities by
// atomic adds (integers, exact in float64).  Each add that raises a count
// from c to c + 1 raises sum m^2 by 2c + 1; those increments are summed per
// wave and added to *msq (integer sums below 2^53: exact in any order).
// Bit 1: outside the grid, bit 2: non-finite.
__global__ __launch_bounds__(256) void k_dd_splat(const float* __restrict__ Y, int64_t K, double* __restrict__ cnt,
                                                  double* __restrict__ msq, uint32_t* __restrict__ err, DDGeom g) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double inc = 0.0;
  if (k < K) {
    const int D = g.ndim;
    const double y0 = Y[D * k], y1 = Y[D * k + 1], y2 = D == 3 ? Y[D * k + 2] : 0.0;
    if (!__builtin_isfinite(y0) || !__builtin_isfinite(y1) || !__builtin_isfinite(y2)) {
      atomicOr(err, 2u);
    } else {
      const double fx = __builtin_floor((y0 - g.ox) / g.hx), fy = __builtin_floor((y1 - g.oy) / g.hy);
      const double fz = D == 3 ? __builtin_floor((y2 - g.oz) / g.hz) : 0.0;
      if (!(fx >= 0.0 && fx < (double)g.nx && fy >= 0.0 && fy < (double)g.ny && fz >= 0.0 && fz < (double)g.nz)) {
        atomicOr(err, 1u);
      } else {
        const double old = atomicAdd(&cnt[((int64_t)fz * g.ny + (int64_t)fy) * g.nx + (int64_t)fx], 1.0);
        inc = 2.0 * old + 1.0;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) inc += __shfl_xor(inc, off);
  if ((threadIdx.x & 63) == 0 && inc != 0.0) atomicAdd(msq, inc);
}

// ||g||_2 = sqrt(sum m^2) and the validity threshold
// Theta = c u log2(N_pad) ||f||_1 ||g||_2 / sqrt(N_pad), S_max; clears the
// accumulator for the next call.
__global__ void k_dd_finalize(double* __restrict__ msq, double* __restrict__ scal, DDGeom g, double c_theta,
                              double unit, double l1) {
  if (threadIdx.x != 0) return;
  const double npad = (double)g.Mx * (double)g.My * (double)g.Mz;
  const double gl2 = __builtin_sqrt(*msq);
  *msq = 0.0;
  const double theta = c_theta * unit * (double)(g.logMx + g.logMy + g.logMz) * l1 * gl2 / __builtin_sqrt(npad);
  scal[0] = theta;
  scal[1] = -g.tau * log(theta);
  scal[2] = gl2;
  int e2;
  frexp(theta, &e2);
  scal[3] = ldexp(1.0, e2 - 1);   // the largest power of two <= Theta (scales the adjoint's weights)
}

// Kernels whose dynamic LDS exceeds the default 64 KiB limit must opt in.
template <typename F>
hipError_t allow_lds(F kern, size_t lds) {
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

// Adjacent lines per block of the strided line passes, as a power of two:
// four (a 128-byte run of double-double complex values per row, 256 bytes
// in quad-double) where the block's four lines stay within 64 KiB of LDS,
// else one.
template <class R> static int dd_log_lb(int M, int64_t n_inner) {
  return ((size_t)M * 4 * sizeof(cplx<R>) <= 65536 && n_inner % 4 == 0) ? 2 : 0;
}

// Launches of the strided line passes with L.log_lb adjacent lines per block.
template <class R, int MODE>
static hipError_t launch_line_fwd(const cplx<R>* in, cplx<R>* out, R* tab, const cplx<R>* tw, const DDLines& L,
                                  int scale_e, hipStream_t st) {
  const size_t lds = ((size_t)L.M << L.log_lb) * sizeof(cplx<R>);
  const unsigned blocks = (unsigned)(L.n_lines >> L.log_lb);
  const int nt = block_threads<R>(L.M << L.log_lb);
  hipError_t e;
  if (L.log_lb == 2) {
    if ((e = allow_lds(k_dd_line_fwd<R, MODE, 4>, lds)) != hipSuccess) return e;
    k_dd_line_fwd<R, MODE, 4><<<blocks, nt, lds, st>>>(in, out, tab, tw, L, scale_e);
  } else {
    if ((e = allow_lds(k_dd_line_fwd<R, MODE, 1>, lds)) != hipSuccess) return e;
    k_dd_line_fwd<R, MODE, 1><<<blocks, nt, lds, st>>>(in, out, tab, tw, L, scale_e);
  }
  return hipSuccess;
}
template <class R>
static hipError_t launch_line_inv(const cplx<R>* in, cplx<R>* out, const cplx<R>* tw, const DDLines& L,
                                  hipStream_t st) {
  const size_t lds = ((size_t)L.M << L.log_lb) * sizeof(cplx<R>);
  const unsigned blocks = (unsigned)(L.n_lines >> L.log_lb);
  const int nt = block_threads<R>(L.M << L.log_lb);
  hipError_t e;
  if (L.log_lb == 2) {
    if ((e = allow_lds(k_dd_line_inv<R, 4>, lds)) != hipSuccess) return e;
    k_dd_line_inv<R, 4><<<blocks, nt, lds, st>>>(in, out, tw, L);
  } else {
    if ((e = allow_lds(k_dd_line_inv<R, 1>, lds)) != hipSuccess) return e;
    k_dd_line_inv<R, 1><<<blocks, nt, lds, st>>>(in, out, tw, L);
  }
  return hipSuccess;
}

// 3D tables: rows of the Mz x My sample rows in place, then the y lines in
// place, then the z lines into the real or imaginary spectrum.
template <class R>
static hipError_t build_tables_3d(void* twx, void* twy, void* twz, void* tabs, int n_tabs, int rf_tab, void* G,
                                  const DDGeom& g, hipStream_t st) {
  using C = cplx<R>;
  k_dd_twiddles<R><<<(g.Mz / 2 + 255) / 256, 256, 0, st>>>((C*)twz, g.Mz);
  const int64_t plane = (int64_t)g.Mx * g.My, total = plane * g.Mz;
  const size_t lx = (size_t)g.Mx * sizeof(C);
  hipError_t e = allow_lds(k_dd_row_fwd<R, false>, lx);
  if (e != hipSuccess) return e;
  DDGeom rows = g;
  rows.ny = g.My * g.Mz;   // every sample row
  DDLines ly_{g.My, g.logMy, g.Mx, g.My, g.My, (int64_t)g.Mz * g.Mx, plane, g.Mx, plane, g.Mx, dd_log_lb<R>(g.My, g.Mx)};
  DDLines lz_{g.Mz, g.logMz, (int)plane, g.Mz, g.Mz, plane, 0, plane, 0, plane, dd_log_lb<R>(g.Mz, plane)};
  for (int t = 0; t < n_tabs; ++t) {
    R* tab = (R*)tabs + t * total;
    k_dd_tab_sample<R><<<(unsigned)((total + 255) / 256), 256, 0, st>>>((C*)G, g, t == rf_tab ? kDDKindRF : t);
    k_dd_row_fwd<R, false><<<(unsigned)rows.ny, block_threads<R>(g.Mx), lx, st>>>(nullptr, (C*)G, (const C*)twx, rows);
    if ((e = launch_line_fwd<R, 0>((const C*)G, (C*)G, nullptr, (const C*)twy, ly_, 0, st)) != hipSuccess) return e;
    const int e_scale = -(g.logMx + g.logMy + g.logMz);
    if (t == rf_tab || !dd_imag_channel(t, g.ndim))
      e = launch_line_fwd<R, 1>((const C*)G, nullptr, tab, (const C*)twz, lz_, e_scale, st);
    else
      e = launch_line_fwd<R, 2>((const C*)G, nullptr, tab, (const C*)twz, lz_, e_scale, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

template <class R>
static hipError_t build_tables(void* twx, void* twy, void* twz, void* tabs, int n_tabs, int rf_tab, void* G,
                               const DDGeom& g, hipStream_t st) {
  using C = cplx<R>;
  k_dd_twiddles<R><<<(g.Mx / 2 + 255) / 256, 256, 0, st>>>((C*)twx, g.Mx);
  k_dd_twiddles<R><<<(g.My / 2 + 255) / 256, 256, 0, st>>>((C*)twy, g.My);
  if (g.ndim == 3) return build_tables_3d<R>(twx, twy, twz, tabs, n_tabs, rf_tab, G, g, st);
  const int64_t total = (int64_t)g.Mx * g.My;
  const size_t lx = (size_t)g.Mx * sizeof(C), ly = (size_t)g.My * sizeof(C);
  hipError_t e = allow_lds(k_dd_row_fwd<R, false>, lx);
  if (e == hipSuccess) e = allow_lds(k_dd_col_table<R, false>, ly);
  if (e == hipSuccess) e = allow_lds(k_dd_col_table<R, true>, ly);
  if (e != hipSuccess) return e;
  for (int t = 0; t < n_tabs; ++t) {
    R* tab = (R*)tabs + t * total;
    k_dd_tab_sample<R><<<(unsigned)((total + 255) / 256), 256, 0, st>>>((C*)G, g, t == rf_tab ? kDDKindRF : t);
    k_dd_row_fwd<R, false><<<g.My, block_threads<R>(g.Mx), lx, st>>>(nullptr, (C*)G, (const C*)twx, g);
    if (t == rf_tab || !dd_imag_channel(t, g.ndim))
      k_dd_col_table<R, false><<<g.Mx, block_threads<R>(g.My), ly, st>>>((const C*)G, tab, (const C*)twy, g);
    else
      k_dd_col_table<R, true><<<g.Mx, block_threads<R>(g.My), ly, st>>>((const C*)G, tab, (const C*)twy, g);
  }
  return hipGetLastError();
}

hipError_t dd_build_tables(void* twx, void* twy, void* twz, void* tabs, int n_tabs, int rf_tab, void* G,
                           const DDGeom& g, hipStream_t st) {
  return g.quad ? build_tables<qd>(twx, twy, twz, tabs, n_tabs, rf_tab, G, g, st)
                : build_tables<dd>(twx, twy, twz, tabs, n_tabs, rf_tab, G, g, st);
}

hipError_t dd_launch_splat(const float* Y, int64_t K, double* cnt, double* msq, uint32_t* err, const DDGeom& g,
                           hipStream_t st) {
  k_dd_splat<<<(unsigned)((K + 255) / 256), 256, 0, st>>>(Y, K, cnt, msq, err, g);
  return hipGetLastError();
}

hipError_t dd_launch_finalize(double* msq, double* scal, const DDGeom& g, double c_theta, double unit, double l1,
                              hipStream_t st) {
  k_dd_finalize<<<1, 64, 0, st>>>(msq, scal, g, c_theta, unit, l1);
  return hipGetLastError();
}

template <class R>
static hipError_t row_fwd(const double* cnt, void* G, const void* twx, const DDGeom& g, hipStream_t st) {
  using C = cplx<R>;
  const size_t lds = (size_t)g.Mx * sizeof(C);
  const hipError_t e = allow_lds(k_dd_row_fwd<R, true>, lds);
  if (e != hipSuccess) return e;
  k_dd_row_fwd<R, true><<<g.ny, block_threads<R>(g.Mx), lds, st>>>(cnt, (C*)G, (const C*)twx, g);
  return hipGetLastError();
}
hipError_t dd_launch_row_fwd(const double* cnt, void* G, const void* twx, const DDGeom& g, hipStream_t st) {
  return g.quad ? row_fwd<qd>(cnt, G, twx, g, st) : row_fwd<dd>(cnt, G, twx, g, st);
}

template <class R>
static hipError_t launch_fused(const void* Gin, void* Gout, const void* tabs, const void* tw, const DDFused& F0,
                               int64_t lines, hipStream_t st) {
  using C = cplx<R>;
  DDFused F = F0;
  F.log_lb = dd_log_lb<R>(F.M, lines);
  const size_t lds = ((size_t)F.M << F.log_lb) * sizeof(C);
  const unsigned blocks = (unsigned)(lines >> F.log_lb);
  const int nc = F.ch.C;
  const int nt = block_threads<R>(F.M << F.log_lb);
  const C* gi = (const C*)Gin;
  C* go = (C*)Gout;
  const R* tb = (const R*)tabs;
  const C* w = (const C*)tw;
  hipError_t e;
  if (nc > 1) {
    if ((F.M << F.log_lb) > kSpecPerThread * nt) return hipErrorInvalidValue;
    // four spectrum bins per thread where they suffice; eight otherwise
    // (double-double only: quad-double blocks of 256 threads up to 1024
    // elements and of 512 above cover every length up to 2048 with four)
    constexpr bool kEight = threads_of<R>() == kThreads;
    if (F.log_lb == 2 && (F.M << 2) <= 4 * nt) {
      if ((e = allow_lds(k_dd_col_fused<R, true, 4, 4>, lds)) != hipSuccess) return e;
      k_dd_col_fused<R, true, 4, 4><<<blocks, nt, lds, st>>>(gi, go, tb, w, F, nc);
    } else if (F.log_lb != 2 && F.M <= 4 * nt) {
      if ((e = allow_lds(k_dd_col_fused<R, true, 1, 4>, lds)) != hipSuccess) return e;
      k_dd_col_fused<R, true, 1, 4><<<blocks, nt, lds, st>>>(gi, go, tb, w, F, nc);
    } else if constexpr (kEight) {
      if (F.log_lb == 2) {
        if ((e = allow_lds(k_dd_col_fused<R, true, 4>, lds)) != hipSuccess) return e;
        k_dd_col_fused<R, true, 4><<<blocks, nt, lds, st>>>(gi, go, tb, w, F, nc);
      } else {
        if ((e = allow_lds(k_dd_col_fused<R, true, 1>, lds)) != hipSuccess) return e;
        k_dd_col_fused<R, true, 1><<<blocks, nt, lds, st>>>(gi, go, tb, w, F, nc);
      }
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    if (F.log_lb == 2) {
      if ((e = allow_lds(k_dd_col_fused<R, false, 4>, lds)) != hipSuccess) return e;
      k_dd_col_fused<R, false, 4><<<blocks, nt, lds, st>>>(gi, go, tb, w, F, nc);
    } else {
      if ((e = allow_lds(k_dd_col_fused<R, false, 1>, lds)) != hipSuccess) return e;
      k_dd_col_fused<R, false, 1><<<blocks, nt, lds, st>>>(gi, go, tb, w, F, nc);
    }
  }
  return hipGetLastError();
}

hipError_t dd_convolve_rows(const double* img, void* G, const void* twx, const DDGeom& g, hipStream_t st) {
  DDGeom rows = g;
  rows.ny = g.ny * g.nz;   // the image rows (z, y), y fastest
  return dd_launch_row_fwd(img, G, twx, rows, st);
}

template <class R>
static hipError_t convolve_columns(void* G, void* Gc, const void* tabs, const DDChannels& ch, const void* twy,
                                   const void* twz, const DDGeom& g, hipStream_t st) {
  using C = cplx<R>;
  hipError_t e = hipSuccess;
  if (g.ndim == 2) {
    const DDFused F{g.My, g.logMy, g.ny, g.Mx, (int64_t)g.ny * g.Mx, (int64_t)g.Mx * g.My, ch};
    return launch_fused<R>(G, Gc, tabs, twy, F, g.Mx, st);
  }
  const int64_t MyMx = (int64_t)g.My * g.Mx;
  // forward y: G [z][y < ny][kx] -> Gc [z][ky][kx]
  const int log_lb = dd_log_lb<R>(g.My, g.Mx);
  const DDLines yf{g.My, g.logMy, g.Mx, g.ny, g.My, (int64_t)g.nz * g.Mx, (int64_t)g.ny * g.Mx, g.Mx, MyMx, g.Mx,
                   log_lb};
  if ((e = launch_line_fwd<R, 0>((const C*)G, (C*)Gc, nullptr, (const C*)twy, yf, 0, st)) != hipSuccess) return e;
  // z lines (ky, kx): forward, times each spectrum, inverse -> G [c][z < nz][ky][kx]
  const DDFused F{g.Mz, g.logMz, g.nz, MyMx, (int64_t)g.nz * MyMx, MyMx * g.Mz, ch};
  e = launch_fused<R>(Gc, G, tabs, twz, F, MyMx, st);
  if (e != hipSuccess) return e;
  // inverse y: G [c z][ky][kx] -> Gc [c z][y < ny][kx]
  const DDLines yi{g.My, g.logMy, g.Mx, g.My, g.ny, (int64_t)ch.C * g.nz * g.Mx, MyMx, g.Mx, (int64_t)g.ny * g.Mx,
                   g.Mx, log_lb};
  if ((e = launch_line_inv<R>((const C*)G, (C*)Gc, (const C*)twy, yi, st)) != hipSuccess) return e;
  return hipGetLastError();
}
hipError_t dd_convolve_columns(void* G, void* Gc, const void* tabs, const DDChannels& ch, const void* twy,
                               const void* twz, const DDGeom& g, hipStream_t st) {
  if (ch.C < 1 || ch.C > kDDMaxChannels) return hipErrorInvalidValue;
  return g.quad ? convolve_columns<qd>(G, Gc, tabs, ch, twy, twz, g, st)
                : convolve_columns<dd>(G, Gc, tabs, ch, twy, twz, g, st);
}

template <class R>
static hipError_t row_inv_epi(const void* Gc, int C, const void* twx, double* S, double* grad, double* hess,
                              double* curv, const double* scal, const DDGeom& g, hipStream_t st) {
  using Cx = cplx<R>;
  DDGeom rows = g;
  rows.ny = g.ny * g.nz;
  const size_t lds = (size_t)g.Mx * sizeof(Cx);
  const hipError_t e = allow_lds(k_dd_row_inv_epi<R>, lds);
  if (e != hipSuccess) return e;
  k_dd_row_inv_epi<R><<<(unsigned)rows.ny, block_threads<R>(g.Mx), lds, st>>>((const Cx*)Gc, (const Cx*)twx, S, grad, hess, curv,
                                                                 scal, rows, C);
  return hipGetLastError();
}
hipError_t dd_launch_row_inv_epi(const void* Gc, int C, const void* twx, double* S, double* grad, double* hess,
                                 double* curv, const double* scal, const DDGeom& g, hipStream_t st) {
  if (g.nx > kMaxPerThread * kThreads) return hipErrorInvalidValue;
  return g.quad ? row_inv_epi<qd>(Gc, C, twx, S, grad, hess, curv, scal, g, st)
                : row_inv_epi<dd>(Gc, C, twx, S, grad, hess, curv, scal, g, st);
}

template <class R>
static hipError_t row_inv_plain(const void* Gc, int C, const void* twx, double* out, const DDGeom& g,
                                hipStream_t st) {
  using Cx = cplx<R>;
  DDGeom rows = g;
  rows.ny = g.ny * g.nz;
  const size_t lds = (size_t)g.Mx * sizeof(Cx);
  const hipError_t e = allow_lds(k_dd_row_inv_plain<R>, lds);
  if (e != hipSuccess) return e;
  k_dd_row_inv_plain<R><<<(unsigned)rows.ny, block_threads<R>(g.Mx), lds, st>>>((const Cx*)Gc, (const Cx*)twx, out, rows, C);
  return hipGetLastError();
}
hipError_t dd_launch_row_inv_plain(const void* Gc, int C, const void* twx, double* out, const DDGeom& g,
                                   hipStream_t st) {
  return g.quad ? row_inv_plain<qd>(Gc, C, twx, out, g, st) : row_inv_plain<dd>(Gc, C, twx, out, g, st);
}

hipError_t dd_launch_gather(const float* Y, int64_t K, const double* fields, const double* scal, float* dY,
                            double* partials, int max_blocks, int* n_blocks, const DDGeom& g, hipStream_t st) {
  int64_t blocks = (K + 255) / 256;
  if (blocks > max_blocks) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  *n_blocks = (int)blocks;
  k_dd_gather<<<(unsigned)blocks, 256, 0, st>>>(Y, K, fields, scal, dY, partials, g);
  return hipGetLastError();
}

}  // namespace dt
