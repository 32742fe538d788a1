// Source images, validity scalars and plan-time kernel spectra.
//
//  * splat: sources are snapped to grid nodes (the method works with sources
//    on the grid, Sec. 3, eqs. function_g and krondelta; sampled inputs are
//    rounded to nodes, Sec. 6) and accumulated with multiplicity into the
//    count image g.  For the sign, the weight images g_1, g_2 (2D, tangents
//    Z_k, Sec. 4.1 eq. tangentVec) or g_1..g_3 (3D, area vectors P_k at the
//    triangle incenters, Sec. 4.2) are accumulated the same way.
//  * validity: ||g||_2 and the threshold Theta of the library's contract.
//  * kernel spectra (plan time): every kernel has a definite parity on every
//    axis, so its DFT is (-i)^(#odd axes) times a real table that is a
//    cosine/sine transform over the folded displacement range; it is
//    evaluated in float64 by three separable direct sums.
#include "dt_launch.hpp"

#include <math.h>

namespace dt {

// ---------------------------------------------------------------------------
// Fill
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_fill_zero(T* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = T(0);
}

template <typename T> void launch_fill_zero(T* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_zero<T>, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
}
template void launch_fill_zero<float>(float*, int64_t, hipStream_t);
template void launch_fill_zero<double>(double*, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// Snapping (float64, IEEE division and floor)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool snap_node(const GridGeom& g, const double* y, int64_t& lin, int* idx,
                                          uint32_t* err) {
  bool finite = true, inside = true;
  for (int d = 0; d < g.ndim; ++d) {
    if (!isfinite(y[d])) { finite = false; break; }
    const double q = floor((y[d] - g.o[d]) / g.h[d]);
    if (!(q >= 0.0 && q < (double)g.n[d])) { inside = false; break; }
    idx[d] = (int)q;
  }
  if (!finite || !inside) {
    if (err) atomicOr(err, finite ? kErrRange : kErrNonFinite);
    return false;
  }
  lin = idx[0] + (int64_t)g.n[0] * (idx[1] + (g.ndim == 3 ? (int64_t)g.n[1] * idx[2] : 0));
  return true;
}

// Sum of squared multiplicities, accumulated while splatting: adding one
// source to a node that already holds m of them raises sum m^2 by 2m + 1.
// Every lane of the wave takes part (lanes without a source add 0), then one
// atomic per wave.
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) {
    const int hi = __shfl_xor(__double2hiint(v), off);
    const int lo = __shfl_xor(__double2loint(v), off);
    v += __hiloint2double(hi, lo);
  }
  return v;
}
__device__ __forceinline__ void msq_add(double inc, double* msq) {
  if (!msq) return;
  const double s = wave_sum(inc);
  if ((threadIdx.x & 63) == 0 && s != 0.0) atomicAdd(msq, s);
}
// Add one (scaled) source to the count image; returns the increment of sum m^2.
template <typename T> __device__ __forceinline__ double count_add(T* cnt, int64_t lin, T cval, double inv_cval) {
  const T old = atomicAdd(&cnt[lin], cval);
  return 2.0 * ((double)old * inv_cval) + 1.0;
}

// Point sources: count image only.
template <typename T>
__global__ void __launch_bounds__(256) k_splat_points(const float* __restrict__ Y, int64_t K, GridGeom g,
                                                      T* __restrict__ cnt, T cval, double inv_cval, double* msq,
                                                      uint32_t* err) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double inc = 0.0;
  if (k < K) {
    double y[3];
    for (int d = 0; d < g.ndim; ++d) y[d] = (double)Y[k * g.ndim + d];
    int idx[3];
    int64_t lin;
    if (snap_node(g, y, lin, idx, err)) inc = count_add(cnt, lin, cval, inv_cval);
  }
  msq_add(inc, msq);
}

// Closed polygon: optional count image, tangent images g1 (Z^1) and g2 (Z^2)
// with Z_k = Yhat_{k+1} - Yhat_k on the snapped points (wrapping at K).
template <typename T>
__global__ void __launch_bounds__(256) k_splat_polygon(const float* __restrict__ P, int64_t K, GridGeom g,
                                                       T* __restrict__ cnt, T cval, double inv_cval, double* msq,
                                                       T* __restrict__ g1, T* __restrict__ g2, double w1, double w2,
                                                       uint32_t* err) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double inc = 0.0;
  if (k < K) {
    const int64_t kn = (k + 1 == K) ? 0 : k + 1;
    double y[2] = {(double)P[2 * k], (double)P[2 * k + 1]};
    double yn[2] = {(double)P[2 * kn], (double)P[2 * kn + 1]};
    int idx[3], idn[3];
    int64_t lin, linn;
    if (snap_node(g, y, lin, idx, err)) {
      if (cnt) inc = count_add(cnt, lin, cval, inv_cval);
      // the next point reports its own error
      if (g1 && snap_node(g, yn, linn, idn, nullptr)) {
        const double zx = (double)(idn[0] - idx[0]) * g.h[0];
        const double zy = (double)(idn[1] - idx[1]) * g.h[1];
        atomicAdd(&g1[lin], (T)(zx * w1));
        atomicAdd(&g2[lin], (T)(zy * w2));
      }
    }
  }
  msq_add(inc, msq);
}

// Incenter and area vector of one triangle.  The incenter order of
// operations is fixed (the snapped node must not depend on contraction):
// a = |v1 - v2|, b = |v2 - v0|, c = |v0 - v1|, |u| = sqrt((ux*ux + uy*uy) + uz*uz),
// incenter = ((a*v0 + b*v1) + c*v2) / ((a + b) + c).
__device__ __forceinline__ void triangle_sources(const double* v0, const double* v1, const double* v2,
                                                 double* inc, double* area) {
#pragma clang fp contract(off)
  double e12[3], e20[3], e01[3];
  for (int d = 0; d < 3; ++d) {
    e12[d] = v1[d] - v2[d];
    e20[d] = v2[d] - v0[d];
    e01[d] = v0[d] - v1[d];
  }
  const double a = sqrt((e12[0] * e12[0] + e12[1] * e12[1]) + e12[2] * e12[2]);
  const double b = sqrt((e20[0] * e20[0] + e20[1] * e20[1]) + e20[2] * e20[2]);
  const double c = sqrt((e01[0] * e01[0] + e01[1] * e01[1]) + e01[2] * e01[2]);
  const double den = (a + b) + c;
  for (int d = 0; d < 3; ++d) inc[d] = ((a * v0[d] + b * v1[d]) + c * v2[d]) / den;
  double u[3], w[3];
  for (int d = 0; d < 3; ++d) {
    u[d] = v1[d] - v0[d];
    w[d] = v2[d] - v0[d];
  }
  area[0] = 0.5 * (u[1] * w[2] - u[2] * w[1]);
  area[1] = 0.5 * (u[2] * w[0] - u[0] * w[2]);
  area[2] = 0.5 * (u[0] * w[1] - u[1] * w[0]);
}

// Closed triangle mesh: optional count image at the snapped incenters and
// area-vector images gp[0..2].
template <typename T>
__global__ void __launch_bounds__(256) k_splat_mesh(const float* __restrict__ V, int64_t nv,
                                                    const int32_t* __restrict__ F, int64_t nf, GridGeom g,
                                                    T* __restrict__ cnt, T cval, double inv_cval, double* msq,
                                                    T* __restrict__ gp0, T* __restrict__ gp1, T* __restrict__ gp2,
                                                    double w0, double w1, double w2, uint32_t* err) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double inc = 0.0;
  if (f < nf) {
    double v[3][3];
    bool ok = true;
    for (int c = 0; c < 3 && ok; ++c) {
      const int32_t vi = F[3 * f + c];
      if (vi < 0 || (int64_t)vi >= nv) {
        atomicOr(err, kErrRange);
        ok = false;
      } else {
        for (int d = 0; d < 3; ++d) v[c][d] = (double)V[3 * (int64_t)vi + d];
      }
    }
    double incr[3], area[3];
    int idx[3];
    int64_t lin;
    if (ok) {
      triangle_sources(v[0], v[1], v[2], incr, area);
      if (snap_node(g, incr, lin, idx, err)) {
        if (cnt) inc = count_add(cnt, lin, cval, inv_cval);
        if (gp0) {
          atomicAdd(&gp0[lin], (T)(area[0] * w0));
          atomicAdd(&gp1[lin], (T)(area[1] * w1));
          atomicAdd(&gp2[lin], (T)(area[2] * w2));
        }
      }
    }
  }
  msq_add(inc, msq);
}

template <typename T> void launch_splat_points(const float* Y, int64_t K, const GridGeom& g, T* cnt, T cval,
                                               double inv_cval, double* msq, uint32_t* err, hipStream_t st) {
  if (K <= 0) return;
  hipLaunchKernelGGL(k_splat_points<T>, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, Y, K, g, cnt, cval,
                     inv_cval, msq, err);
}
template <typename T> void launch_splat_polygon(const float* P, int64_t K, const GridGeom& g, T* cnt, T cval,
                                                double inv_cval, double* msq, T* g1, T* g2, double w1, double w2,
                                                uint32_t* err, hipStream_t st) {
  if (K <= 0) return;
  hipLaunchKernelGGL(k_splat_polygon<T>, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, P, K, g, cnt,
                     cval, inv_cval, msq, g1, g2, w1, w2, err);
}
template <typename T> void launch_splat_mesh(const float* V, int64_t nv, const int32_t* F, int64_t nf,
                                             const GridGeom& g, T* cnt, T cval, double inv_cval, double* msq, T* gp0,
                                             T* gp1, T* gp2, double w0, double w1, double w2, uint32_t* err,
                                             hipStream_t st) {
  if (nf <= 0) return;
  hipLaunchKernelGGL(k_splat_mesh<T>, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, V, nv, F, nf, g,
                     cnt, cval, inv_cval, msq, gp0, gp1, gp2, w0, w1, w2, err);
}
#define DT_INST_SPLAT(T)                                                                                   \
  template void launch_splat_points<T>(const float*, int64_t, const GridGeom&, T*, T, double, double*,    \
                                       uint32_t*, hipStream_t);                                           \
  template void launch_splat_polygon<T>(const float*, int64_t, const GridGeom&, T*, T, double, double*,   \
                                        T*, T*, double, double, uint32_t*, hipStream_t);                  \
  template void launch_splat_mesh<T>(const float*, int64_t, const int32_t*, int64_t, const GridGeom&, T*, \
                                     T, double, double*, T*, T*, T*, double, double, double, uint32_t*,    \
                                     hipStream_t);
DT_INST_SPLAT(float)
DT_INST_SPLAT(double)

// ---------------------------------------------------------------------------
// Validity scalars: Theta = c * u * log2(N_pad) * ||f||_1 * ||g||_2 / sqrt(N_pad)
// ---------------------------------------------------------------------------
// Validity scalars from the sum of squared multiplicities accumulated by the
// splat (msq[0]), which is cleared for the next call.
__global__ void k_finalize_theta_msq(double* __restrict__ msq, double coef, double tau, double* __restrict__ scal) {
  if (threadIdx.x != 0) return;
  const double gl2 = sqrt(msq[0]);
  msq[0] = 0.0;
  const double theta = coef * gl2;
  scal[0] = theta;
  scal[1] = -tau * log(theta);
  scal[2] = gl2;
  int e;
  frexp(theta, &e);
  scal[3] = ldexp(1.0, e - 1);
}
void launch_finalize_theta_msq(double* msq, double coef, double tau, double* scal, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_theta_msq, dim3(1), dim3(64), 0, st, msq, coef, tau, scal);
}


// ---------------------------------------------------------------------------
// Plan-time kernel spectra
// ---------------------------------------------------------------------------
// Kernel values at physical displacement D (kind, axes i, j); all are 0 at
// D = 0 except f (1 there).
__device__ double kernel_value(const TabKernel& kd, const double* D, int ndim) {
  double r2 = 0.0;
  for (int a = 0; a < ndim; ++a) r2 += D[a] * D[a];
  const double r = sqrt(r2);
  const double tau = kd.tau;
  if (r == 0.0) return kd.kind == KER_F ? 1.0 : 0.0;
  const double f = exp(-r / tau);
  switch (kd.kind) {
    case KER_F: return f;
    case KER_U: return D[kd.i] / r * f;
    case KER_H: {
      const double ni = D[kd.i] / r, nj = D[kd.j] / r;
      const double delta = kd.i == kd.j ? 1.0 : 0.0;
      return (-ni * nj / tau + (delta - ni * nj) / r) * f;
    }
    case KER_W2: return kd.coef * D[kd.i] / r2;             // winding-number kernels
    case KER_D3: return kd.coef * D[kd.i] / (r2 * r);       // topological-degree kernels
    case KER_RF: return r * f;
  }
  return 0.0;
}

// Sample on the folded range d_a in [0, Mh_a) (d_a = M_a/2 set to zero) and
// accumulate the l1 norm over the full padded grid (weights 1 at d = 0, 2 else).
__global__ void __launch_bounds__(256) k_tab_sample(TabKernel kd, TabGeom tg, double* __restrict__ out,
                                                    double* __restrict__ partials) {
  __shared__ double red[256];
  const int64_t total = (int64_t)tg.H[0] * tg.H[1] * tg.H[2];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    int d[3];
    d[0] = (int)(i % tg.H[0]);
    d[1] = (int)((i / tg.H[0]) % tg.H[1]);
    d[2] = (int)(i / ((int64_t)tg.H[0] * tg.H[1]));
    bool nyq = false;
    double w = 1.0, D[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < tg.ndim; ++a) {
      if (2 * d[a] == tg.M[a]) nyq = true;
      if (tg.cut[a] > 0 && d[a] > tg.cut[a]) nyq = true;   // outside the truncation box: 0 as well
      if (d[a] > 0) w *= 2.0;
      D[a] = (double)d[a] * tg.h[a];
    }
    const double val = nyq ? 0.0 : kernel_value(kd, D, tg.ndim);
    out[i] = val;
    acc += w * fabs(val);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// One separable stage along `axis`: out(k) = sum_{d < M/2} c_d in(d) trig(2 pi k d / M),
// trig = cos for an even axis, sin for an odd one, c_0 = 1, c_d = 2, for every
// line of the folded grid along that axis.  Written as the product of the
// H x M/2 matrix C(k, d) = c_d trig(2 pi k d / M) with the lines: a block
// computes a 64 x 64 tile of (k, line) outputs, staging 16-deep slices of C
// and of the input lines in LDS; each thread keeps a 4 x 4 tile of sums,
// accumulated in increasing d.
constexpr int kTabTK = 64, kTabTC = 64, kTabTD = 16;
__global__ void __launch_bounds__(256) k_tab_axis(TabGeom tg, int axis, int odd, const double2* __restrict__ trig,
                                                  const double* __restrict__ in, double* __restrict__ out) {
  __shared__ double sC[kTabTD][kTabTK + 1];
  __shared__ double sX[kTabTD][kTabTC + 1];
  const int H = tg.H[axis], M = tg.M[axis], Dn = M / 2;
  int64_t L = 1, U = 1;   // line count below and above the axis
  for (int a = 0; a < 3; ++a) {
    if (a < axis) L *= tg.H[a];
    if (a > axis) U *= tg.H[a];
  }
  const int64_t ncol = L * U;
  const int k0 = blockIdx.y * kTabTK;
  const int64_t c0 = (int64_t)blockIdx.x * kTabTC;
  const int tid = threadIdx.x;
  const int tk = tid / 16, tc = tid % 16;     // outputs k0 + 4 tk + i, columns c0 + tc + 16 j
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int d0 = 0; d0 < Dn; d0 += kTabTD) {
    for (int e = tid; e < kTabTD * kTabTK; e += 256) {
      const int dd = e / kTabTK, kk = e % kTabTK;
      const int d = d0 + dd, k = k0 + kk;
      double v = 0.0;
      if (d < Dn && k < H) {
        const double2 w = trig[(int)(((int64_t)k * d) % M)];   // (cos, -sin) of 2 pi k d / M
        v = (d == 0 ? 1.0 : 2.0) * (odd ? -w.y : w.x);
      }
      sC[dd][kk] = v;
    }
    for (int e = tid; e < kTabTD * kTabTC; e += 256) {
      const int dd = e / kTabTC, cc = e % kTabTC;
      const int d = d0 + dd;
      const int64_t col = c0 + cc;
      double v = 0.0;
      if (d < Dn && col < ncol) {
        const int64_t hi = col / L, lo = col - hi * L;
        v = in[(hi * H + d) * L + lo];
      }
      sX[dd][cc] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int dd = 0; dd < kTabTD; ++dd) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sC[dd][4 * tk + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sX[dd][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = c0 + tc + 16 * j;
    if (col >= ncol) continue;
    const int64_t hi = col / L, lo = col - hi * L;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = k0 + 4 * tk + i;
      if (k < H) out[(hi * H + k) * L + lo] = acc[i][j];
    }
  }
}

// Store in the tile-major layout read by the fused pass: element (x, y, z)
// of the folded range goes to ((outer * tiles + x / nb) * H_line + line) * nb + x % nb
// with (line, outer) = (z, y) in 3D and (y, -) in 2D.
template <typename T>
__global__ void __launch_bounds__(256) k_tab_store(TabGeom tg, const double* __restrict__ in, double scale,
                                                   T* __restrict__ out, int nb, int tiles) {
  const int64_t total = (int64_t)tg.H[0] * tg.H[1] * tg.H[2];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t x = i % tg.H[0];
  const int64_t y = (i / tg.H[0]) % tg.H[1];
  const int64_t z = i / ((int64_t)tg.H[0] * tg.H[1]);
  const int64_t line = tg.ndim == 3 ? z : y;
  const int64_t outer = tg.ndim == 3 ? y : 0;
  const int64_t H_line = tg.ndim == 3 ? tg.H[2] : tg.H[1];
  out[((outer * tiles + x / nb) * H_line + line) * nb + x % nb] = (T)(in[i] * scale);
}

int launch_tab_sample(const TabKernel& kd, const TabGeom& tg, double* out, double* partials, hipStream_t st) {
  const int64_t total = (int64_t)tg.H[0] * tg.H[1] * tg.H[2];
  int blocks = (int)((total + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_tab_sample, dim3(blocks), dim3(256), 0, st, kd, tg, out, partials);
  return blocks;
}
void launch_tab_axis(const TabGeom& tg, int axis, int odd, const void* trig, const double* in, double* out,
                     hipStream_t st) {
  const int64_t total = (int64_t)tg.H[0] * tg.H[1] * tg.H[2];
  const int64_t ncol = total / tg.H[axis];
  const dim3 grid((unsigned)((ncol + kTabTC - 1) / kTabTC), (unsigned)((tg.H[axis] + kTabTK - 1) / kTabTK));
  hipLaunchKernelGGL(k_tab_axis, grid, dim3(256), 0, st, tg, axis, odd, (const double2*)trig, in, out);
}
template <typename T> void launch_tab_store(const TabGeom& tg, const double* in, double scale, T* out, int nb,
                                            int tiles, hipStream_t st) {
  const int64_t total = (int64_t)tg.H[0] * tg.H[1] * tg.H[2];
  hipLaunchKernelGGL(k_tab_store<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, tg, in, scale, out,
                     nb, tiles);
}
template void launch_tab_store<float>(const TabGeom&, const double*, double, float*, int, int, hipStream_t);
template void launch_tab_store<double>(const TabGeom&, const double*, double, double*, int, int, hipStream_t);

}  // namespace dt
