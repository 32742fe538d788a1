// Adjoint of the distance field (not in the paper; derived from Sec. 2.3,
// eq. STilde).  For a loss with G = dL/dS on the grid:
//   dS(X)/dY_k = -p_k(X) n_k(X),  p_k = exp(-r_k/tau)/phi,  n_k = (X - Y_k)/r_k
//   => dL/dY_k = -sum_X w(X) u(X - Y_k) = (w * u)(Y_k),   w = G/phi = G exp(S/tau)
// because the gradient kernel u(Z) = (Z/|Z|) exp(-|Z|/tau) is odd; the same
// kernel spectra as the forward gradient are reused.  For tau:
//   dS/dtau = (S - <r>)/tau, <r> = ((r f) * g)/phi, and
//   sum_X G <r> = sum_k (w * (r f))(Y_k)  (r f is even),
// so dL/dtau = (sum_valid G S - sum_k (w * rf)(Y_k)) / tau.
// Truncated nodes (S >= S_max) hold a constant and get w = 0.
#include <math.h>

#include "dt_launch.hpp"
#include "fft_engine.hpp"

namespace dt {

// w = G exp(S/tau) * 2^floor(log2 Theta) on valid nodes, else 0; per-block
// partial sums of G*S over valid nodes.  The power-of-two factor keeps
// |w| <= |G| (phi >= Theta on valid nodes).
template <typename T>
__global__ void __launch_bounds__(256) k_prep_w(const T* __restrict__ S, const T* __restrict__ G, int64_t n,
                                                const double* __restrict__ scal, double tau, T* __restrict__ w,
                                                double* __restrict__ partials) {
  __shared__ double red[256];
  const T smax = (T)scal[1];
  const T p2 = (T)scal[3];
  const T itau = (T)(1.0 / tau);
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T s = S[i];
    const T gv = G[i];
    const bool valid = s < smax;
    w[i] = valid ? gv * (exp(s * itau) * p2) : T(0);
    if (valid) acc += (double)gv * (double)s;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

template <typename T> int launch_prep_w(const T* S, const T* G, int64_t n, const double* scal, double tau, T* w,
                                        double* partials, hipStream_t st) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_prep_w<T>, dim3(blocks), dim3(256), 0, st, S, G, n, scal, tau, w, partials);
  return blocks;
}
template int launch_prep_w<float>(const float*, const float*, int64_t, const double*, double, float*, double*,
                                  hipStream_t);
template int launch_prep_w<double>(const double*, const double*, int64_t, const double*, double, double*,
                                   double*, hipStream_t);

// One wavefront per source: evaluate the real inverse x-transform of each
// channel's half-spectrum row at the source's x node,
//   x[m] = X[0] + (-1)^m X[M/2] + 2 Re sum_{k=1}^{M/2-1} X[k] exp(2 pi i k m / M),
// and write dL/dY.  Per-block sums of the r f channel go to partials.
template <typename T>
__global__ void __launch_bounds__(256) k_gather(GatherParams p) {
  using V = Cx<T>;
  __shared__ double red[4];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int nch = p.nu + (p.has_rf ? 1 : 0);
  const double inv_p2 = 1.0 / p.scal[3];
  const V* tw = (const V*)p.tw;
  const int half = p.Mx / 2;
  double rf_sum = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 4 + wv; k < p.K; k += (int64_t)gridDim.x * 4) {
    double y[3];
    for (int d = 0; d < p.g.ndim; ++d) y[d] = (double)p.Y[k * p.g.ndim + d];
    bool ok = true;
    int idx[3] = {0, 0, 0};
    for (int d = 0; d < p.g.ndim; ++d) {
      const double qd = floor((y[d] - p.g.o[d]) / p.g.h[d]);
      if (!(qd >= 0.0 && qd < (double)p.g.n[d])) ok = false; else idx[d] = (int)qd;
    }
    double accs[4] = {0.0, 0.0, 0.0, 0.0};
    if (ok) {
      const int64_t row = idx[1] + (p.g.ndim == 3 ? (int64_t)p.g.n[1] * idx[2] : 0);
      // twiddle index (kk x) mod M, advanced by (64 x) mod M per step
      // (x < n <= 1024, M <= 2048: the products fit 32 bits)
      const int step = (64 * idx[0]) % p.Mx;
      int m = (lane * idx[0]) % p.Mx;
      const V* base = (const V*)p.spec + row * p.pitch;
      // kU bins per lane per round, all loads issued before the sums (the
      // order of the sums is that of kk, as one bin at a time)
      constexpr int kU = 4;
      for (int kk0 = lane; kk0 <= half; kk0 += 64 * kU) {
        V w[kU], X[kU][4];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int kk = kk0 + 64 * u;
          const bool on = kk <= half;
          w[u] = on ? cconj(tw[m]) : mk<V>(T(0), T(0));   // exp(+2 pi i kk x / M)
          m += step;
          if (m >= p.Mx) m -= p.Mx;
#pragma unroll
          for (int c = 0; c < 4; ++c)
            X[u][c] = (on && c < nch) ? base[(int64_t)c * p.ch_stride + kk] : mk<V>(T(0), T(0));
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int kk = kk0 + 64 * u;
          if (kk > half) break;
          const double wt = (kk == 0 || kk == half) ? 1.0 : 2.0;
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (c < nch) accs[c] += wt * (double)(X[u][c].x * w[u].x - X[u][c].y * w[u].y);
        }
      }
    }
    for (int c = 0; c < nch; ++c) {
      double a = accs[c];
      for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
      accs[c] = a * p.ch_scale[c] * inv_p2;
    }
    if (lane == 0) {
      for (int d = 0; d < p.nu; ++d) p.dY[k * p.nu + d] = ok ? (float)accs[d] : 0.0f;
      if (p.has_rf && ok) rf_sum += accs[p.nu];
    }
  }
  if (lane == 0) red[wv] = rf_sum;
  __syncthreads();
  if (threadIdx.x == 0 && p.partials) p.partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T> int launch_gather(const GatherParams& p, hipStream_t st) {
  int64_t blocks = (p.K + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  if (blocks <= 0) return 0;
  hipLaunchKernelGGL(k_gather<T>, dim3((unsigned)blocks), dim3(256), 0, st, p);
  return (int)blocks;
}
template int launch_gather<float>(const GatherParams&, hipStream_t);
template int launch_gather<double>(const GatherParams&, hipStream_t);

// dL/dtau = (sum_valid G S - sum_k (w * rf)(Y_k)) / tau
__global__ void __launch_bounds__(256) k_finalize_dtau(const double* __restrict__ gs, int n_gs,
                                                       const double* __restrict__ rf, int n_rf, double tau,
                                                       double* __restrict__ scal, double* __restrict__ user_out) {
  __shared__ double r1[256], r2[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n_gs; i += blockDim.x) a += gs[i];
  for (int i = threadIdx.x; i < n_rf; i += blockDim.x) b += rf[i];
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r1[threadIdx.x] += r1[threadIdx.x + s];
      r2[threadIdx.x] += r2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = (r1[0] - r2[0]) / tau;
    scal[4] = v;
    if (user_out) *user_out = v;
  }
}

void launch_finalize_dtau(const double* gs_partials, int n_gs, const double* rf_partials, int n_rf,
                          double rf_scale, double tau, double* scal, double* user_out, hipStream_t st) {
  (void)rf_scale;
  hipLaunchKernelGGL(k_finalize_dtau, dim3(1), dim3(256), 0, st, gs_partials, n_gs, rf_partials, n_rf, tau, scal,
                     user_out);
}

}  // namespace dt
