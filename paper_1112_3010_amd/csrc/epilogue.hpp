// Per-node epilogue of the final row pass (Table 1 step 6 and Sec. 5):
// undo the power-of-two scales, validity test against Theta, S = -tau log phi,
// gradient u / phi, Hessian h / phi + S_i S_j / tau, winding number or degree
// and the sign label.
#pragma once

#include "dt_internal.hpp"

namespace dt {

// Natural log and reciprocal for the epilogue.  float32 uses the hardware
// log2 and reciprocal (about one ulp), far below the float32 convolution
// error the validity threshold admits; float64 keeps the IEEE routines.
__device__ __forceinline__ float epi_log(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309417f; }
__device__ __forceinline__ double epi_log(double x) { return log(x); }
__device__ __forceinline__ float epi_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double epi_rcp(double x) { return 1.0 / x; }

__device__ __forceinline__ void hess_pair(int ndim, int h, int& i, int& j) {
  if (ndim == 2) {
    const int a[3] = {0, 0, 1}, c[3] = {0, 1, 1};
    i = a[h]; j = c[h];
  } else {
    const int a[6] = {0, 0, 0, 1, 1, 2}, c[6] = {0, 1, 2, 1, 2, 2};
    i = a[h]; j = c[h];
  }
}

template <typename T>
__device__ __forceinline__ void epilogue_cell(const EpiParams& e, const T* vals, int64_t node) {
  const T theta = (T)e.theta[0];
  const T smax = (T)e.theta[1];
  const T tau = (T)e.tau;
  T label = T(1);
  if (e.ch_mu >= 0) {
    const T mu = vals[e.ch_mu] * (T)e.scale_mu;
    label = mu >= T(0.5) ? T(1) : T(-1);
    if (e.label) e.label[node] = (int8_t)(mu >= T(0.5) ? 1 : -1);
    if (e.mu) ((T*)e.mu)[node] = mu;
  }
  if (e.ch_phi < 0) return;
  const T cphi = vals[e.ch_phi];
  const T phi = cphi * (T)e.scale_phi;
  const bool valid = phi >= theta;
  const T sgn = (e.signed_out && e.ch_mu >= 0) ? label : T(1);
  if (e.S) ((T*)e.S)[node] = sgn * (valid ? -tau * epi_log(phi) : smax);
  if (e.ch_u[0] < 0) return;
  T g[3] = {T(0), T(0), T(0)};
  const T inv = valid ? epi_rcp(cphi) : T(0);
  for (int a = 0; a < e.ndim; ++a) g[a] = valid ? vals[e.ch_u[a]] * inv * (T)e.scale_u[a] : T(0);
  if (e.grad)
    for (int a = 0; a < e.ndim; ++a) ((T*)e.grad)[a * e.plane + node] = sgn * g[a];
  if (e.hess && e.ch_h[0] >= 0) {
    const int nh = e.ndim == 2 ? 3 : 6;
    for (int h = 0; h < nh; ++h) {
      int i, j;
      hess_pair(e.ndim, h, i, j);
      const T hv = valid ? vals[e.ch_h[h]] * inv * (T)e.scale_h[h] + g[i] * g[j] / tau : T(0);
      ((T*)e.hess)[h * e.plane + node] = hv;
    }
  }
}

}  // namespace dt
