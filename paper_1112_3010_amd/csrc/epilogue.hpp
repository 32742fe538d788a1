// Per-node epilogue of the final row pass (Table 1 step 6 and Sec. 5):
// undo the power-of-two scales, validity test against Theta, S = -tau log phi,
// gradient u / phi, Hessian h / phi + S_i S_j / tau, curvatures, winding
// number or degree and the sign label.
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

// Curvatures from grad S (g) and the Hessian (h, library channel order), the
// derived quantities named at the end of Sec. 5.  c = mean, Gaussian, k1, k2
// with k1,2 = mean +/- sqrt(max(mean^2 - Gaussian, 0)).
template <typename T> __device__ __forceinline__ void principal(T mean, T gauss, T* c) {
  const T s = sqrt(fmax(mean * mean - gauss, T(0)));
  c[0] = mean;
  c[1] = gauss;
  c[2] = mean + s;
  c[3] = mean - s;
}
// 2D: the graph surface (x, y, S) with the upward normal; h = xx, xy, yy.
template <typename T> __device__ __forceinline__ void curvature_graph(const T* g, const T* h, T* c) {
  const T gx2 = g[0] * g[0], gy2 = g[1] * g[1];
  const T W = T(1) + gx2 + gy2;
  const T gauss = (h[0] * h[2] - h[1] * h[1]) / (W * W);
  const T mean = ((T(1) + gy2) * h[0] - T(2) * g[0] * g[1] * h[1] + (T(1) + gx2) * h[2]) / (T(2) * W * sqrt(W));
  principal(mean, gauss, c);
}
// |grad S| below which the 3D level surface is not defined by the derivatives
constexpr double kCurvGradMin = 1e-3;
// 3D: the level surface of S through the node, normal g / |g|;
// h = xx, xy, xz, yy, yz, zz.  Mean (|g|^2 tr h - g^T h g) / (2 |g|^3),
// Gaussian g^T adj(h) g / |g|^4.
template <typename T> __device__ __forceinline__ void curvature_level_set(const T* g, const T* h, T* c) {
  const T a = h[0], b = h[1], cc = h[2], d = h[3], e = h[4], f = h[5];
  const T q = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  if (!(q >= T(kCurvGradMin * kCurvGradMin))) {
    c[0] = c[1] = c[2] = c[3] = T(0);
    return;
  }
  const T gHg = g[0] * g[0] * a + g[1] * g[1] * d + g[2] * g[2] * f +
                T(2) * (g[0] * g[1] * b + g[0] * g[2] * cc + g[1] * g[2] * e);
  // adjugate of the symmetric Hessian
  const T A00 = d * f - e * e, A01 = cc * e - b * f, A02 = b * e - cc * d;
  const T A11 = a * f - cc * cc, A12 = b * cc - a * e, A22 = a * d - b * b;
  const T gAg = g[0] * g[0] * A00 + g[1] * g[1] * A11 + g[2] * g[2] * A22 +
                T(2) * (g[0] * g[1] * A01 + g[0] * g[2] * A02 + g[1] * g[2] * A12);
  const T mean = (q * (a + d + f) - gHg) / (T(2) * q * sqrt(q));
  const T gauss = gAg / (q * q);
  principal(mean, gauss, c);
}

// Per-call constants of the epilogue, read once per thread (the threshold
// from the device and the power-of-two scales), so that the per-node code
// reads nothing but the node's channels.
template <typename T> struct EpiConst {
  T theta, smax, tau, inv_tau, scale_phi, scale_mu;
  T scale_u[3], scale_h[6];
};
template <typename T> __device__ __forceinline__ EpiConst<T> epi_const(const EpiParams& e) {
  EpiConst<T> k;
  k.theta = (T)e.theta[0];
  k.smax = (T)e.theta[1];
  k.tau = (T)e.tau;
  k.inv_tau = (T)(1.0 / e.tau);
  k.scale_phi = (T)e.scale_phi;
  k.scale_mu = (T)e.scale_mu;
#pragma unroll
  for (int a = 0; a < 3; ++a) k.scale_u[a] = (T)e.scale_u[a];
#pragma unroll
  for (int h = 0; h < 6; ++h) k.scale_h[h] = (T)e.scale_h[h];
  return k;
}

// Hessian of S in D dimensions from the channels: h / phi + S_i S_j / tau, in
// the library's channel order (xx, xy, [xz,] yy, [yz,] zz).
template <typename T, int D, typename Ch>
__device__ __forceinline__ void hessian_of(const EpiParams& e, const EpiConst<T>& k, const Ch& ch, bool valid, T inv,
                                           const T* g, T* hv) {
  constexpr int NH = D == 2 ? 3 : 6;
  constexpr int I[6] = {0, 0, D == 2 ? 1 : 0, 1, 1, 2};
  constexpr int J[6] = {0, 1, D == 2 ? 1 : 2, 1, 2, 2};
#pragma unroll
  for (int h = 0; h < NH; ++h)
    hv[h] = valid ? ch(e.ch_h[h]) * inv * k.scale_h[h] + g[I[h]] * g[J[h]] * k.inv_tau : T(0);
}

// One node of the final row pass.  ch(c) returns channel c of the node.
// CURV: the instantiation that also writes curvatures (kept apart so that the
// other outputs' final pass keeps its register budget).
template <typename T, bool CURV, typename Ch>
__device__ __forceinline__ void epilogue_node(const EpiParams& e, const EpiConst<T>& k, const Ch& ch, int64_t node) {
  T label = T(1);
  if (e.ch_mu >= 0) {
    const T mu = ch(e.ch_mu) * k.scale_mu;
    label = mu >= T(0.5) ? T(1) : T(-1);
    if (e.label) e.label[node] = (int8_t)(mu >= T(0.5) ? 1 : -1);
    if (e.mu) ((T*)e.mu)[node] = mu;
  }
  if (e.ch_phi < 0) return;
  const T cphi = ch(e.ch_phi);
  const T phi = cphi * k.scale_phi;
  const bool valid = phi >= k.theta;
  const T sgn = (e.signed_out && e.ch_mu >= 0) ? label : T(1);
  if (e.S) ((T*)e.S)[node] = sgn * (valid ? -k.tau * epi_log(phi) : k.smax);
  if (e.ch_u[0] < 0) return;
  const bool d3 = e.ndim == 3;
  const T inv = valid ? epi_rcp(cphi) : T(0);
  T g[3];
  g[0] = valid ? ch(e.ch_u[0]) * inv * k.scale_u[0] : T(0);
  g[1] = valid ? ch(e.ch_u[1]) * inv * k.scale_u[1] : T(0);
  g[2] = (d3 && valid) ? ch(e.ch_u[2]) * inv * k.scale_u[2] : T(0);
  if (e.grad) {
    T* gr = (T*)e.grad;
    gr[node] = sgn * g[0];
    gr[e.plane + node] = sgn * g[1];
    if (d3) gr[2 * e.plane + node] = sgn * g[2];
  }
  if constexpr (!CURV) {
    if (e.hess && e.ch_h[0] >= 0) {
      T hv[6];
      T* hs = (T*)e.hess;
      if (d3) {
        hessian_of<T, 3>(e, k, ch, valid, inv, g, hv);
#pragma unroll
        for (int h = 0; h < 6; ++h) hs[h * e.plane + node] = hv[h];
      } else {
        hessian_of<T, 2>(e, k, ch, valid, inv, g, hv);
#pragma unroll
        for (int h = 0; h < 3; ++h) hs[h * e.plane + node] = hv[h];
      }
    }
  } else {
    T hv[6];
    T c[4];
    if (d3) {
      hessian_of<T, 3>(e, k, ch, valid, inv, g, hv);
      curvature_level_set(g, hv, c);
    } else {
      hessian_of<T, 2>(e, k, ch, valid, inv, g, hv);
      curvature_graph(g, hv, c);
    }
    if (e.hess) {
#pragma unroll
      for (int h = 0; h < 6; ++h)
        if (h < (d3 ? 6 : 3)) ((T*)e.hess)[h * e.plane + node] = hv[h];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) ((T*)e.curv)[q * e.plane + node] = c[q];
  }
}

}  // namespace dt
