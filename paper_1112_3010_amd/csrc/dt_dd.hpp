// Host interface of the extended-precision pipelines, double-double and
// quad-double (kernels in k_dd.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dt {

// Geometry of an extended-precision plan; Mx, My, Mz are powers of two (a
// 2D plan has nz = Mz = 1, logMz = 0).  quad selects quad-double values
// (four float64 parts) instead of double-double (two).
struct DDGeom {
  int nx, ny, Mx, My, logMx, logMy;
  double hx, hy, ox, oy, tau;
  int ndim, nz, Mz, logMz;
  double hz, oz;
  int quad;
};

// Bytes of one real extended value (16 or 32) and of one complex one.
inline size_t dd_real_bytes(const DDGeom& g) { return g.quad ? 32 : 16; }
inline size_t dd_complex_bytes(const DDGeom& g) { return 2 * dd_real_bytes(g); }

// Channels of one convolution pass: channel c multiplies the image spectrum
// by spectrum tab_of[c], imaginary (the odd gradient kernels: the product
// takes the factor i) where bit c of imag is set.
constexpr int kDDMaxChannels = 12;
struct DDChannels {
  int C;
  int tab_of[kDDMaxChannels];
  unsigned imag;
};
// Sample kind of the r f kernel (the adjoint's tau channel) in the table builder.
constexpr int kDDKindRF = 100;

// Plan time: twiddles of every axis (twz unused in 2D), then for each table
// t < n_tabs (0: f, 1 + a: the gradient kernel of axis a, then the Hessian
// kernels xx, xy, [xz,] yy, [yz,] zz; table rf_tab, if >= 0, the r f kernel)
// the samples into G (scratch, Mz x My x Mx complex) and their transform;
// tabs receives the scaled real (f, Hessian, r f) or imaginary (gradient)
// spectra, Mz x My x Mx each.
hipError_t dd_build_tables(void* twx, void* twy, void* twz, void* tabs, int n_tabs, int rf_tab, void* G,
                           const DDGeom& g, hipStream_t st);
// Multiplicities into cnt (cleared by the caller) and sum m^2 into *msq
// (left at 0 by dd_launch_finalize, which consumes it).
hipError_t dd_launch_splat(const float* Y, int64_t K, double* cnt, double* msq, uint32_t* err, const DDGeom& g,
                           hipStream_t st);
hipError_t dd_launch_finalize(double* msq, double* scal, const DDGeom& g, double c_theta, double unit, double l1,
                              hipStream_t st);
// Forward row transforms of the image rows (ny x nx, or nz x ny x nx) into G.
hipError_t dd_launch_row_fwd(const double* cnt, void* G, const void* twx, const DDGeom& g, hipStream_t st);
// The convolution of the real image img with each channel's kernel up to the
// last (x) inverse transform, in two steps: the forward row transforms into
// G, then the column passes, after which Gc holds C x (nz ny) x Mx row
// spectra.  2D: the fused y pass into Gc.  3D: forward y into Gc, the fused
// z pass into G (C x nz x My x Mx), inverse y into Gc.
hipError_t dd_convolve_rows(const double* img, void* G, const void* twx, const DDGeom& g, hipStream_t st);
hipError_t dd_convolve_columns(void* G, void* Gc, const void* tabs, const DDChannels& ch, const void* twy,
                               const void* twz, const DDGeom& g, hipStream_t st);
// Inverse row transforms of the C channels and the epilogue: S (ny x nx),
// with the gradient channels (C >= 1 + ndim) grad (ndim x ny x nx), with the
// Hessian channels (C = 1 + ndim + ndim (ndim + 1) / 2) hess (xx, xy, [xz,]
// yy, [yz,] zz, each ny x nx) and curv (mean, Gaussian, k1, k2, each
// ny x nx; needs the Hessian channels); any of them may be null.
hipError_t dd_launch_row_inv_epi(const void* Gc, int C, const void* twx, double* S, double* grad, double* hess,
                                 double* curv, const double* scal, const DDGeom& g, hipStream_t st);

// Inverse row transforms of C channels into plain float64 fields
// (C x nodes), for the adjoint.
hipError_t dd_launch_row_inv_plain(const void* Gc, int C, const void* twx, double* out, const DDGeom& g,
                                   hipStream_t st);
// The adjoint at the sources from the fields (ndim gradient channels, then
// r f): dY (K x ndim float32) and per-block sums of the r f term in
// partials (at most max_blocks blocks; the count goes to *n_blocks).
hipError_t dd_launch_gather(const float* Y, int64_t K, const double* fields, const double* scal, float* dY,
                            double* partials, int max_blocks, int* n_blocks, const DDGeom& g, hipStream_t st);

}  // namespace dt
