// Host interface of the double-double pipeline (kernels in k_dd.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dt {

// Geometry of a double-double plan; Mx, My, Mz are powers of two (a 2D
// plan has nz = Mz = 1, logMz = 0).
struct DDGeom {
  int nx, ny, Mx, My, logMx, logMy;
  double hx, hy, ox, oy, tau;
  int ndim, nz, Mz, logMz;
  double hz, oz;
};

// Bytes of one complex double-double value and one real one.
constexpr size_t kDDComplexBytes = 32, kDDRealBytes = 16;

// Plan time: twiddles of every axis (twz unused in 2D), then for each table
// t < n_tabs (0: f, 1 + a: the gradient kernel of axis a, then the Hessian
// kernels xx, xy, [xz,] yy, [yz,] zz) the samples into G
// (scratch, Mz x My x Mx complex) and their transform; tabs receives the
// scaled real (f, Hessian) or imaginary (gradient) spectra, Mz x My x Mx
// each.
hipError_t dd_build_tables(void* twx, void* twy, void* twz, void* tabs, int n_tabs, void* G, const DDGeom& g,
                           hipStream_t st);
// Multiplicities into cnt (cleared by the caller) and sum m^2 into *msq
// (left at 0 by dd_launch_finalize, which consumes it).
hipError_t dd_launch_splat(const float* Y, int64_t K, double* cnt, double* msq, uint32_t* err, const DDGeom& g,
                           hipStream_t st);
hipError_t dd_launch_finalize(double* msq, double* scal, const DDGeom& g, double c_theta, double unit, double l1,
                              hipStream_t st);
// Forward row transforms of the ny source rows into G.
hipError_t dd_launch_row_fwd(const double* cnt, void* G, const void* twx, const DDGeom& g, hipStream_t st);
// Columns of G: forward, times each of the C spectra, inverse, into Gout
// (C x ny x Mx).
hipError_t dd_launch_col_fused(const void* Gin, void* Gout, const void* tabs, int C, const void* twy, const DDGeom& g,
                               hipStream_t st);
// Inverse row transforms of the C channels and the epilogue: S (ny x nx),
// with the gradient channels (C >= 1 + ndim) grad (ndim x ny x nx), with the
// Hessian channels (C = 1 + ndim + ndim (ndim + 1) / 2) hess (xx, xy, [xz,]
// yy, [yz,] zz, each ny x nx) and curv (mean, Gaussian, k1, k2, each
// ny x nx; needs the Hessian channels); any of them may be null.
hipError_t dd_launch_row_inv_epi(const void* Gc, int C, const void* twx, double* S, double* grad, double* hess,
                                 double* curv, const double* scal, const DDGeom& g, hipStream_t st);

// 3D: the forward pipeline of a double-double plan with C = 1 (f), 4 (f
// and the three gradient kernels) or 10 (and the six Hessian kernels): rows
// of the nz x ny source rows into G, forward y into Gc, z columns forward /
// times each spectrum / inverse into G (C x nz x My x Mx), inverse y into Gc
// (C x nz x ny x Mx), inverse rows with the epilogue.
hipError_t dd_launch_forward_3d(const double* cnt, void* G, void* Gc, const void* tabs, int C, const void* twx,
                                const void* twy, const void* twz, double* S, double* grad, double* hess,
                                double* curv, const double* scal, const DDGeom& g, hipStream_t st);

}  // namespace dt
