// Host interface of the double-double pipeline (kernels in k_dd.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dt {

// Geometry of a 2D double-double plan; Mx, My are powers of two.
struct DDGeom {
  int nx, ny, Mx, My, logMx, logMy;
  double hx, hy, ox, oy, tau;
};

// Bytes of one complex double-double value and one real one.
constexpr size_t kDDComplexBytes = 32, kDDRealBytes = 16;

// Plan time: twiddles of both axes, then f sampled into G and transformed;
// tab receives the scaled real spectrum.  G is scratch (My x Mx complex).
hipError_t dd_build_tables(void* twx, void* twy, void* tab, void* G, const DDGeom& g, hipStream_t st);
// Multiplicities into cnt (cleared by the caller) and sum m^2 into *msq
// (left at 0 by dd_launch_finalize, which consumes it).
hipError_t dd_launch_splat(const float* Y, int64_t K, double* cnt, double* msq, uint32_t* err, const DDGeom& g,
                           hipStream_t st);
hipError_t dd_launch_finalize(double* msq, double* scal, const DDGeom& g, double c_theta, double unit, double l1,
                              hipStream_t st);
hipError_t dd_launch_row_fwd(const double* cnt, void* G, const void* twx, const DDGeom& g, hipStream_t st);
hipError_t dd_launch_col_fused(void* G, const void* tab, const void* twy, const DDGeom& g, hipStream_t st);
hipError_t dd_launch_row_inv_epi(const void* G, const void* twx, double* S, const double* scal, const DDGeom& g,
                                 hipStream_t st);

}  // namespace dt
