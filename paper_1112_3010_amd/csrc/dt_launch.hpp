// Host-callable launchers for the HIP kernels (one translation unit per kernel
// family).  All launches are asynchronous on the given stream.
#pragma once

#include <vector>

#include "dt_internal.hpp"

namespace dt {

struct GridGeom {
  int ndim;
  int n[3];
  double o[3];
  double h[3];
};

enum KernelKind { KER_F = 0, KER_U = 1, KER_H = 2, KER_W2 = 3, KER_D3 = 4, KER_RF = 5 };

struct TabKernel {
  int kind;
  int i, j;       // axes for U/H/W2/D3
  double tau;
  double coef;    // constant factor for W2/D3 (sign and 1/(2 pi) or 1/(4 pi))
};

struct TabGeom {
  int ndim;
  int M[3];       // padded lengths (1 for an absent axis)
  int H[3];       // folded lengths M/2 + 1 (1 for an absent axis)
  double h[3];
  int cut[3];     // > 0: the kernel is 0 where some |d_a| > cut[a] cells (truncation box)
};

// Host: exp(-2 pi i m / M) for m < M as interleaved (re, im) float64.
void make_twiddles(int M, std::vector<double>& out);

template <typename T> void launch_fill_zero(T* p, int64_t n, hipStream_t st);
// Splats: inv_cval = 1 / cval (a power of two); msq (nullable) accumulates
// the sum of squared multiplicities of the count image.
template <typename T> void launch_splat_points(const float* Y, int64_t K, const GridGeom& g, T* cnt, T cval,
                                               double inv_cval, double* msq, uint32_t* err, hipStream_t st);
template <typename T> void launch_splat_polygon(const float* P, int64_t K, const GridGeom& g, T* cnt, T cval,
                                                double inv_cval, double* msq, T* g1, T* g2, double w1, double w2,
                                                uint32_t* err, hipStream_t st);
template <typename T> void launch_splat_mesh(const float* V, int64_t nv, const int32_t* F, int64_t nf,
                                             const GridGeom& g, T* cnt, T cval, double inv_cval, double* msq, T* gp0,
                                             T* gp1, T* gp2, double w0, double w1, double w2, uint32_t* err,
                                             hipStream_t st);
void launch_finalize_theta_msq(double* msq, double coef, double tau, double* scal, hipStream_t st);

int launch_tab_sample(const TabKernel& kd, const TabGeom& tg, double* out, double* partials, hipStream_t st);
void launch_tab_axis(const TabGeom& tg, int axis, int odd, const void* trig, const double* in, double* out,
                     hipStream_t st);
template <typename T> void launch_tab_store(const TabGeom& tg, const double* in, double scale, T* out, int nb,
                                            int tiles, hipStream_t st);

// FFT passes (return false if the length is not supported).
template <typename T> bool launch_row_r2c(const T* in, void* out, const RowParams& p, int N, hipStream_t st);
template <typename T> bool launch_col_c2c(const void* in, void* out, const ColParams& p, int N, int dir,
                                          int tiles, int outer, int chans, hipStream_t st);
template <typename T> bool launch_col_fused(const void* in, void* out, const ColParams& p, const FusedSpec& fs,
                                            int N, int tiles, int outer, hipStream_t st);
template <typename T> bool launch_row_c2r_epi(const void* in, const RowParams& p, const EpiParams& e, int N,
                                              hipStream_t st);

// Backward helpers.
template <typename T> int launch_prep_w(const T* S, const T* G, int64_t n, const double* scal, double tau,
                                        T* w, double* partials, hipStream_t st);
struct GatherParams {
  GridGeom g;
  const float* Y;
  int64_t K;
  const void* spec;     // [c][rows][kx] half-spectrum rows after all column passes
  int64_t ch_stride;    // complex elements between channels
  int pitch;            // complex elements between rows
  int inner;            // M_x/2 + 1
  int Mx;
  const void* tw;       // exp(-2 pi i m / M_x)
  int nu;               // number of gradient channels (= ndim)
  int has_rf;           // channel nu holds (r f) * w
  double ch_scale[4];   // 2^e of each channel's kernel table (undoes its scale)
  const double* scal;   // device validity scalars; [3] is the power of two applied to w
  float* dY;            // K x ndim
  double* partials;     // per-block sums of the r f channel
};
template <typename T> int launch_gather(const GatherParams& p, hipStream_t st);
void launch_finalize_dtau(const double* gs_partials, int n_gs, const double* rf_partials, int n_rf,
                          double rf_scale, double tau, double* scal, double* user_out, hipStream_t st);

}  // namespace dt
