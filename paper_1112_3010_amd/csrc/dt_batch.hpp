// Batched 2D path: many independent instances (own grid, spacing, origin and
// tau) in one sequence of launches.  Each launch covers every instance; its
// blocks come from a host-built list of (instance, first row or first kx,
// count) items, so instances of different sizes share the chip.
#pragma once

#include "dt_launch.hpp"
#include "fft_mixed.hpp"

namespace dt {

constexpr int kBatchChan = 3;   // f, u_x, u_y
constexpr int kMixedFamilies = 6;   // radix schedules per length (batch.cpp, mixed_plan_for)
constexpr int kDefaultFamily = 4;   // fused radices, powers of two first

// Device-resident description of one instance (set up once per plan).
struct BatchInst {
  int nx, ny;           // grid nodes
  int sx;               // M_x / 2: length of the packed complex row transform
  int My;               // padded length along y
  int pitch;            // complex elements per half-spectrum row (>= sx + 1)
  int e_f, e_u[2];      // power-of-two exponents of the f, u_x, u_y tables
  double ox, oy, hx, hy, tau;
  double theta_coef;    // c_theta * u * log2(N_pad) * ||f||_1 / sqrt(N_pad)
  int64_t img_off;      // working elements: count image [ny][nx]
  int64_t spec_off;     // complex elements: half-spectrum rows [ny][pitch]
  int64_t fused_off;    // complex elements: column-pass outputs [C][ny][pitch]
  int64_t out_off;      // output elements: S [ny][nx]; grad [2][ny][nx] at 2 * out_off
  int64_t tab_off;      // working elements: tables [3][My/2 + 1][pitch]
  int64_t tab_stride;   // elements between the three tables
  int64_t twx_off;      // complex elements: exp(-2 pi i m / M_x), m < M_x
  int64_t twy_off;      // complex elements: exp(-2 pi i m / M_y), m < M_y
  MixedPlan px;         // radix schedule of length sx (forward row transform)
  MixedPlan py;         // radix schedule of length M_y (column pass)
  MixedPlan pxi;        // radix schedule of length sx (inverse row transform)
  uint32_t m_sx, m_sx1, m_nx;   // fastdiv_magic of sx, sx + 1 and nx
};

// One block of a batched pass: rows [first, first + count) of an instance
// (row passes) or kx bins [first, first + count) (column pass).
struct BatchBlock {
  int inst, first, count;
  int magic;   // fastdiv_magic of the block's line count (count, or count * C in the final row pass)
};

struct BatchArgs {
  const BatchInst* inst;
  int n_inst;
  const BatchBlock* blocks;
  const int64_t* koff;   // n_inst + 1 source offsets into Y
  double* scal;          // per instance: [0] Theta, [1] S_max, [2] ||g||_2, [3] sum m^2
  uint32_t* err;         // sticky error word
  const void* in;
  void* out;
  const void* tw;        // twiddle tables (working complex type)
  const void* tab;       // kernel tables (working real type)
  void* S;               // packed outputs (NULL = not wanted)
  void* grad;
  int C;                 // channels after the column pass (1 = f only, 3 = f, u_x, u_y)
};

template <typename T> void launch_batch_splat(const float* Y, int64_t K_total, const BatchArgs& a, T* img,
                                              hipStream_t st);
void launch_batch_finalize(const BatchArgs& a, hipStream_t st);
// ecap: elements per thread the launch needs (<= 32); lds: dynamic LDS bytes.
template <typename T> bool launch_batch_row_r2c(const BatchArgs& a, int n_blocks, int nthr, int ecap, size_t lds,
                                                hipStream_t st);
template <typename T> bool launch_batch_col_fused(const BatchArgs& a, int n_blocks, int nthr, int ecap,
                                                  size_t lds, hipStream_t st);
template <typename T> bool launch_batch_row_c2r_epi(const BatchArgs& a, int n_blocks, int nthr, int ecap,
                                                    size_t lds, hipStream_t st);
// Raise the dynamic-LDS limit of every batched kernel to `bytes`.
template <typename T> bool batch_set_lds_limit(int bytes);

}  // namespace dt
