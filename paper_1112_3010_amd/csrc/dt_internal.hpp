// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dt {

constexpr int kMaxTables = 16;
constexpr int kMaxIn = 4;     // input channels of one fused group
constexpr int kMaxOut = 12;   // output channels of one fused group
// s_waitcnt immediate with vmcnt = 0 and expcnt, lgkmcnt at their maxima (no wait on those)
constexpr int kWaitVmcnt0 = 0x0F70;

// Sticky device error bits (first word of the workspace scalars).
constexpr uint32_t kErrRange = 1u;
constexpr uint32_t kErrNonFinite = 2u;

// Real-valued symmetric kernel spectrum table: the DFT of a kernel with a
// definite parity on every axis is (-i)^(number of odd axes) times a real
// table that is even/odd along each axis.  Stored for k_a in [0, M_a/2]
// (kx fastest, pitch = padded half-spectrum pitch).
struct TabRef {
  const void* ptr;   // float or double, layout [kzf][kyf][kx]
  int phase;         // number of odd axes mod 4: spectrum = (-i)^phase * T
  int odd_line;      // parity along the transform axis of the fused pass
  int odd_outer;     // parity along the outer axis (3D: y); 0 in 2D
};

// One fused multiply group of the last forward column pass.
// mode 0: one input channel, n_out outputs, output c uses table tab[c].
// mode 1: n_in inputs, one output, sum over inputs of tab[i] * input i.
struct FusedGroup {
  int mode;
  int n_in;
  int in_ch[kMaxIn];
  int n_out;
  int out_ch[kMaxOut];
  int tab[kMaxOut];
};

// One block column of the fused pass computes group `group`'s outputs
// [c0, c1) (mode 0) or its single output (mode 1).
struct FusedItem {
  int group, c0, c1;
};

struct FusedSpec {
  int n_groups;
  FusedGroup g[2];
  int n_items;               // grid.z of the fused pass
  FusedItem items[kMaxOut + 1];
  TabRef tabs[kMaxTables];
  // Table element (folded outer k, kx tile, folded line k, bin in tile) sits at
  // of * tab_outer_stride + tile * tab_tile_stride + lf * tab_line_stride + b:
  // each block's slice is one contiguous run.
  int64_t tab_line_stride;
  int64_t tab_outer_stride;
  int64_t tab_tile_stride;
};

// Strided column pass over tiles of consecutive kx bins.
struct ColParams {
  int64_t in_line, in_outer, in_ch;      // complex-element strides
  int64_t out_line, out_outer, out_ch;
  int inner;        // number of valid kx bins (M_x/2 + 1)
  int n_in;         // rows 0..n_in-1 of the input are present, the rest are zero
  int n_out;        // rows 0..n_out-1 of the output are stored
  int outer_len;    // length of the outer axis (for table folding)
  const void* tw;   // twiddle table exp(-2 pi i m / L), L = N * tw_stride
  int tw_stride;
};

// Row (x) passes.
struct RowParams {
  int64_t n_lines;  // rows to transform
  int nx;           // real samples per row
  int pitch;        // complex pitch of half-spectrum rows
  int inner;        // M_x/2 + 1
  const void* tw;   // exp(-2 pi i m / M_x), m < M_x
};

// Epilogue channel map and scalars (final row pass).
struct EpiParams {
  int C;                    // channels per row in the input buffer
  int64_t ch_stride;        // complex elements between channels
  int ch_phi, ch_u[3], ch_h[6], ch_mu;   // -1 when absent
  double scale_phi;         // 2^(e_g + e_f): undoes the power-of-two scales
  double scale_u[3];        // 2^(e_u - e_f)
  double scale_h[6];        // 2^(e_h - e_f)
  double scale_mu;          // 2^(e_w + e_mu)
  double tau;
  const double* theta;      // device: [0] theta, [1] s_max
  int ndim;
  int64_t n_rows;           // rows of the output grid (ny * nz)
  int nx;
  int64_t plane;            // nodes per output field (N)
  void* S;                  // outputs (plan type), NULL = not wanted
  void* grad;
  void* hess;
  int8_t* label;
  void* mu;
  int signed_out;
  void* curv;               // 4 x N: mean, Gaussian, k1, k2 (NULL = not wanted)
};

}  // namespace dt
