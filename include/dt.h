/*
 * dt.h - C ABI of libdt, an MI355X (gfx950) library for the fast convolution
 * approximation of the signed Euclidean distance function of
 * Gurumoorthy and Rangarajan, "Fast convolution based method for computing
 * the signed distance function and its derivatives" (arXiv:1112.3010).
 *
 * What the library computes (paper references in brackets):
 *   phi(X) = sum_k exp(-||X - Y_k|| / tau)       [Sec. 2.3, eq. wavefunc]
 *   S(X)   = -tau log phi(X)                      [Sec. 2.3, eq. STilde]
 * on every node X of a regular 2D or 3D grid, as a zero-padded discrete
 * convolution of the source indicator g with the kernel f = exp(-r/tau),
 * evaluated with FFTs                             [Sec. 3, Table 1];
 * the gradient and Hessian of S as ratios of further kernel convolutions
 *                                                 [Sec. 5, eqs. SxSyconv, Sxx, Syy, Sxy];
 * the sign from the discrete winding number (2D) [Sec. 4.1, eq. kappadiscretefinal]
 * or topological degree (3D)                      [Sec. 4.2, eq. mudef];
 * and the adjoint (gradients of a grid loss with respect to the sources
 * and tau), which the paper does not give; it is derived from eq. STilde.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid.   ndim = 2 or 3.  dims[] = (nx, ny[, nz]) nodes, spacing[] = h per
 *         axis, origin[] = o per axis.  Node i sits at o + (i + 1/2) h
 *         (cell centred).  Fields are C-ordered [z][y][x] (x fastest).
 * Sources. Y is a device pointer to K x ndim float32, row-major (x, y[, z])
 *         per point.  The paper places sources on grid nodes (Sec. 3); a
 *         source is assigned to node idx_d = floor((y_d - o_d) / h_d),
 *         evaluated in float64.  Coincident sources count with multiplicity.
 *         A source outside the grid, or non-finite, is skipped and raises
 *         a sticky device error (DT_E_RANGE) reported by dt_last_error().
 * Padding. Every axis is zero-padded to M_d >= 2 n_d (a power of two), so
 *         the FFT evaluates the linear (not circular) convolution; plans
 *         made by dt_create_plan_reduced pad less, with truncated kernels.
 * Precision. DT_FP32_SCALED works in float32 with power-of-two scaling of
 *         the source image and kernel spectra (exact, so only the range is
 *         affected); DT_FP64 works in float64.  Output fields have the
 *         plan's working type (float or double).  DT_FP64X2 carries the
 *         whole convolution in double-double arithmetic (pairs of float64,
 *         about 106 significand bits; u = 2^-104), the GPU counterpart of
 *         the multiple-precision FFT that Sec. 3.2 resorts to when float64
 *         fails far from the sources: S_max grows from about 25-30 tau to
 *         about 60 tau.  It is built for 2D plans and for 3D plans of at
 *         most 256 nodes per axis whose out_mask holds only DT_OUT_S,
 *         DT_OUT_GRAD, DT_OUT_HESS, DT_OUT_CURV and DT_OUT_BACKWARD
 *         (dt_distance, dt_gradient, dt_hessian, dt_backward, dt_forward
 *         with S, grad, hess and/or curv; float64 output; other requests
 *         return DT_E_UNSUPPORTED); DT_AUTO considers it for such plans
 *         after float32 and float64.  DT_FP64X4 carries it in quad-double
 *         arithmetic (four float64 parts, about 212 bits; u taken as
 *         2^-208), which doubles the band again (S_max about 130 tau),
 *         for the same outputs, 2D plans and 3D plans of at most 128 nodes
 *         per axis; DT_AUTO considers it last.  The paper's experiments
 *         use 512-bit arithmetic; quad-double is the widest format here.
 * Validity. An FFT convolution in finite precision has an absolute error
 *         floor; nodes where phi falls below the threshold
 *           Theta = c_theta * u * log2(N_pad) * ||f||_1 * ||g||_2 / sqrt(N_pad)
 *         (u = 2^-24, 2^-53, 2^-104 or 2^-208, N_pad = prod M_d, ||f||_1 = sum of the padded
 *         kernel, ||g||_2 = sqrt(sum of squared multiplicities)) report
 *         S = S_max = -tau log Theta and zero derivatives.  The paper notes
 *         the effect (Sec. 3.2) but gives no rule; this threshold is the
 *         library's contract.
 * Streams. Every compute call is enqueued on the given HIP stream (NULL =
 *         the default stream) and returns without synchronising.  Argument
 *         errors are detected on the host, return at once and enqueue
 *         nothing.  A plan is not thread-safe; distinct plans are.
 * Logging. With the environment variable DT_LOG set (not "0"), plan
 *         creation, workspace attach and dt_last_stats / dt_batch_stats print
 *         the plan's choices to stderr: padded lengths and truncation box,
 *         precision, row radices, column tiles, tables, ||f||_1, Theta and
 *         S_max for one source, the last call's Theta; for batched plans the
 *         per-instance padding, radix schedules and tiles.
 * Memory. The library never allocates device memory: the caller provides
 *         one workspace per plan (dt_plan_workspace_size) and owns all
 *         inputs and outputs.  Kernel spectra live in the workspace.  For
 *         small plans the workspace may instead be a fixed array the
 *         library holds per device (dt_plan_set_static_workspace).
 */
#ifndef DT_H
#define DT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dt_plan_s* dt_plan;

typedef enum {
  DT_OK = 0,
  DT_E_ARG = 1,          /* invalid argument (host check; nothing enqueued) */
  DT_E_RANGE = 2,        /* a source fell outside the grid or was non-finite (sticky) */
  DT_E_PRECISION = 3,    /* DT_AUTO: the requested distance is not representable */
  DT_E_WORKSPACE = 4,    /* workspace missing, too small or misaligned */
  DT_E_HIP = 5,          /* a HIP runtime call failed */
  DT_E_UNSUPPORTED = 6   /* valid request this build does not implement */
} dt_status;

typedef enum { DT_FP32_SCALED = 0, DT_FP64 = 1, DT_AUTO = 2, DT_FP64X2 = 3, DT_FP64X4 = 4 } dt_precision;

/* Kernel families a plan prepares (bit mask for dt_create_plan). */
enum {
  DT_OUT_S = 1,          /* distance S (kernel f)                         */
  DT_OUT_GRAD = 2,       /* gradient of S (kernels (X_i/r) f)             */
  DT_OUT_HESS = 4,       /* Hessian of S (kernels H_ij)                    */
  DT_OUT_SIGN = 8,       /* winding number / topological degree kernels   */
  DT_OUT_BACKWARD = 16,  /* adjoint: gradient kernels and r f for d/dtau  */
  DT_OUT_CURV = 32       /* curvatures: the gradient and Hessian kernels   */
};

/* Closed boundary for the sign (and, optionally, the sources). */
typedef struct {
  int kind;              /* DT_SHAPE_POLYGON (2D) or DT_SHAPE_MESH (3D) */
  /* polygon: ordered closed polyline, point k+1 follows k, K+1 wraps to 1.
   * Counter-clockwise order gives mu ~ +1 inside. Device, K x 2 float32. */
  const float* points;
  int64_t n_points;
  /* mesh: closed, consistently outward-wound triangle mesh.
   * vertices: device nv x 3 float32; faces: device nf x 3 int32. */
  const float* vertices;
  int64_t n_vertices;
  const int32_t* faces;
  int64_t n_faces;
} dt_shape;
enum { DT_SHAPE_POLYGON = 1, DT_SHAPE_MESH = 2 };

/* Output buffers for dt_forward (device pointers; NULL = not wanted).
 * S: N values; grad: ndim x N (channel first); hess: ndim(ndim+1)/2 x N in
 * the order xx, xy, [xz,] yy, [yz,] zz; label: N int8 (+1 inside, -1
 * outside); mu: N values.  N = prod dims.  Value type = plan type.
 * curv (needs DT_OUT_CURV or DT_OUT_HESS): 4 x N, channel first: mean,
 * Gaussian and the two principal curvatures k1 >= k2 (the derived quantities
 * named at the end of Sec. 5), computed per node from grad S and the Hessian
 * of the unsigned S.  2D: of the graph surface (x, y, S), upward normal:
 * W = 1 + |grad S|^2, Gaussian = det(H) / W^2, mean = ((1 + S_y^2) S_xx
 * - 2 S_x S_y S_xy + (1 + S_x^2) S_yy) / (2 W^1.5).  3D: of the level surface
 * of S through the node, normal grad S / |grad S|: mean = (|g|^2 tr H
 * - g^T H g) / (2 |g|^3), Gaussian = g^T adj(H) g / |g|^4, and 0 for all four
 * where |grad S| < 1e-3.  k1,2 = mean +/- sqrt(max(mean^2 - Gaussian, 0)).
 * Nodes outside the valid band (zero derivatives) get 0. */
typedef struct {
  void* S;
  void* grad;
  void* hess;
  int8_t* label;
  void* mu;
  int signed_outputs;    /* nonzero: S and grad are multiplied by the label */
  void* curv;
} dt_outputs;

typedef struct {
  int ndim;
  int64_t dims[3];
  int64_t padded[3];     /* M_d */
  double spacing[3];
  double origin[3];
  double tau;
  int precision;         /* DT_FP32_SCALED, DT_FP64, DT_FP64X2 or DT_FP64X4 after DT_AUTO resolves */
  unsigned out_mask;
  double c_theta;
  double kernel_l1;      /* ||f||_1 over the padded grid (after set_workspace) */
  double unit_roundoff;
  size_t workspace_bytes;
  int n_tables;
  int64_t k_max;         /* 0: full padding; else the source limit of a reduced plan */
  int cut[3];            /* kernel truncation box in cells per axis (0: none) */
} dt_plan_info_t;

typedef struct {
  double g_l2;           /* sqrt(sum of squared multiplicities) of the last call */
  double theta;          /* validity threshold of the last call */
  double s_max;          /* -tau log theta */
  double dL_dtau;        /* last backward's d/dtau (also written to the user pointer) */
  uint32_t error_bits;   /* sticky device error bits (1 = range, 2 = non-finite) */
} dt_call_stats;

/* Create a plan.  dims/spacing/origin have ndim entries (x first); tau > 0
 * is fixed for the plan's lifetime (its kernel spectra are built for it; a
 * different tau needs a new plan).
 * out_mask selects the kernel families to prepare.  trunc_dist and k_hint
 * only matter for DT_AUTO: the plan uses float32 if a node at distance
 * trunc_dist from an isolated source stays valid for k_hint distinct
 * sources, else float64 if that holds in float64, else (plans of S, grad S,
 * the Hessian and curvatures; 3D up to 256 nodes per axis) double-double if
 * it holds there, else (3D up to 128 nodes per axis) quad-double if it holds
 * there, else DT_E_PRECISION.
 * c_theta <= 0 selects the default safety factor 256. Host only. */
dt_status dt_create_plan(dt_plan* out, int ndim, const int64_t* dims, const double* spacing,
                         const double* origin, double tau, int precision, unsigned out_mask,
                         double trunc_dist, int64_t k_hint, double c_theta);

/* A plan for calls that bring at most k_max sources (k_max >= 1), on a
 * smaller padded grid (the convolution of Sec. 3 with kernels truncated where
 * they fall below the rounding floor).  A call with K sources in the grid
 * has ||g||_2 >= sqrt(K) (integer multiplicities), so its validity threshold
 * is at least sqrt(K) Theta_low, Theta_low that of one source on the full
 * padding.  A source farther than d_cut = tau (ln(c_theta sqrt(k_max))
 * - ln Theta_low) from a node adds at most e^(-d_cut/tau) to phi there, so
 * the K sources together lose at most sqrt(K) Theta_low / c_theta <=
 * Theta / c_theta: results change only below the validity threshold (the
 * same bound as the rounding model).  The kernels are truncated to the box
 * |d_a| <= c_a = ceil(d_cut / h_a) cells, and axis a is padded to M_a, the
 * smallest length >= max(64, n_a + c_a) among the powers of two, 288 and
 * 392;
 * that keeps a truncated kernel from wrapping onto a node.  Where M_a is not below the full padding the axis
 * keeps it, untruncated (dt_plan_info reports M_a and c_a, 0 for such an
 * axis).  Precision
 * DT_FP32_SCALED or DT_FP64 (else DT_E_ARG); out_mask without DT_OUT_SIGN,
 * whose kernels do not decay (else DT_E_UNSUPPORTED).  Compute calls with
 * more than k_max sources (points, polygon points or mesh faces) return
 * DT_E_ARG.  Otherwise as dt_create_plan. Host only. */
dt_status dt_create_plan_reduced(dt_plan* out, int ndim, const int64_t* dims, const double* spacing,
                                 const double* origin, double tau, int precision, unsigned out_mask,
                                 int64_t k_max, double c_theta);

/* Bytes of device workspace the plan needs (256-byte aligned pointer). */
dt_status dt_plan_workspace_size(dt_plan plan, size_t* bytes);

/* Attach the workspace and build the kernel spectra on `stream` (this call
 * synchronises the stream once: plan set-up is not a hot path). */
dt_status dt_plan_set_workspace(dt_plan plan, void* dev_ptr, size_t bytes, void* stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * attach as dt_plan_set_workspace, with the workspace taken from a fixed
 * array of DT_STATIC_WORKSPACE_BYTES that the library holds on each device
 * it runs on until the process ends.  Calls no allocator.  The array is that
 * of the current device.  Plans whose workspace is larger (about 2D up to
 * 1024^2 in float32, 3D up to 64^3) get DT_E_WORKSPACE and keep their
 * previous workspace, if any.  One plan per device holds the array: the
 * last plan attached takes it over (after waiting for the device), and the
 * compute, dt_last_error and dt_last_stats calls of an earlier holder return
 * DT_E_WORKSPACE until it is attached again.  The array keeps the last
 * call's contents; each call clears what it needs.  Calls of its holder that
 * overlap in time (several streams) race, as for any one workspace.
 * Synchronises the stream (and, on take-over, the device) once. */
#define DT_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
dt_status dt_plan_set_static_workspace(dt_plan plan, void* stream);

dt_status dt_plan_info(dt_plan plan, dt_plan_info_t* info);
dt_status dt_destroy_plan(dt_plan plan);

/* Sources for the compute calls below: Y holds K points (x first, float32,
 * device memory, K x ndim row-major), K >= 1.  An empty set has no distance
 * field (phi = 0 on every node), so K < 1 or a NULL Y is refused with
 * DT_E_ARG on the host before anything is enqueued (dt_forward alone also
 * accepts Y = NULL with K = 0 when a shape supplies the sources). */

/* Distance S only (needs DT_OUT_S). */
dt_status dt_distance(dt_plan plan, const float* Y, int64_t K, void* S, void* stream);
/* S (optional, may be NULL) and grad S (needs DT_OUT_GRAD). */
dt_status dt_gradient(dt_plan plan, const float* Y, int64_t K, void* S_or_null, void* grad, void* stream);
/* Hessian of S (needs DT_OUT_HESS). */
dt_status dt_hessian(dt_plan plan, const float* Y, int64_t K, void* hess, void* stream);
/* Sign labels (and mu if non-NULL) of the closed shape (needs DT_OUT_SIGN). */
dt_status dt_sign(dt_plan plan, const dt_shape* shape, int8_t* label, void* mu_or_null, void* stream);
/* Any subset of outputs in one pipeline.  Sources: Y (K points) if Y is
 * non-NULL, else the shape's points (polygon) or triangle incenters (mesh).
 * The sign needs a shape.
 * dt_distance, dt_gradient, dt_hessian, dt_sign, dt_forward and dt_backward
 * only enqueue kernels on the given stream: no device allocation, no host
 * synchronisation and no memset nodes, so a caller may capture them into a
 * HIP graph (with plan timing off) and replay it with new contents of the
 * captured buffers (same K, same pointers). */
dt_status dt_forward(dt_plan plan, const float* Y, int64_t K, const dt_shape* shape_or_null,
                     const dt_outputs* out, void* stream);
/* Adjoint of dt_distance (needs DT_OUT_BACKWARD).  S: the forward's output
 * for the same Y; dL_dS: upstream gradient (plan type, N values).  Writes
 * dL/dY (device K x ndim float32) and, if non-NULL, dL/dtau (device
 * double).  Nodes with S >= S_max are treated as truncated (zero weight).
 * The tau derivative holds the kernel spectra and Theta fixed. */
dt_status dt_backward(dt_plan plan, const float* Y, int64_t K, const void* S, const void* dL_dS,
                      float* dL_dY, double* dL_dtau_or_null, void* stream);

/* Synchronise the plan's last stream; return DT_E_RANGE if a source of any
 * call since the previous dt_last_error was skipped, and clear the flag. */
dt_status dt_last_error(dt_plan plan);
/* Synchronise and report the per-call scalars of the last call. */
dt_status dt_last_stats(dt_plan plan, dt_call_stats* stats);

/* Optional per-pass timing (for profiling; off by default).  When enabled,
 * every kernel launch of a call is bracketed by HIP events recorded on the
 * call's stream; dt_plan_timings synchronises and reports, per pass name,
 * the number of launches and their summed duration since the last reset. */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} dt_pass_timing;
dt_status dt_plan_set_timing(dt_plan plan, int enable);
dt_status dt_plan_timings(dt_plan plan, dt_pass_timing* out, int max_entries, int* n_entries);
dt_status dt_plan_reset_timings(dt_plan plan);

/* ------------------------------------------------------------------------
 * Batched 2D distance fields (many independent instances per call)
 *
 * Each instance is its own 2D problem (dims, spacing, origin, tau) with its
 * own sources; S and grad S are those of eqs. STilde and SxSyconv per
 * instance, exactly as dt_gradient would give them except for the padding:
 * every axis is padded to M = 2 s with s the smallest 2^a 3^b 5^c 7^d >= n,
 * which still gives the linear convolution (Table 1 with M >= 2n - 1).  The
 * validity threshold uses each instance's own N_pad, ||f||_1 and ||g||_2.
 * One call launches each pass once for all instances (the blocks of a pass
 * are a list of (instance, rows or kx bins) items) so that small instances
 * share the chip; the launch sequence can be captured once into a HIP graph
 * and replayed.
 *
 * Sources: Y packs every instance's points (float32, x then y), instance i
 *   owning rows [K_offsets[i], K_offsets[i+1]) (K_offsets: host array of
 *   n_inst + 1 nondecreasing values, K_offsets[0] = 0).  An instance with no
 *   sources gets S = +inf and zero gradient.  Out-of-grid or non-finite
 *   sources are skipped and set the sticky error (dt_batch_last_error).
 * Outputs: S packs the instances' [ny][nx] fields back to back, instance i
 *   at node_offset(i) = sum_{j<i} nx_j ny_j; grad packs [2][ny][nx] per
 *   instance at 2 node_offset(i).  Both have the plan's working type.
 * Memory: the caller provides the workspace (dt_batch_workspace_size) and
 *   all inputs and outputs; the library allocates no device memory.  With
 *   graph replay enabled, one non-blocking stream (default priority) and
 *   the graph itself are created on the first call and kept by the plan.
 * ------------------------------------------------------------------------ */
typedef struct dt_batch_plan_s* dt_batch_plan;

typedef struct {
  int64_t dims[2];     /* nx, ny (2 .. 1024) */
  double spacing[2];   /* hx, hy > 0 */
  double origin[2];
  double tau;          /* > 0, physical units */
  /* 0: linear-convolution padding M_a = 2 s_a, s_a the smallest 7-smooth
   * number >= n_a.  > 0: reduced padding for calls with at most k_max sources
   * in this instance.  The kernels are truncated to the box |d_a| <= c_a
   * cells, c_a = ceil(d_cut / h_a) with d_cut = tau (ln(c_theta
   * sqrt(k_max)) - ln Theta_low), Theta_low the validity threshold for one
   * source on the full padding (a call with K sources has ||g||_2 >=
   * sqrt(K), so its Theta is at least sqrt(K) Theta_low).  The padded length
   * is M_a = 2 s'_a, s'_a the smallest 7-smooth number >= (n_a + c_a) / 2,
   * and at most the full one.  The K sources a truncated kernel drops add at
   * most K e^(-d_cut/tau) <= sqrt(K) Theta_low / c_theta <= Theta / c_theta
   * to phi, so results change only below the validity threshold.  A call
   * with more sources in the instance returns DT_E_ARG. */
  int64_t k_max;
} dt_instance_desc;

typedef struct {
  int64_t padded[2];     /* M_x, M_y */
  int64_t node_offset;   /* offset of the instance in the packed S */
  int64_t total_nodes;   /* length of the packed S */
  int precision;
  double kernel_l1;      /* ||f||_1 over the instance's padded grid */
} dt_batch_instance_info_t;

/* Launch shape of the batched passes: column tile width (kx bins per block
 * for the instances with the longest columns; an instance with shorter
 * columns takes proportionally more bins, up to 64) and threads per block of
 * the column pass and of the two row passes. */
typedef struct {
  int col_nb;
  int col_threads;   /* 64 .. 1024 */
  int row_threads;   /* 64 .. 512 */
} dt_batch_tiles;

/* precision: DT_FP32_SCALED or DT_FP64; out_mask: DT_OUT_S and/or
 * DT_OUT_GRAD; c_theta <= 0 selects 256.  DT_E_UNSUPPORTED for n > 1024. */
dt_status dt_create_batch_plan(dt_batch_plan* out, int n_inst, const dt_instance_desc* inst, int precision,
                               unsigned out_mask, double c_theta);
dt_status dt_batch_workspace_size(dt_batch_plan plan, size_t* bytes);
/* Attaches the workspace (>= the size above, 256-byte aligned), builds the
 * kernel spectra of every distinct geometry and the default tiles;
 * synchronises the stream. */
dt_status dt_batch_set_workspace(dt_batch_plan plan, void* dev_ptr, size_t bytes, void* stream);
dt_status dt_batch_instance_info(dt_batch_plan plan, int i, dt_batch_instance_info_t* info);
/* Tiles: DT_E_UNSUPPORTED (previous tiles kept) when a pass would exceed
 * 32 elements per thread or the device's LDS per block. */
dt_status dt_batch_set_tiles(dt_batch_plan plan, const dt_batch_tiles* tiles);
dt_status dt_batch_get_tiles(dt_batch_plan plan, dt_batch_tiles* tiles);
/* enable != 0: calls capture their launch sequence into a HIP graph the
 * first time and replay it while Y, S, grad and K_offsets are unchanged. */
dt_status dt_batch_set_graph(dt_batch_plan plan, int enable);
/* S and/or grad (device, packed as above) as the plan's out_mask requests.
 * When K_offsets differ from the previous call they are copied to the
 * workspace first (a synchronous host-to-device copy). */
dt_status dt_forward_batched(dt_batch_plan plan, const float* Y, const int64_t* K_offsets, void* S, void* grad,
                             void* stream);
/* Radix schedule of the batched transforms: fams[3 i + k] is the schedule
 * of pass k of instance i (k = 0: forward row transform, 1: column pass,
 * 2: inverse row transform with the epilogue), one of six radix schedules
 * of the 7-smooth length: 0 radix 8 while possible, then one 4 or 2, then
 * 7, 5, 3; 1 the odd radices first, then as 0; 2 radix 4 while possible,
 * then one 2, then 7, 5, 3; 3 the one 4 or 2 first, then radix 8, then 7, 5,
 * 3; 4 fused radices up to 16 (two prime-power stages per register DFT):
 * radix 16 while possible, a leftover 2 joined to the smallest odd factor
 * (6, 10, 14) and a leftover 4 to a factor 3 (12), else alone, then the odd
 * factors paired largest with smallest where the product is at most 15 (9,
 * 15); 5 the same with the odd radices first.
 * All give the same transform up to rounding.  Default 4 everywhere;
 * dt_batch_autotune chooses them per (pass, length).  fams holds 3 n_inst
 * ints; values outside 0..5 give DT_E_ARG and change nothing. */
dt_status dt_batch_set_schedule(dt_batch_plan plan, const int* fams);
dt_status dt_batch_get_schedule(dt_batch_plan plan, int* fams);
/* Times every feasible tile choice (reps calls each, eager, on `stream`)
 * and keeps the fastest; then, per pass and per padded length, times that
 * pass alone over the instances of that length under each distinct radix
 * schedule and keeps the fastest (read it with dt_batch_get_schedule); then
 * times the tile choices once more under those schedules.  The final tiles
 * are returned in *best (may be NULL).  Overwrites S and grad.
 * Synchronises the stream. */
dt_status dt_batch_autotune(dt_batch_plan plan, const float* Y, const int64_t* K_offsets, void* S, void* grad,
                            int reps, void* stream, dt_batch_tiles* best);
/* Synchronises the plan's stream; returns and clears the sticky error. */
dt_status dt_batch_last_error(dt_batch_plan plan);
/* Validity scalars (theta, s_max, g_l2) of instance i from the last call;
 * synchronises the plan's stream. */
dt_status dt_batch_stats(dt_batch_plan plan, int i, dt_call_stats* stats);
dt_status dt_destroy_batch_plan(dt_batch_plan plan);

const char* dt_status_str(dt_status status);

#ifdef __cplusplus
}
#endif

#endif /* DT_H */
