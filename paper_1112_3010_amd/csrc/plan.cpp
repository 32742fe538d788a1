// Host side of libdt: plan creation and validation, workspace layout,
// plan-time kernel spectra, and the launch sequences of the C ABI calls.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dt.h"
#include "dt_dd.hpp"
#include "dt_launch.hpp"
#include "dt_log.hpp"
#include "dt_static.hpp"

using namespace dt;

namespace dt {
int col_tile_width(int N, bool fp64, bool fused);
int row_points_per_thread(int N);
int row_radices(int N, int* radix, int cap);
}

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kPartials = 4096;     // per-block partial sums (each region)
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Reduced padded length: the smallest length >= need (at least 64) that the
// passes have engines for: powers of two, 288 = 2 * 12^2 and 392 = 2 * 14^2
// (pair-split register engines for the columns, 12 x 12 and 14 x 14
// Stockham for the rows).
int64_t reduced_length(int64_t need) {
  int64_t m = 64;
  while (m < need) m *= 2;
  for (const int64_t l : {288, 392})
    if (need <= l && l < m) m = l;
  return m;
}

int64_t pad_length(int64_t n) {
  int64_t m = 64;
  while (m < 2 * n) m *= 2;
  return m;
}

int ceil_log2(double v) {
  if (!(v > 0)) return 0;
  int e;
  const double f = std::frexp(v, &e);  // v = f 2^e, f in [0.5, 1)
  return f == 0.5 ? e - 1 : e;
}

struct Table {
  TabKernel kd;
  int par[3];   // odd (1) / even (0) per axis x, y, z
  int phase;
  double l1;
  int e;        // table scaled by 2^-e / N_pad
  size_t off;
};

}  // namespace

struct dt_plan_s {
  int ndim = 0;
  int64_t n[3] = {1, 1, 1};
  int64_t M[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  double o[3] = {0, 0, 0};
  double tau = 0;
  int prec = DT_FP32_SCALED;
  unsigned mask = 0;
  double c_theta = 256.0;
  bool fp64 = false;
  size_t w = 4;          // bytes per real
  int Mh = 0, MhP = 0;   // half spectrum length and pitch along x
  int NB = 16;           // column tile width (the half-spectrum pitch is a multiple of it)
  int NBf = 16;          // tile width of the fused pass (kernel tables are laid out for it)
  std::vector<Table> tabs;
  int t_f = -1, t_u[3] = {-1, -1, -1}, t_h[6] = {-1, -1, -1, -1, -1, -1}, t_sign[3] = {-1, -1, -1}, t_rf = -1;
  int e_sign_tab = 0;
  int in_max = 0, out_max = 0;
  size_t off_scal = 0, off_err = 0, off_partA = 0, off_partB = 0, off_tw[3] = {0, 0, 0}, off_tw64[3] = {0, 0, 0};
  size_t off_tabs = 0, tab_elems = 0, off_R1 = 0, off_R2 = 0, R1 = 0, R2 = 0, ws_bytes = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  double kernel_l1 = 0;
  bool ready = false;
  // reduced padding: calls bring at most k_max sources (0: full padding);
  // kernels are zero outside the box |d_a| <= cut[a] cells (0: no truncation)
  int64_t k_max = 0;
  int cut[3] = {0, 0, 0};
  // workspace = the library's fixed device array (dt_plan_set_static_workspace):
  // the device it lives on and the token that marks this plan as its holder
  int static_dev = -1;
  uint64_t static_token = 0;
  // tables built and, for the fixed array, not since taken over by another plan
  bool usable() const { return ready && (static_dev < 0 || dt::static_ws_owner(static_dev) == static_token); }
  void release_static() {
    if (static_dev >= 0) dt::static_ws_release(static_dev, static_token);
    static_dev = -1;
    static_token = 0;
  }
  // double-double and quad-double plans (S, grad S, Hessian, curvatures,
  // adjoint) use their own workspace regions; quad marks quad-double
  bool dd = false;
  bool quad = false;
  DDGeom ddg{};
  int dd_tabs = 1;       // 1: f; 1 + ndim: and the gradient kernels; + ndim (ndim + 1) / 2: and the Hessian's
  int dd_rf_tab = -1;    // table of r f (adjoint plans), else -1
  size_t off_dd_twx = 0, off_dd_twy = 0, off_dd_twz = 0, off_dd_tab = 0, off_dd_cnt = 0, off_dd_G = 0, off_dd_Gc = 0;
  // optional per-pass timing
  bool timing = false;
  struct Pending { std::string name; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<std::string, std::pair<int64_t, double>>> acc;
  hipEvent_t take_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~dt_plan_s() {
    for (auto& q : pending) {
      if (q.a) (void)hipEventDestroy(q.a);
      if (q.b) (void)hipEventDestroy(q.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }

  int64_t nodes() const { return n[0] * n[1] * n[2]; }
  int64_t rows() const { return n[1] * n[2]; }
  double npad() const { return (double)M[0] * (double)M[1] * (double)M[2]; }
  double unit() const { return std::ldexp(1.0, unit_log2()); }
  int unit_log2() const { return dd ? (quad ? -208 : -104) : fp64 ? -53 : -24; }
  double* scal() const { return (double*)(ws + off_scal); }
  double* msq() const { return scal() + 16; }   // splat accumulator of sum m^2 (cleared by the finalize)
  uint32_t* err() const { return (uint32_t*)(ws + off_err); }
  double* partA() const { return (double*)(ws + off_partA); }
  double* partB() const { return (double*)(ws + off_partB); }
  char* R1p() const { return ws + off_R1; }
  char* R2p() const { return ws + off_R2; }
  const void* tab_ptr(int t) const { return ws + off_tabs + tabs[t].off; }
  GridGeom geom() const {
    GridGeom g;
    g.ndim = ndim;
    for (int a = 0; a < 3; ++a) {
      g.n[a] = (int)n[a];
      g.o[a] = o[a];
      g.h[a] = h[a];
    }
    return g;
  }
};

namespace {

// Brackets one pass with events when timing is enabled.
struct PassTimer {
  dt_plan p;
  hipStream_t st;
  std::string name;
  hipEvent_t a = nullptr;
  PassTimer(dt_plan p_, hipStream_t st_, const char* n) : p(p_), st(st_), name(n) {
    if (p->timing) {
      a = p->take_event();
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~PassTimer() {
    if (!a) return;
    hipEvent_t b = p->take_event();
    if (!b) return;
    (void)hipEventRecord(b, st);
    p->pending.push_back({name, a, b});
  }
};

}  // namespace

// Twiddles exp(-2 pi i m / M) in float64 with octant reduction of the angle.
void dt::make_twiddles(int M, std::vector<double>& out) {
  out.resize(2 * (size_t)M);
  for (int m = 0; m < M; ++m) {
    // angle = 2 pi m / M; reduce to [0, pi/4] by symmetry for accuracy
    const int64_t e8 = (int64_t)m * 8;
    const int oct = (int)(e8 / M);
    const int64_t rem = e8 % M;  // angle within octant = (pi/4) * rem / M
    double c, s;
    auto cs = [&](int64_t num, double& cc, double& ss) {  // angle = (pi/4) num / M
      const double a = (kPi / 4.0) * (double)num / (double)M;
      cc = std::cos(a);
      ss = std::sin(a);
    };
    double ca, sa;
    switch (oct) {
      case 0: cs(rem, ca, sa); c = ca; s = sa; break;
      case 1: cs(M - rem, ca, sa); c = sa; s = ca; break;
      case 2: cs(rem, ca, sa); c = -sa; s = ca; break;
      case 3: cs(M - rem, ca, sa); c = -ca; s = sa; break;
      case 4: cs(rem, ca, sa); c = -ca; s = -sa; break;
      case 5: cs(M - rem, ca, sa); c = -sa; s = -ca; break;
      case 6: cs(rem, ca, sa); c = sa; s = -ca; break;
      default: cs(M - rem, ca, sa); c = ca; s = -sa; break;
    }
    out[2 * (size_t)m] = c;
    out[2 * (size_t)m + 1] = -s;
  }
}

namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

int add_table(dt_plan p, int kind, int i, int j, double coef) {
  Table t{};
  t.kd.kind = kind;
  t.kd.i = i;
  t.kd.j = j;
  t.kd.tau = p->tau;
  t.kd.coef = coef;
  t.par[0] = t.par[1] = t.par[2] = 0;
  switch (kind) {
    case KER_U: case KER_W2: case KER_D3: t.par[i] ^= 1; break;
    case KER_H: if (i != j) { t.par[i] ^= 1; t.par[j] ^= 1; } break;
    default: break;
  }
  t.phase = (t.par[0] + t.par[1] + t.par[2]) & 3;
  p->tabs.push_back(t);
  return (int)p->tabs.size() - 1;
}

// Host estimate of ||f||_1 over the padded grid (used by DT_AUTO only).
double host_kernel_l1(const int64_t* M, const double* h, int ndim, double tau) {
  double total = 0.0;
  const int64_t hz = ndim == 3 ? M[2] / 2 : 1;
  for (int64_t z = 0; z < hz; ++z)
    for (int64_t y = 0; y < M[1] / 2; ++y) {
      const double wzy = (z > 0 ? 2.0 : 1.0) * (y > 0 ? 2.0 : 1.0);
      const double dz = ndim == 3 ? z * h[2] : 0.0, dy = y * h[1];
      for (int64_t x = 0; x < M[0] / 2; ++x) {
        const double dx = x * h[0];
        total += wzy * (x > 0 ? 2.0 : 1.0) * std::exp(-std::sqrt(dx * dx + dy * dy + dz * dz) / tau);
      }
    }
  return total;
}

dt_status hip_status(hipError_t e) { return e == hipSuccess ? DT_OK : DT_E_HIP; }

int log2_exact(int64_t m) {
  int e = 0;
  while ((int64_t(1) << e) < m) ++e;
  return e;
}

// Workspace of an extended-precision plan: scalars and error word (same offsets
// as the other precisions, so the stats calls are shared), twiddles, the
// spectra, the multiplicities, the complex work grid and the column-pass
// outputs.
// The outputs and sizes the extended-precision pipelines serve: every output
// but the sign; 3D up to 256 nodes per axis in double-double (512^3 padded:
// about 22 GB of workspace) and 128 in quad-double.
bool xp_supported(int precision, int ndim, const int64_t* dims, unsigned out_mask) {
  if (out_mask & ~(unsigned)(DT_OUT_S | DT_OUT_GRAD | DT_OUT_HESS | DT_OUT_CURV | DT_OUT_BACKWARD)) return false;
  const int64_t cap = precision == DT_FP64X4 ? 128 : 256;
  if (ndim == 3)
    for (int a = 0; a < 3; ++a)
      if (dims[a] > cap) return false;
  return true;
}

void setup_dd(dt_plan p) {
  p->dd = true;
  const bool d3 = p->ndim == 3;
  const int nh = p->ndim == 2 ? 3 : 6;
  // tables: f, the gradient kernels (also for the adjoint), the Hessian's, then r f for the adjoint
  const int n_fwd = (p->mask & (DT_OUT_HESS | DT_OUT_CURV)) ? 1 + p->ndim + nh
                    : (p->mask & (DT_OUT_GRAD | DT_OUT_BACKWARD)) ? 1 + p->ndim : 1;
  p->dd_rf_tab = (p->mask & DT_OUT_BACKWARD) ? n_fwd : -1;
  p->dd_tabs = n_fwd + ((p->mask & DT_OUT_BACKWARD) ? 1 : 0);
  p->fp64 = true;  // outputs are float64
  p->w = 8;
  DDGeom& g = p->ddg;
  g.ndim = p->ndim;
  g.nx = (int)p->n[0];
  g.ny = (int)p->n[1];
  g.nz = d3 ? (int)p->n[2] : 1;
  g.Mx = (int)p->M[0];
  g.My = (int)p->M[1];
  g.Mz = d3 ? (int)p->M[2] : 1;
  g.logMx = log2_exact(p->M[0]);
  g.logMy = log2_exact(p->M[1]);
  g.logMz = d3 ? log2_exact(p->M[2]) : 0;
  g.hx = p->h[0];
  g.hy = p->h[1];
  g.hz = d3 ? p->h[2] : 1.0;
  g.ox = p->o[0];
  g.oy = p->o[1];
  g.oz = d3 ? p->o[2] : 0.0;
  g.tau = p->tau;
  g.quad = p->quad ? 1 : 0;
  const size_t npad = (size_t)g.Mx * g.My * g.Mz, C = (size_t)p->dd_tabs;
  const size_t cb = dd_complex_bytes(g), rb = dd_real_bytes(g);
  // 2D: G holds the row spectra, Gc the column-pass outputs.  3D: G holds
  // the table samples, the row spectra and the z-pass outputs; Gc the y-pass
  // outputs in both directions.
  const size_t Gsz = d3 ? std::max(npad, C * g.nz * g.My * g.Mx) : npad;
  const size_t Gcsz = d3 ? std::max((size_t)g.nz * g.My * g.Mx, C * g.nz * g.ny * g.Mx) : C * g.ny * g.Mx;
  size_t off = 0;
  p->off_scal = off; off = align_up(off + 64 * sizeof(double));
  p->off_err = off; off = align_up(off + sizeof(uint32_t));
  p->off_partA = off; off = align_up(off + kPartials * sizeof(double));
  p->off_partB = off; off = align_up(off + kPartials * sizeof(double));
  p->off_R1 = off;  // end of the region cleared at attach
  p->off_dd_twx = off; off = align_up(off + (size_t)g.Mx / 2 * cb);
  p->off_dd_twy = off; off = align_up(off + (size_t)g.My / 2 * cb);
  p->off_dd_twz = off; off = align_up(off + (size_t)std::max(g.Mz / 2, 1) * cb);
  p->off_dd_tab = off; off = align_up(off + C * npad * rb);
  p->off_dd_cnt = off; off = align_up(off + (size_t)g.nx * g.ny * g.nz * sizeof(double));
  p->off_dd_G = off; off = align_up(off + Gsz * cb);
  p->off_dd_Gc = off; off = align_up(off + Gcsz * cb);
  p->ws_bytes = off;
}

template <typename T> size_t complex_bytes() { return 2 * sizeof(T); }

// -- plan log (DT_LOG) --------------------------------------------------------
// "256x256x256" / "0.01 0.01" for the plan's axes
std::string axes_i(const int64_t* v, int n) {
  std::string s;
  for (int a = 0; a < n; ++a) s += (a ? "x" : "") + std::to_string((long long)v[a]);
  return s;
}
std::string axes_d(const double* v, int n) {
  std::string s;
  char b[32];
  for (int a = 0; a < n; ++a) {
    std::snprintf(b, sizeof(b), "%s%.6g", a ? " " : "", v[a]);
    s += b;
  }
  return s;
}
std::string table_name(const Table& t) {
  static const char ax[3] = {'x', 'y', 'z'};
  switch (t.kd.kind) {
    case KER_F: return "f";
    case KER_U: return std::string("u_") + ax[t.kd.i];
    case KER_H: return std::string("h_") + ax[t.kd.i] + ax[t.kd.j];
    case KER_W2: return std::string("w_") + ax[t.kd.i];
    case KER_D3: return std::string("d_") + ax[t.kd.i];
    case KER_RF: return "rf";
    default: return "?";
  }
}
// Threshold of one source of multiplicity one (||g||_2 = 1): Theta of a call
// with K distinct sources is sqrt(K) times this.
double theta_one(dt_plan p) {
  const double np = p->npad();
  return p->c_theta * p->unit() * std::log2(np) * p->kernel_l1 / std::sqrt(np);
}

void log_created(dt_plan p) {
  if (!log_enabled()) return;
  const int D = p->ndim;
  char mb[96];
  logf("plan %p created: %dD grid %s, h = %s, origin = %s, tau = %.6g (%.3g h_x), precision %s (u = 2^-%d), "
       "outputs %s, c_theta = %g",
       (void*)p, D, axes_i(p->n, D).c_str(), axes_d(p->h, D).c_str(), axes_d(p->o, D).c_str(), p->tau,
       p->tau / p->h[0], precision_name(p->prec), -p->unit_log2(), mask_names(p->mask, mb, sizeof(mb)),
       p->c_theta);
  if (p->k_max > 0) {
    int64_t cut[3] = {p->cut[0], p->cut[1], p->cut[2]};
    logf("  padded %s, reduced for at most %lld sources: kernels truncated to %s cells (0: axis untruncated)",
         axes_i(p->M, D).c_str(), (long long)p->k_max, axes_i(cut, D).c_str());
  } else {
    logf("  padded %s (full zero padding)", axes_i(p->M, D).c_str());
  }
  if (p->dd) {
    logf("  passes: %s radix-2 transforms staged in LDS (rows %lld, columns %s); %d spectra; "
         "workspace %.1f MB",
         p->quad ? "quad-double" : "double-double", (long long)p->M[0], axes_i(p->M + 1, D - 1).c_str(),
         p->dd_tabs, p->ws_bytes / 1e6);
    return;
  }
  const int Q = (int)(p->M[0] / 2);
  int rad[8];
  const int ns = row_radices(Q, rad, 8);
  std::string rs;
  for (int i = 0; i < ns && i < 8; ++i) rs += (i ? "x" : "") + std::to_string(rad[i]);
  logf("  passes: rows R2C / C2R of %lld points (%d-point complex, radices %s, %d points per thread); "
       "half spectrum %d bins (pitch %d)",
       (long long)p->M[0], Q, rs.c_str(), row_points_per_thread(Q), p->Mh, p->MhP);
  if (D == 3)
    logf("  columns: y %lld points, tiles of %d bins; fused z pass (forward, tables, inverse) %lld points, "
         "tiles of %d bins",
         (long long)p->M[1], p->NB, (long long)p->M[2], p->NBf);
  else
    logf("  columns: fused y pass (forward, tables, inverse) %lld points, tiles of %d bins", (long long)p->M[1],
         p->NBf);
  std::string names;
  for (const auto& t : p->tabs) names += (names.empty() ? "" : " ") + table_name(t);
  logf("  tables: %s (%zu of %.1f MB); channels in <= %d, out <= %d; workspace %.1f MB", names.c_str(),
       p->tabs.size(), p->tab_elems * p->w / 1e6, p->in_max, p->out_max, p->ws_bytes / 1e6);
}

void log_attached(dt_plan p) {
  if (!log_enabled()) return;
  const double th = theta_one(p);
  logf("plan %p attached: ||f||_1 = %.9g; one source: Theta = %.4g, S_max = %.3f tau", (void*)p, p->kernel_l1, th,
       -std::log(th));
  if (p->k_max > 0)
    logf("  at k_max = %lld distinct sources: Theta = %.4g, S_max = %.3f tau", (long long)p->k_max,
         th * std::sqrt((double)p->k_max), -std::log(th * std::sqrt((double)p->k_max)));
  for (const auto& t : p->tabs)
    logf("  table %-4s ||.||_1 = %.6g, stored scaled by 2^-%d / N_pad", table_name(t).c_str(), t.l1, t.e);
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan creation
// ---------------------------------------------------------------------------
static dt_status create_plan(dt_plan* out, int ndim, const int64_t* dims, const double* spacing,
                             const double* origin, double tau, int precision, unsigned out_mask, double trunc_dist,
                             int64_t k_hint, double c_theta, int64_t k_max) {
  if (!out) return DT_E_ARG;
  *out = nullptr;
  if (ndim != 2 && ndim != 3) return DT_E_ARG;
  if (!dims || !spacing || !origin) return DT_E_ARG;
  if (!finite_pos(tau)) return DT_E_ARG;
  if (precision != DT_FP32_SCALED && precision != DT_FP64 && precision != DT_AUTO && precision != DT_FP64X2 &&
      precision != DT_FP64X4)
    return DT_E_ARG;
  const unsigned known = DT_OUT_S | DT_OUT_GRAD | DT_OUT_HESS | DT_OUT_SIGN | DT_OUT_BACKWARD | DT_OUT_CURV;
  if (out_mask == 0 || (out_mask & ~known)) return DT_E_ARG;
  if (!(c_theta <= 0) && !finite_pos(c_theta)) return DT_E_ARG;
  for (int a = 0; a < ndim; ++a) {
    if (dims[a] < 2) return DT_E_ARG;
    if (!finite_pos(spacing[a]) || !std::isfinite(origin[a])) return DT_E_ARG;
    if (dims[a] > 1024) return DT_E_UNSUPPORTED;
  }
  dt_plan p = new (std::nothrow) dt_plan_s();
  if (!p) return DT_E_ARG;
  p->ndim = ndim;
  for (int a = 0; a < ndim; ++a) {
    p->n[a] = dims[a];
    p->h[a] = spacing[a];
    p->o[a] = origin[a];
    p->M[a] = pad_length(dims[a]);
  }
  p->tau = tau;
  p->mask = out_mask;
  p->c_theta = c_theta > 0 ? c_theta : 256.0;
  if (k_max > 0) {
    // A call with K <= k_max sources inside the grid has ||g||_2 >= sqrt(K)
    // (integer multiplicities), ||f||_1 >= f(0) = 1, and log2(N)/sqrt(N) falls
    // with N, so its Theta is at least sqrt(K) Theta_low, Theta_low the
    // threshold of one source on the full padding.  Sources farther than
    // d_cut = tau (ln(c_theta sqrt(k_max)) - ln Theta_low) add at most
    // K e^(-d_cut/tau) <= sqrt(K) Theta_low / c_theta <= Theta / c_theta to
    // phi, below what the contract treats as noise: the kernels are truncated
    // to |d_a| <= c_a = ceil(d_cut / h_a) cells and each axis is padded to the
    // smallest length with an engine >= n_a + c_a (so that no truncated kernel
    // value wraps onto a node), where that is below the full padding.
    // The winding-number and degree kernels do not decay: they are never truncated.
    if (out_mask & DT_OUT_SIGN) {
      delete p;
      return DT_E_UNSUPPORTED;
    }
    if (precision != DT_FP32_SCALED && precision != DT_FP64) {
      delete p;
      return DT_E_ARG;
    }
    p->k_max = k_max;
    const double u = precision == DT_FP64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
    const double np_full = p->npad();
    const double theta_low = p->c_theta * u * std::log2(np_full) / std::sqrt(np_full);
    const double d_cut = tau * (std::log(p->c_theta * std::sqrt((double)k_max)) - std::log(theta_low));
    for (int a = 0; a < ndim; ++a) {
      const double c = std::ceil(d_cut / spacing[a]);
      const int64_t ci = c < 1e9 ? (int64_t)c : (int64_t)1000000000;
      const int64_t m = reduced_length(dims[a] + ci);
      if (m < p->M[a]) {
        p->M[a] = m;
        p->cut[a] = (int)ci;
      }
    }
  }

  if (precision == DT_AUTO) {
    if (!(trunc_dist >= 0) || !std::isfinite(trunc_dist) || k_hint < 1) {
      delete p;
      return DT_E_ARG;
    }
    const double l1 = host_kernel_l1(p->M, p->h, ndim, tau);
    const double np = p->npad();
    int chosen = -1;
    // double-double and quad-double are candidates wherever they are built:
    // every output but the sign (3D up to 256, resp. 128, nodes per axis)
    const int cands[4] = {DT_FP32_SCALED, DT_FP64, DT_FP64X2, DT_FP64X4};
    const int ubits[4] = {24, 53, 104, 208};
    for (int c = 0; c < 4 && chosen < 0; ++c) {
      if (c >= 2 && !xp_supported(cands[c], ndim, dims, out_mask)) continue;
      const double u = std::ldexp(1.0, -ubits[c]);
      const double theta = p->c_theta * u * std::log2(np) * l1 * std::sqrt((double)k_hint) / std::sqrt(np);
      if (trunc_dist <= -tau * std::log(theta)) chosen = cands[c];
    }
    if (chosen < 0) {
      delete p;
      return DT_E_PRECISION;
    }
    precision = chosen;
  }
  p->prec = precision;
  if (precision == DT_FP64X2 || precision == DT_FP64X4) {
    if (!xp_supported(precision, ndim, dims, out_mask)) {
      delete p;
      return DT_E_UNSUPPORTED;
    }
    p->quad = precision == DT_FP64X4;
    setup_dd(p);
    log_created(p);
    *out = p;
    return DT_OK;
  }
  p->fp64 = precision == DT_FP64;
  p->w = p->fp64 ? 8 : 4;
  p->Mh = (int)(p->M[0] / 2 + 1);
  // the half-spectrum pitch is a multiple of every column tile width
  p->NB = 1;
  for (int a = 1; a < ndim; ++a)
    for (int fused = 0; fused < 2; ++fused) p->NB = std::max(p->NB, col_tile_width((int)p->M[a], p->fp64, fused));
  p->MhP = (p->Mh + p->NB - 1) / p->NB * p->NB;
  p->NBf = col_tile_width((int)p->M[ndim - 1], p->fp64, true);

  // kernel tables
  const int D = ndim;
  // curvatures need the gradient and Hessian kernels
  const bool hessfam = out_mask & (DT_OUT_HESS | DT_OUT_CURV);
  const bool dist = (out_mask & (DT_OUT_S | DT_OUT_GRAD)) || hessfam;
  const bool grad = (out_mask & (DT_OUT_GRAD | DT_OUT_BACKWARD)) || hessfam;
  if (dist) p->t_f = add_table(p, KER_F, 0, 0, 1.0);
  if (grad)
    for (int a = 0; a < D; ++a) p->t_u[a] = add_table(p, KER_U, a, 0, 1.0);
  if (hessfam) {
    int hcount = 0;
    for (int i = 0; i < D; ++i)
      for (int j = i; j < D; ++j) p->t_h[hcount++] = add_table(p, KER_H, i, j, 1.0);
  }
  if (out_mask & DT_OUT_SIGN) {
    if (D == 2) {
      p->t_sign[0] = add_table(p, KER_W2, 1, 0, 1.0 / (2 * kPi));   // applied to Z^1 weights
      p->t_sign[1] = add_table(p, KER_W2, 0, 0, -1.0 / (2 * kPi));  // applied to Z^2 weights
    } else {
      for (int a = 0; a < 3; ++a) p->t_sign[a] = add_table(p, KER_D3, a, 0, -1.0 / (4 * kPi));
    }
  }
  if (out_mask & DT_OUT_BACKWARD) p->t_rf = add_table(p, KER_RF, 0, 0, 1.0);

  // channel counts
  const int nh = D == 2 ? 3 : 6;
  const int in_fwd = (dist ? 1 : 0) + ((out_mask & DT_OUT_SIGN) ? D : 0);
  const int out_fwd = (dist ? 1 : 0) + (((out_mask & DT_OUT_GRAD) || hessfam) ? D : 0) + (hessfam ? nh : 0) +
                      ((out_mask & DT_OUT_SIGN) ? 1 : 0);
  p->in_max = std::max(in_fwd, (out_mask & DT_OUT_BACKWARD) ? 1 : 0);
  p->out_max = std::max(out_fwd, (out_mask & DT_OUT_BACKWARD) ? D + 1 : 0);
  p->in_max = std::max(p->in_max, 1);  // the backward's count image needs one channel

  // workspace layout
  const size_t cs = 2 * p->w;
  const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const int64_t My = p->M[1];
  size_t R1, R2;
  const size_t splat = (size_t)p->in_max * nx * ny * nz * p->w;
  if (D == 2) {
    const size_t A = (size_t)p->in_max * ny * p->MhP * cs;
    const size_t C = (size_t)p->out_max * ny * p->MhP * cs;
    R1 = std::max(splat, C);
    R2 = A;
  } else {
    const size_t A = (size_t)p->in_max * nz * ny * p->MhP * cs;
    const size_t B = (size_t)p->in_max * nz * My * p->MhP * cs;
    const size_t C = (size_t)p->out_max * nz * My * p->MhP * cs;
    const size_t Dd = (size_t)p->out_max * nz * ny * p->MhP * cs;
    R1 = std::max({splat, B, Dd});
    R2 = std::max(A, C);
  }
  // plan-time float64 scratch for the folded kernel samples
  const int64_t H0 = p->M[0] / 2 + 1, H1 = p->M[1] / 2 + 1, H2 = D == 3 ? p->M[2] / 2 + 1 : 1;
  const size_t fold = (size_t)H0 * H1 * H2 * sizeof(double);
  R1 = std::max(R1, fold);
  R2 = std::max(R2, fold);
  p->tab_elems = (size_t)p->MhP * H1 * H2;

  size_t off = 0;
  p->off_scal = off; off = align_up(off + 64 * sizeof(double));
  p->off_err = off; off = align_up(off + sizeof(uint32_t));
  p->off_partA = off; off = align_up(off + kPartials * sizeof(double));
  p->off_partB = off; off = align_up(off + kPartials * sizeof(double));
  for (int a = 0; a < D; ++a) {
    p->off_tw[a] = off; off = align_up(off + (size_t)p->M[a] * cs);
    p->off_tw64[a] = off; off = align_up(off + (size_t)p->M[a] * 16);
  }
  p->off_tabs = off;
  for (auto& t : p->tabs) {
    t.off = off - p->off_tabs;
    off = align_up(off + p->tab_elems * p->w);
  }
  p->off_R1 = off; off = align_up(off + R1);
  p->off_R2 = off; off = align_up(off + R2);
  p->R1 = R1;
  p->R2 = R2;
  p->ws_bytes = off;
  log_created(p);
  *out = p;
  return DT_OK;
}

extern "C" dt_status dt_create_plan(dt_plan* out, int ndim, const int64_t* dims, const double* spacing,
                                    const double* origin, double tau, int precision, unsigned out_mask,
                                    double trunc_dist, int64_t k_hint, double c_theta) {
  return create_plan(out, ndim, dims, spacing, origin, tau, precision, out_mask, trunc_dist, k_hint, c_theta, 0);
}

extern "C" dt_status dt_create_plan_reduced(dt_plan* out, int ndim, const int64_t* dims, const double* spacing,
                                            const double* origin, double tau, int precision, unsigned out_mask,
                                            int64_t k_max, double c_theta) {
  if (k_max < 1) return DT_E_ARG;
  return create_plan(out, ndim, dims, spacing, origin, tau, precision, out_mask, 0.0, 0, c_theta, k_max);
}

extern "C" dt_status dt_plan_workspace_size(dt_plan p, size_t* bytes) {
  if (!p || !bytes) return DT_E_ARG;
  *bytes = p->ws_bytes;
  return DT_OK;
}

extern "C" dt_status dt_destroy_plan(dt_plan p) {
  if (!p) return DT_E_ARG;
  p->release_static();
  delete p;
  return DT_OK;
}

extern "C" dt_status dt_plan_info(dt_plan p, dt_plan_info_t* info) {
  if (!p || !info) return DT_E_ARG;
  std::memset(info, 0, sizeof(*info));
  info->ndim = p->ndim;
  for (int a = 0; a < 3; ++a) {
    info->dims[a] = p->n[a];
    info->padded[a] = p->M[a];
    info->spacing[a] = p->h[a];
    info->origin[a] = p->o[a];
  }
  info->tau = p->tau;
  info->precision = p->prec;
  info->out_mask = p->mask;
  info->c_theta = p->c_theta;
  info->kernel_l1 = p->kernel_l1;
  info->unit_roundoff = p->unit();
  info->workspace_bytes = p->ws_bytes;
  info->n_tables = (int)p->tabs.size();
  info->k_max = p->k_max;
  for (int a = 0; a < 3; ++a) info->cut[a] = p->cut[a];
  return DT_OK;
}

// ---------------------------------------------------------------------------
// Workspace attach and plan-time spectra
// ---------------------------------------------------------------------------
namespace {

template <typename T> dt_status build_tables(dt_plan p, hipStream_t st) {
  const int D = p->ndim;
  // twiddles
  for (int a = 0; a < D; ++a) {
    std::vector<double> tw;
    make_twiddles((int)p->M[a], tw);
    std::vector<T> twt(tw.size());
    for (size_t i = 0; i < tw.size(); ++i) twt[i] = (T)tw[i];
    if (hipMemcpyAsync(p->ws + p->off_tw[a], twt.data(), twt.size() * sizeof(T), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return DT_E_HIP;
    if (hipMemcpyAsync(p->ws + p->off_tw64[a], tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return DT_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
  }
  TabGeom tg{};
  tg.ndim = D;
  for (int a = 0; a < 3; ++a) {
    tg.M[a] = a < D ? (int)p->M[a] : 1;
    tg.H[a] = a < D ? (int)(p->M[a] / 2 + 1) : 1;
    tg.h[a] = a < D ? p->h[a] : 1.0;
    tg.cut[a] = a < D ? p->cut[a] : 0;
  }
  double* buf0 = (double*)p->R1p();
  double* buf1 = (double*)p->R2p();
  std::vector<double> part(kPartials);
  // sample every kernel, record l1
  for (auto& t : p->tabs) {
    const int nb = launch_tab_sample(t.kd, tg, buf0, p->partA(), st);
    if (hipMemcpyAsync(part.data(), p->partA(), nb * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
      return DT_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
    double l1 = 0.0;
    for (int i = 0; i < nb; ++i) l1 += part[i];
    t.l1 = l1;
    t.e = ceil_log2(l1);
  }
  // the sign tables share one exponent (their products are summed)
  int es = -1000000;
  for (int a = 0; a < 3; ++a)
    if (p->t_sign[a] >= 0) es = std::max(es, p->tabs[p->t_sign[a]].e);
  for (int a = 0; a < 3; ++a)
    if (p->t_sign[a] >= 0) p->tabs[p->t_sign[a]].e = es;
  p->e_sign_tab = es;
  if (p->t_f >= 0) p->kernel_l1 = p->tabs[p->t_f].l1;
  else {
    // the validity threshold needs ||f||_1 even when f itself is not tabulated
    TabKernel kf{};
    kf.kind = KER_F;
    kf.tau = p->tau;
    const int nb = launch_tab_sample(kf, tg, buf0, p->partA(), st);
    if (hipMemcpyAsync(part.data(), p->partA(), nb * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
      return DT_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
    double l1 = 0.0;
    for (int i = 0; i < nb; ++i) l1 += part[i];
    p->kernel_l1 = l1;
  }
  // transform and store
  for (auto& t : p->tabs) {
    launch_tab_sample(t.kd, tg, buf0, p->partA(), st);
    double* cur = buf0;
    double* nxt = buf1;
    for (int a = 0; a < D; ++a) {
      launch_tab_axis(tg, a, t.par[a], p->ws + p->off_tw64[a], cur, nxt, st);
      std::swap(cur, nxt);
    }
    const double scale = std::ldexp(1.0, -t.e) / p->npad();
    launch_tab_store<T>(tg, cur, scale, (T*)(p->ws + p->off_tabs + t.off), p->NBf, p->MhP / p->NBf, st);
  }
  if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
  return hip_status(hipGetLastError());
}

}  // namespace

// Attach a workspace and build the plan-time tables in it (shared by
// dt_plan_set_workspace and dt_plan_set_static_workspace).
dt_status dt::plan_attach(dt_plan p, void* dev_ptr, size_t bytes, void* stream) {
  if (!p || !dev_ptr) return DT_E_ARG;
  if (bytes < p->ws_bytes || ((uintptr_t)dev_ptr % kAlign) != 0) return DT_E_WORKSPACE;
  p->release_static();
  hipStream_t st = (hipStream_t)stream;
  p->ws = (char*)dev_ptr;
  p->stream = st;
  p->ready = false;
  // clear the scalars, the error word and the pitch padding of the table region
  launch_fill_zero<double>((double*)p->ws, (int64_t)(p->off_R1 / sizeof(double)), st);
  if (p->dd) {
    hipError_t e = dd_build_tables(p->ws + p->off_dd_twx, p->ws + p->off_dd_twy, p->ws + p->off_dd_twz,
                                   p->ws + p->off_dd_tab, p->dd_tabs, p->dd_rf_tab, p->ws + p->off_dd_G, p->ddg, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return DT_E_HIP;
    p->kernel_l1 = host_kernel_l1(p->M, p->h, p->ndim, p->tau);
    p->ready = true;
    log_attached(p);
    return DT_OK;
  }
  const dt_status s = p->fp64 ? build_tables<double>(p, st) : build_tables<float>(p, st);
  if (s != DT_OK) return s;
  p->ready = true;
  log_attached(p);
  return DT_OK;
}

void dt::plan_mark_static(dt_plan p, int dev, uint64_t token) {
  p->static_dev = dev;
  p->static_token = token;
}

extern "C" dt_status dt_plan_set_workspace(dt_plan p, void* dev_ptr, size_t bytes, void* stream) {
  return dt::plan_attach(p, dev_ptr, bytes, stream);
}

// ---------------------------------------------------------------------------
// Calls
// ---------------------------------------------------------------------------
namespace {

struct Request {
  bool dist = false, grad = false, hess = false, sign = false;
};

dt_status check_shape(dt_plan p, const dt_shape* s) {
  if (!s) return DT_E_ARG;
  if (p->ndim == 2) {
    if (s->kind != DT_SHAPE_POLYGON || !s->points || s->n_points < 3) return DT_E_ARG;
  } else {
    if (s->kind != DT_SHAPE_MESH || !s->vertices || !s->faces || s->n_vertices < 3 || s->n_faces < 1)
      return DT_E_ARG;
  }
  return DT_OK;
}

struct Layout3 {
  int64_t lineA, zA, chA;   // after the x pass  [ch][z][y][kx]
  int64_t lineB, zB, chB;   // after the y pass  [ch][z][ky][kx]
  int64_t lineD, zD, chD;   // after the inverse y pass [c][z][y][kx]
};

template <typename T>
dt_status run_passes(dt_plan p, int n_in, const FusedSpec& fs, int n_out, hipStream_t st) {
  const int D = p->ndim;
  const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const int64_t My = p->M[1];
  const int MhP = p->MhP;
  auto tiles_for = [&](int64_t len, bool fused) {
    const int nb = col_tile_width((int)len, p->fp64, fused);
    return (p->Mh + nb - 1) / nb;
  };
  RowParams rp{};
  rp.n_lines = (int64_t)n_in * ny * nz;
  rp.nx = (int)nx;
  rp.pitch = MhP;
  rp.inner = p->Mh;
  rp.tw = p->ws + p->off_tw[0];
  {
    PassTimer t(p, st, "row_r2c");
    if (!launch_row_r2c<T>((const T*)p->R1p(), p->R2p(), rp, (int)(p->M[0] / 2), st)) return DT_E_UNSUPPORTED;
  }
  if (D == 2) {
    ColParams cp{};
    cp.in_line = MhP; cp.in_outer = 0; cp.in_ch = ny * MhP;
    cp.out_line = MhP; cp.out_outer = 0; cp.out_ch = ny * MhP;
    cp.inner = p->Mh; cp.n_in = (int)ny; cp.n_out = (int)ny; cp.outer_len = 1;
    cp.tw = p->ws + p->off_tw[1]; cp.tw_stride = 1;
    PassTimer t(p, st, "col_fused");
    if (!launch_col_fused<T>(p->R2p(), p->R1p(), cp, fs, (int)My, tiles_for(My, true), 1, st)) return DT_E_UNSUPPORTED;
  } else {
    const int64_t Mz = p->M[2];
    ColParams c2{};
    c2.in_line = MhP; c2.in_outer = ny * MhP; c2.in_ch = nz * ny * MhP;
    c2.out_line = MhP; c2.out_outer = My * MhP; c2.out_ch = nz * My * MhP;
    c2.inner = p->Mh; c2.n_in = (int)ny; c2.n_out = (int)My; c2.outer_len = (int)nz;
    c2.tw = p->ws + p->off_tw[1]; c2.tw_stride = 1;
    ColParams c3{};
    c3.in_line = My * MhP; c3.in_outer = MhP; c3.in_ch = nz * My * MhP;
    c3.out_line = My * MhP; c3.out_outer = MhP; c3.out_ch = nz * My * MhP;
    c3.inner = p->Mh; c3.n_in = (int)nz; c3.n_out = (int)nz; c3.outer_len = (int)My;
    c3.tw = p->ws + p->off_tw[2]; c3.tw_stride = 1;
    ColParams c4{};
    c4.in_line = MhP; c4.in_outer = My * MhP; c4.in_ch = nz * My * MhP;
    c4.out_line = MhP; c4.out_outer = ny * MhP; c4.out_ch = nz * ny * MhP;
    c4.inner = p->Mh; c4.n_in = (int)My; c4.n_out = (int)ny; c4.outer_len = (int)nz;
    c4.tw = p->ws + p->off_tw[1]; c4.tw_stride = 1;
    {
      PassTimer t(p, st, "col_fwd_y");
      if (!launch_col_c2c<T>(p->R2p(), p->R1p(), c2, (int)My, +1, tiles_for(My, false), (int)nz, n_in, st))
        return DT_E_UNSUPPORTED;
    }
    {
      PassTimer t(p, st, "col_fused");
      if (!launch_col_fused<T>(p->R1p(), p->R2p(), c3, fs, (int)Mz, tiles_for(Mz, true), (int)My, st))
        return DT_E_UNSUPPORTED;
    }
    {
      PassTimer t(p, st, "col_inv_y");
      if (!launch_col_c2c<T>(p->R2p(), p->R1p(), c4, (int)My, -1, tiles_for(My, false), (int)nz, n_out, st))
        return DT_E_UNSUPPORTED;
    }
  }
  return DT_OK;
}

// Work items of the fused pass: one per group (a mode-0 group's block
// column computes all of its outputs from one forward transform).
void fill_items(FusedSpec& fs) {
  fs.n_items = 0;
  for (int g = 0; g < fs.n_groups; ++g) {
    const FusedGroup& G = fs.g[g];
    fs.items[fs.n_items++] = {g, 0, G.mode == 1 ? 1 : G.n_out};
  }
}

void fill_tabrefs(dt_plan p, FusedSpec& fs) {
  for (size_t t = 0; t < p->tabs.size() && t < (size_t)kMaxTables; ++t) {
    TabRef& r = fs.tabs[t];
    r.ptr = p->tab_ptr((int)t);
    r.phase = p->tabs[t].phase;
    const int line_axis = p->ndim == 3 ? 2 : 1;
    r.odd_line = p->tabs[t].par[line_axis];
    r.odd_outer = p->ndim == 3 ? p->tabs[t].par[1] : 0;
  }
  const int64_t H_line = p->M[p->ndim - 1] / 2 + 1;
  const int64_t tiles = p->MhP / p->NBf;
  fs.tab_line_stride = p->NBf;
  fs.tab_tile_stride = H_line * p->NBf;
  fs.tab_outer_stride = p->ndim == 3 ? tiles * H_line * p->NBf : 0;
}

template <typename T>
dt_status run_forward(dt_plan p, const float* Y, int64_t K, const dt_shape* shape, const dt_outputs* out,
                      hipStream_t st) {
  const int D = p->ndim;
  Request rq;
  rq.hess = out->hess != nullptr || out->curv != nullptr;
  rq.grad = out->grad != nullptr || rq.hess;
  rq.dist = out->S != nullptr || rq.grad;
  rq.sign = out->label != nullptr || out->mu != nullptr;
  if (!rq.dist && !rq.sign) return DT_E_ARG;
  if (out->signed_outputs && !rq.sign) return DT_E_ARG;
  if (rq.dist && p->t_f < 0) return DT_E_ARG;
  if (rq.grad && p->t_u[0] < 0) return DT_E_ARG;
  if (rq.hess && p->t_h[0] < 0) return DT_E_ARG;
  if (rq.sign && p->t_sign[0] < 0) return DT_E_ARG;
  if (rq.sign || (rq.dist && !Y)) {
    const dt_status s = check_shape(p, shape);
    if (s != DT_OK) return s;
  }
  if (rq.dist && Y && K < 1) return DT_E_ARG;
  // the truncation holds for at most k_max sources
  if (p->k_max > 0 && rq.dist && (Y ? K : (D == 2 ? shape->n_points : shape->n_faces)) > p->k_max) return DT_E_ARG;
  if (!p->usable()) return DT_E_WORKSPACE;

  const int nh = D == 2 ? 3 : 6;
  const int n_in = (rq.dist ? 1 : 0) + (rq.sign ? D : 0);
  const int sign_in0 = rq.dist ? 1 : 0;
  int n_out = 0;
  FusedSpec fs{};
  fill_tabrefs(p, fs);
  EpiParams ep{};
  ep.ch_phi = -1;
  ep.ch_mu = -1;
  for (int a = 0; a < 3; ++a) ep.ch_u[a] = -1;
  for (int a = 0; a < 6; ++a) ep.ch_h[a] = -1;
  const GridGeom g = p->geom();
  const int64_t N = p->nodes();
  T* img = (T*)p->R1p();
  {
    PassTimer t(p, st, "fill");
    launch_fill_zero<T>(img, (int64_t)n_in * N, st);
  }

  // source counts
  int64_t Kc = 0;
  if (rq.dist) Kc = Y ? K : (D == 2 ? shape->n_points : shape->n_faces);
  const int e_g = rq.dist ? ceil_log2((double)Kc) : 0;
  const T cval = (T)std::ldexp(1.0, -e_g);
  // sign weight scale: |Z^i| <= extent, |P^i| <= extent^2 / 2
  double ext = 0.0;
  for (int a = 0; a < D; ++a) ext = std::max(ext, (double)p->n[a] * p->h[a]);
  int64_t Ks = rq.sign ? (D == 2 ? shape->n_points : shape->n_faces) : 0;
  const int e_s = rq.sign ? ceil_log2((double)Ks * (D == 2 ? ext : 0.5 * ext * ext)) : 0;
  const double ws_scale = std::ldexp(1.0, -e_s);

  T* cnt = rq.dist ? img : nullptr;
  T* sg[3] = {nullptr, nullptr, nullptr};
  if (rq.sign)
    for (int a = 0; a < D; ++a) sg[a] = img + (int64_t)(sign_in0 + a) * N;
  PassTimer* splat_t = new PassTimer(p, st, "splat");
  const double inv_cval = std::ldexp(1.0, e_g);
  double* msq = p->msq();
  if (rq.dist && Y) launch_splat_points<T>(Y, K, g, cnt, cval, inv_cval, msq, p->err(), st);
  const bool shape_counts = rq.dist && !Y;
  if (D == 2 && shape && (rq.sign || shape_counts))
    launch_splat_polygon<T>(shape->points, shape->n_points, g, shape_counts ? cnt : nullptr, cval, inv_cval,
                            shape_counts ? msq : nullptr, rq.sign ? sg[0] : nullptr, rq.sign ? sg[1] : nullptr,
                            ws_scale, ws_scale, p->err(), st);
  if (D == 3 && shape && (rq.sign || shape_counts))
    launch_splat_mesh<T>(shape->vertices, shape->n_vertices, shape->faces, shape->n_faces, g,
                         shape_counts ? cnt : nullptr, cval, inv_cval, shape_counts ? msq : nullptr, sg[0], sg[1],
                         sg[2], ws_scale, ws_scale, ws_scale, p->err(), st);
  delete splat_t;

  // validity scalars (the splat accumulated the sum of squared multiplicities)
  if (rq.dist) {
    PassTimer t(p, st, "validity");
    const double coef = p->c_theta * p->unit() * std::log2(p->npad()) * p->kernel_l1 / std::sqrt(p->npad());
    launch_finalize_theta_msq(msq, coef, p->tau, p->scal(), st);
  }

  // fused groups and epilogue channel map
  int gi = 0;
  if (rq.dist) {
    FusedGroup& G = fs.g[gi++];
    G.mode = 0;
    G.n_in = 1;
    G.in_ch[0] = 0;
    G.n_out = 0;
    auto push = [&](int tab) {
      G.out_ch[G.n_out] = n_out;
      G.tab[G.n_out] = tab;
      ++G.n_out;
      return n_out++;
    };
    const int ef = p->tabs[p->t_f].e;
    ep.ch_phi = push(p->t_f);
    ep.scale_phi = std::ldexp(1.0, e_g + ef);
    if (rq.grad)
      for (int a = 0; a < D; ++a) {
        ep.ch_u[a] = push(p->t_u[a]);
        ep.scale_u[a] = std::ldexp(1.0, p->tabs[p->t_u[a]].e - ef);
      }
    if (rq.hess)
      for (int hh = 0; hh < nh; ++hh) {
        ep.ch_h[hh] = push(p->t_h[hh]);
        ep.scale_h[hh] = std::ldexp(1.0, p->tabs[p->t_h[hh]].e - ef);
      }
  }
  if (rq.sign) {
    FusedGroup& G = fs.g[gi++];
    G.mode = 1;
    G.n_in = D;
    for (int a = 0; a < D; ++a) {
      G.in_ch[a] = sign_in0 + a;
      G.tab[a] = p->t_sign[a];
    }
    G.n_out = 1;
    G.out_ch[0] = n_out;
    ep.ch_mu = n_out++;
    ep.scale_mu = std::ldexp(1.0, e_s + p->e_sign_tab);
  }
  fs.n_groups = gi;
  fill_items(fs);

  dt_status s = run_passes<T>(p, n_in, fs, n_out, st);
  if (s != DT_OK) return s;

  // final x pass with the epilogue
  const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
  RowParams rp{};
  rp.n_lines = ny * nz;
  rp.nx = (int)nx;
  rp.pitch = p->MhP;
  rp.inner = p->Mh;
  rp.tw = p->ws + p->off_tw[0];
  ep.C = n_out;
  ep.ch_stride = (int64_t)nz * ny * p->MhP;
  ep.tau = p->tau;
  ep.theta = p->scal();
  ep.ndim = D;
  ep.n_rows = ny * nz;
  ep.nx = (int)nx;
  ep.plane = N;
  ep.S = out->S;
  ep.grad = out->grad;
  ep.hess = out->hess;
  ep.label = out->label;
  ep.mu = out->mu;
  ep.signed_out = out->signed_outputs;
  ep.curv = out->curv;
  {
    PassTimer t(p, st, "row_c2r_epi");
    if (!launch_row_c2r_epi<T>(p->R1p(), rp, ep, (int)(p->M[0] / 2), st)) return DT_E_UNSUPPORTED;
  }
  return hip_status(hipGetLastError());
}

template <typename T>
dt_status run_backward(dt_plan p, const float* Y, int64_t K, const void* S, const void* G, float* dY, double* dtau,
                       hipStream_t st) {
  const int D = p->ndim;
  const int64_t N = p->nodes();
  const GridGeom g = p->geom();
  T* img = (T*)p->R1p();
  // validity threshold of the forward call with the same sources
  const int e_g = ceil_log2((double)K);
  const T cval = (T)std::ldexp(1.0, -e_g);
  {
    PassTimer t(p, st, "fill");
    launch_fill_zero<T>(img, N, st);
  }
  {
    PassTimer t(p, st, "splat");
    launch_splat_points<T>(Y, K, g, img, cval, std::ldexp(1.0, e_g), p->msq(), p->err(), st);
  }
  {
    PassTimer t(p, st, "validity");
    const double coef = p->c_theta * p->unit() * std::log2(p->npad()) * p->kernel_l1 / std::sqrt(p->npad());
    launch_finalize_theta_msq(p->msq(), coef, p->tau, p->scal(), st);
  }
  // w = G exp(S/tau) on valid nodes (overwrites the count image)
  int ngs;
  {
    PassTimer t(p, st, "prep_w");
    ngs = launch_prep_w<T>((const T*)S, (const T*)G, N, p->scal(), p->tau, img, p->partA(), st);
  }
  // w * u_i and w * (r f)
  FusedSpec fs{};
  fill_tabrefs(p, fs);
  fs.n_groups = 1;
  FusedGroup& Gr = fs.g[0];
  Gr.mode = 0;
  Gr.n_in = 1;
  Gr.in_ch[0] = 0;
  Gr.n_out = D + 1;
  for (int a = 0; a < D; ++a) {
    Gr.out_ch[a] = a;
    Gr.tab[a] = p->t_u[a];
  }
  Gr.out_ch[D] = D;
  Gr.tab[D] = p->t_rf;
  fill_items(fs);
  dt_status s = run_passes<T>(p, 1, fs, D + 1, st);
  if (s != DT_OK) return s;
  GatherParams gp{};
  gp.g = g;
  gp.Y = Y;
  gp.K = K;
  gp.spec = p->R1p();
  gp.ch_stride = (int64_t)p->n[2] * p->n[1] * p->MhP;
  gp.pitch = p->MhP;
  gp.inner = p->Mh;
  gp.Mx = (int)p->M[0];
  gp.tw = p->ws + p->off_tw[0];
  gp.nu = D;
  gp.has_rf = 1;
  for (int a = 0; a < D; ++a) gp.ch_scale[a] = std::ldexp(1.0, p->tabs[p->t_u[a]].e);
  gp.ch_scale[D] = std::ldexp(1.0, p->tabs[p->t_rf].e);
  gp.scal = p->scal();
  gp.dY = dY;
  gp.partials = p->partB();
  PassTimer* gt = new PassTimer(p, st, "gather");
  const int nrf = launch_gather<T>(gp, st);
  launch_finalize_dtau(p->partA(), ngs, p->partB(), nrf, 1.0, p->tau, p->scal(), dtau, st);
  delete gt;
  return hip_status(hipGetLastError());
}

}  // namespace

// The extended-precision pipeline (double-double or quad-double): S, grad S,
// the Hessian and curvatures from explicit sources.
static dt_status run_forward_dd(dt_plan p, const float* Y, int64_t K, const dt_shape* shape, const dt_outputs* out,
                         hipStream_t st) {
  if (out->label || out->mu || out->signed_outputs || shape) return DT_E_UNSUPPORTED;
  if ((!out->S && !out->grad && !out->hess && !out->curv) || !Y || K < 1) return DT_E_ARG;
  const int nh = p->ndim == 2 ? 3 : 6;
  const bool second = out->hess || out->curv;
  if (out->grad && p->dd_tabs < 1 + p->ndim) return DT_E_ARG;   // gradient kernels not prepared
  if (second && p->dd_tabs < 1 + p->ndim + nh) return DT_E_ARG;  // Hessian kernels not prepared
  const int C = second ? 1 + p->ndim + nh : out->grad ? 1 + p->ndim : 1;
  if (!p->usable()) return DT_E_WORKSPACE;
  const DDGeom& g = p->ddg;
  double* cnt = (double*)(p->ws + p->off_dd_cnt);
  char* G = p->ws + p->off_dd_G;
  hipError_t e;
  {
    PassTimer t(p, st, "splat");
    launch_fill_zero<double>(cnt, (int64_t)g.nx * g.ny * g.nz, st);
    e = dd_launch_splat(Y, K, cnt, p->msq(), p->err(), g, st);
    if (e == hipSuccess) e = dd_launch_finalize(p->msq(), p->scal(), g, p->c_theta, p->unit(), p->kernel_l1, st);
  }
  if (e != hipSuccess) return DT_E_HIP;
  DDChannels ch{};
  ch.C = C;
  for (int c = 0; c < C; ++c) {
    ch.tab_of[c] = c;
    if (c >= 1 && c <= p->ndim) ch.imag |= 1u << c;
  }
  {
    PassTimer t(p, st, "dd_row_fwd");
    e = dd_convolve_rows(cnt, G, p->ws + p->off_dd_twx, g, st);
  }
  if (e != hipSuccess) return DT_E_HIP;
  {
    PassTimer t(p, st, g.ndim == 2 ? "dd_col_fused" : "dd_columns_3d");
    e = dd_convolve_columns(G, p->ws + p->off_dd_Gc, p->ws + p->off_dd_tab, ch, p->ws + p->off_dd_twy,
                            p->ws + p->off_dd_twz, g, st);
  }
  if (e != hipSuccess) return DT_E_HIP;
  {
    PassTimer t(p, st, "dd_row_inv_epi");
    e = dd_launch_row_inv_epi(p->ws + p->off_dd_Gc, C, p->ws + p->off_dd_twx, (double*)out->S, (double*)out->grad,
                              (double*)out->hess, (double*)out->curv, p->scal(), g, st);
  }
  return hip_status(e);
}

// The extended-precision adjoint (as run_backward): w = G exp(S / tau) p2 on
// valid nodes, its convolutions with the gradient kernels and with r f in
// the plan's extended type, their values at the sources' nodes.
static dt_status run_backward_dd(dt_plan p, const float* Y, int64_t K, const double* S, const double* Gr, float* dY,
                                 double* dtau, hipStream_t st) {
  const DDGeom& g = p->ddg;
  const int D = p->ndim;
  const int64_t N = (int64_t)g.nx * g.ny * g.nz;
  double* img = (double*)(p->ws + p->off_dd_cnt);
  char* G = p->ws + p->off_dd_G;
  hipError_t e;
  int ngs = 0, nrf = 0;
  {
    PassTimer t(p, st, "splat");
    launch_fill_zero<double>(img, N, st);
    e = dd_launch_splat(Y, K, img, p->msq(), p->err(), g, st);
    if (e == hipSuccess) e = dd_launch_finalize(p->msq(), p->scal(), g, p->c_theta, p->unit(), p->kernel_l1, st);
  }
  if (e != hipSuccess) return DT_E_HIP;
  {
    PassTimer t(p, st, "prep_w");
    ngs = launch_prep_w<double>(S, Gr, N, p->scal(), p->tau, img, p->partA(), st);
  }
  DDChannels ch{};
  ch.C = D + 1;
  for (int a = 0; a < D; ++a) {
    ch.tab_of[a] = 1 + a;
    ch.imag |= 1u << a;
  }
  ch.tab_of[D] = p->dd_rf_tab;
  {
    PassTimer t(p, st, "dd_convolve");
    e = dd_convolve_rows(img, G, p->ws + p->off_dd_twx, g, st);
    if (e == hipSuccess)
      e = dd_convolve_columns(G, p->ws + p->off_dd_Gc, p->ws + p->off_dd_tab, ch, p->ws + p->off_dd_twy,
                              p->ws + p->off_dd_twz, g, st);
  }
  if (e != hipSuccess) return DT_E_HIP;
  {
    PassTimer t(p, st, "dd_gather");
    e = dd_launch_row_inv_plain(p->ws + p->off_dd_Gc, D + 1, p->ws + p->off_dd_twx, (double*)G, g, st);
    if (e == hipSuccess) e = dd_launch_gather(Y, K, (const double*)G, p->scal(), dY, p->partB(), kPartials, &nrf, g, st);
    if (e == hipSuccess) launch_finalize_dtau(p->partA(), ngs, p->partB(), nrf, 1.0, p->tau, p->scal(), dtau, st);
  }
  if (e != hipSuccess) return DT_E_HIP;
  return hip_status(hipGetLastError());
}

extern "C" dt_status dt_forward(dt_plan p, const float* Y, int64_t K, const dt_shape* shape, const dt_outputs* out,
                                void* stream) {
  if (!p || !out) return DT_E_ARG;
  if (!Y && K != 0) return DT_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  p->stream = st;
  if (p->dd) return run_forward_dd(p, Y, K, shape, out, st);
  return p->fp64 ? run_forward<double>(p, Y, K, shape, out, st) : run_forward<float>(p, Y, K, shape, out, st);
}

extern "C" dt_status dt_distance(dt_plan p, const float* Y, int64_t K, void* S, void* stream) {
  if (!p || !Y || !S || K < 1) return DT_E_ARG;
  dt_outputs o{};
  o.S = S;
  return dt_forward(p, Y, K, nullptr, &o, stream);
}

extern "C" dt_status dt_gradient(dt_plan p, const float* Y, int64_t K, void* S_or_null, void* grad, void* stream) {
  if (!p || !Y || !grad || K < 1) return DT_E_ARG;
  dt_outputs o{};
  o.S = S_or_null;
  o.grad = grad;
  return dt_forward(p, Y, K, nullptr, &o, stream);
}

extern "C" dt_status dt_hessian(dt_plan p, const float* Y, int64_t K, void* hess, void* stream) {
  if (!p || !Y || !hess || K < 1) return DT_E_ARG;
  dt_outputs o{};
  o.hess = hess;
  return dt_forward(p, Y, K, nullptr, &o, stream);
}

extern "C" dt_status dt_sign(dt_plan p, const dt_shape* shape, int8_t* label, void* mu, void* stream) {
  if (!p || !shape || (!label && !mu)) return DT_E_ARG;
  dt_outputs o{};
  o.label = label;
  o.mu = mu;
  return dt_forward(p, nullptr, 0, shape, &o, stream);
}

extern "C" dt_status dt_backward(dt_plan p, const float* Y, int64_t K, const void* S, const void* dL_dS,
                                 float* dL_dY, double* dL_dtau, void* stream) {
  if (!p || !Y || K < 1 || !S || !dL_dS || !dL_dY) return DT_E_ARG;
  if (!(p->mask & DT_OUT_BACKWARD)) return DT_E_ARG;
  if (p->k_max > 0 && K > p->k_max) return DT_E_ARG;
  if (!p->usable()) return DT_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  p->stream = st;
  if (p->dd) return run_backward_dd(p, Y, K, (const double*)S, (const double*)dL_dS, dL_dY, dL_dtau, st);
  return p->fp64 ? run_backward<double>(p, Y, K, S, dL_dS, dL_dY, dL_dtau, st)
                 : run_backward<float>(p, Y, K, S, dL_dS, dL_dY, dL_dtau, st);
}

extern "C" dt_status dt_last_error(dt_plan p) {
  if (!p) return DT_E_ARG;
  if (!p->ws || !p->usable()) return DT_E_WORKSPACE;
  uint32_t bits = 0;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return DT_E_HIP;
  if (hipMemcpy(&bits, p->err(), sizeof(bits), hipMemcpyDeviceToHost) != hipSuccess) return DT_E_HIP;
  const uint32_t zero = 0;
  if (hipMemcpy(p->err(), &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) return DT_E_HIP;
  return bits ? DT_E_RANGE : DT_OK;
}

extern "C" dt_status dt_last_stats(dt_plan p, dt_call_stats* st) {
  if (!p || !st) return DT_E_ARG;
  if (!p->ws || !p->usable()) return DT_E_WORKSPACE;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return DT_E_HIP;
  double s[5];
  if (hipMemcpy(s, p->scal(), sizeof(s), hipMemcpyDeviceToHost) != hipSuccess) return DT_E_HIP;
  uint32_t bits = 0;
  if (hipMemcpy(&bits, p->err(), sizeof(bits), hipMemcpyDeviceToHost) != hipSuccess) return DT_E_HIP;
  st->theta = s[0];
  st->s_max = s[1];
  st->g_l2 = s[2];
  st->dL_dtau = s[4];
  st->error_bits = bits;
  logf("plan %p last call: ||g||_2 = %.6g, Theta = %.4g, S_max = %.3f tau, error bits %u", (void*)p, st->g_l2,
       st->theta, st->s_max / p->tau, bits);
  return DT_OK;
}

extern "C" dt_status dt_plan_set_timing(dt_plan p, int enable) {
  if (!p) return DT_E_ARG;
  p->timing = enable != 0;
  return DT_OK;
}

extern "C" dt_status dt_plan_timings(dt_plan p, dt_pass_timing* out, int max_entries, int* n_entries) {
  if (!p || !n_entries || (max_entries > 0 && !out)) return DT_E_ARG;
  if (!p->pending.empty() && hipStreamSynchronize(p->stream) != hipSuccess) return DT_E_HIP;
  for (auto& q : p->pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, q.a, q.b) != hipSuccess) return DT_E_HIP;
    bool found = false;
    for (auto& e : p->acc)
      if (e.first == q.name) {
        e.second.first += 1;
        e.second.second += ms;
        found = true;
      }
    if (!found) p->acc.push_back({q.name, {1, (double)ms}});
    p->pool.push_back(q.a);
    p->pool.push_back(q.b);
  }
  p->pending.clear();
  int n = 0;
  for (auto& e : p->acc) {
    if (n < max_entries) {
      std::memset(out[n].name, 0, sizeof(out[n].name));
      std::strncpy(out[n].name, e.first.c_str(), sizeof(out[n].name) - 1);
      out[n].launches = e.second.first;
      out[n].total_ms = e.second.second;
    }
    ++n;
  }
  *n_entries = n;
  return DT_OK;
}

extern "C" dt_status dt_plan_reset_timings(dt_plan p) {
  if (!p) return DT_E_ARG;
  int n = 0;
  const dt_status s = dt_plan_timings(p, nullptr, 0, &n);
  p->acc.clear();
  return s;
}

extern "C" const char* dt_status_str(dt_status s) {
  // A C caller may pass any int: read the bits as an int rather than load a
  // C++ enum value outside the enumerators' range.
  int v;
  std::memcpy(&v, &s, sizeof(v));
  switch (v) {
    case DT_OK: return "ok";
    case DT_E_ARG: return "invalid argument";
    case DT_E_RANGE: return "a source was outside the grid or non-finite";
    case DT_E_PRECISION: return "requested distance not representable in any supported precision";
    case DT_E_WORKSPACE: return "workspace missing, too small or misaligned";
    case DT_E_HIP: return "HIP runtime error";
    case DT_E_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}
