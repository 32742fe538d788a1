// Host side of the batched 2D path: plan creation (7-smooth padding, radix
// schedules, workspace layout), plan-time kernel spectra per distinct
// geometry, block lists per pass, the launch sequence (eager or replayed from
// a captured HIP graph) and the tile autotuner.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "dt.h"
#include "dt_batch.hpp"
#include "dt_log.hpp"

using namespace dt;

namespace {

constexpr size_t kAlignB = 256;
constexpr int kPartialsB = 4096;
constexpr int kLdsRowBudget = 65536;   // bytes of LDS per row-pass block

size_t align_b(size_t v) { return (v + kAlignB - 1) / kAlignB * kAlignB; }

int ceil_log2_d(double v) {
  if (!(v > 0)) return 0;
  int e;
  const double f = std::frexp(v, &e);
  return f == 0.5 ? e - 1 : e;
}

bool finite_pos_b(double v) { return std::isfinite(v) && v > 0; }

dt_status hip_st(hipError_t e) { return e == hipSuccess ? DT_OK : DT_E_HIP; }

}  // namespace

namespace dt {

// Smallest 2^a 3^b 5^c 7^d >= n.
int64_t smooth7_at_least(int64_t n) {
  for (int64_t m = std::max<int64_t>(n, 1);; ++m) {
    int64_t r = m;
    for (int p : {2, 3, 5, 7})
      while (r % p == 0) r /= p;
    if (r == 1) return m;
  }
}

// Radix schedules of a 7-smooth length; dt_batch_autotune picks one per pass
// and length:
//   0: radix 8 while possible, then one 4 or 2, then 7, 5, 3;
//   1: the odd radices 7, 5, 3 first, then as 0;
//   2: radix 4 while possible, then one 2, then 7, 5, 3;
//   3: the one 4 or 2 first, then radix 8, then 7, 5, 3.
// Returns false if the length is not 7-smooth or needs too many stages.
bool mixed_plan_for(int64_t N, int family, MixedPlan& mp) {
  if (family < 0 || family >= kMixedFamilies || N < 1) return false;
  int64_t r = N;
  int a2 = 0;
  while (r % 2 == 0) {
    r /= 2;
    ++a2;
  }
  std::vector<int> odd, pow2;
  for (int q : {7, 5, 3})
    while (r % q == 0) {
      r /= q;
      odd.push_back(q);
    }
  if (r != 1) return false;
  if (family >= 4) {
    // Fused radices up to 16: radix 16 while possible; a leftover 2 joins the
    // smallest odd factor (6, 10, 14), a leftover 4 a factor 3 (12); the odd
    // factors pair largest with smallest where the product is at most 15
    // (9, 15).  Family 4 puts the powers of two first, family 5 the odd
    // radices.
    std::vector<int> p2, od;
    for (; a2 >= 4; a2 -= 4) p2.push_back(16);
    std::sort(odd.begin(), odd.end());
    if (a2 > 0 && !odd.empty() && (1 << a2) * odd.front() <= 14) {
      od.push_back((1 << a2) * odd.front());
      odd.erase(odd.begin());
    } else if (a2 > 0) {
      p2.push_back(1 << a2);
    }
    size_t lo = 0, hi = odd.size();
    while (hi > lo) {
      if (hi - lo >= 2 && odd[hi - 1] * odd[lo] <= 15) {
        od.push_back(odd[hi - 1] * odd[lo]);
        ++lo;
        --hi;
      } else {
        od.push_back(odd[hi - 1]);
        --hi;
      }
    }
    std::vector<int> rad = family == 4 ? p2 : od;
    const std::vector<int>& rest = family == 4 ? od : p2;
    rad.insert(rad.end(), rest.begin(), rest.end());
    if ((int)rad.size() > kMixedMaxStages) return false;
    mp.n_st = (int)rad.size();
    int64_t ns = 1;
    for (int st = 0; st < mp.n_st; ++st) {
      if (!mixed_radix_supported(rad[st])) return false;
      mp.radix[st] = rad[st];
      mp.m_ns[st] = fastdiv_magic((uint32_t)ns);
      mp.m_nbf[st] = fastdiv_magic((uint32_t)(N / rad[st]));
      ns *= rad[st];
    }
    return true;
  }
  if (family == 2) {
    for (; a2 >= 2; a2 -= 2) pow2.push_back(4);
    if (a2) pow2.push_back(2);
  } else {
    const int small = a2 % 3 == 2 ? 4 : a2 % 3 == 1 ? 2 : 0;
    if (family == 3 && small) pow2.push_back(small);
    for (int i = 0; i < a2 / 3; ++i) pow2.push_back(8);
    if (family != 3 && small) pow2.push_back(small);
  }
  std::vector<int> rad = family == 1 ? odd : pow2;
  const std::vector<int>& rest = family == 1 ? pow2 : odd;
  rad.insert(rad.end(), rest.begin(), rest.end());
  if ((int)rad.size() > kMixedMaxStages) return false;
  mp.n_st = (int)rad.size();
  int64_t ns = 1;
  for (int st = 0; st < mp.n_st; ++st) {
    mp.radix[st] = rad[st];
    mp.m_ns[st] = fastdiv_magic((uint32_t)ns);
    mp.m_nbf[st] = fastdiv_magic((uint32_t)(N / rad[st]));
    ns *= rad[st];
  }
  return true;
}

bool same_plan(const MixedPlan& a, const MixedPlan& b) {
  if (a.n_st != b.n_st) return false;
  for (int s = 0; s < a.n_st; ++s)
    if (a.radix[s] != b.radix[s]) return false;
  return true;
}

}  // namespace dt

struct dt_batch_plan_s {
  int n = 0;
  bool fp64 = false;
  unsigned mask = 0;
  int C = 1;
  double c_theta = 256.0;
  std::vector<dt_instance_desc> desc;
  std::vector<BatchInst> inst;
  std::vector<int> geo_of;
  struct Geo {
    int64_t Mx, My, pitch;
    int cut[2];                 // truncation box in cells (0: none)
    double hx, hy, tau;
    int64_t tab_off;
    double l1;
    int e[kBatchChan];
  };
  std::vector<Geo> geos;
  std::map<int64_t, int64_t> tw_off, tw64_off;   // length -> element offset
  int64_t n_tw = 0, n_tw64 = 0, n_tab = 0, n_img = 0, n_spec = 0, n_fused = 0, n_scratch = 0;
  int64_t total_nodes = 0;
  size_t off_inst = 0, off_blk[3] = {0, 0, 0}, off_koff = 0, off_scal = 0, off_err = 0, off_part = 0, off_tw = 0,
         off_tw64 = 0, off_tab = 0, off_A = 0, off_B = 0, ws_bytes = 0;
  int64_t blk_cap[3] = {0, 0, 0};
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool ready = false;
  int lds_max = 65536;
  dt_batch_tiles tiles{8, 256, 256};
  bool tiles_set = false;   // the caller chose tiles before the workspace was attached
  int nblk[3] = {0, 0, 0}, ecap[3] = {0, 0, 0};
  size_t lds[3] = {0, 0, 0};
  bool blocks_valid = false;
  std::vector<int> sched;          // radix schedule family per instance and pass (3 per instance)
  std::vector<int64_t> koff;       // offsets the device copy holds
  bool koff_valid = false;
  // graph replay
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  const float* g_Y = nullptr;
  void* g_S = nullptr;
  void* g_grad = nullptr;
  hipStream_t g_stream = nullptr;
  int64_t version = 0, g_version = -1;

  size_t wsz() const { return fp64 ? 8 : 4; }
  double unit() const { return fp64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24); }
  BatchInst* d_inst() const { return (BatchInst*)(ws + off_inst); }
  BatchBlock* d_blk(int i) const { return (BatchBlock*)(ws + off_blk[i]); }
  int64_t* d_koff() const { return (int64_t*)(ws + off_koff); }
  double* d_scal() const { return (double*)(ws + off_scal); }
  uint32_t* d_err() const { return (uint32_t*)(ws + off_err); }
  double* d_part() const { return (double*)(ws + off_part); }
  char* d_tw() const { return ws + off_tw; }
  double* d_tw64() const { return (double*)(ws + off_tw64); }
  char* d_tab() const { return ws + off_tab; }
  char* d_A() const { return ws + off_A; }
  char* d_B() const { return ws + off_B; }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    g_version = -1;
  }
};

namespace {

// Pass indices of the block lists.
enum { P_R2C = 0, P_COL = 1, P_EPI = 2 };

// Rows per block of a row pass: as many as fit ECAP_max * nthr elements and
// the LDS budget, at most the rows left.
int rows_per_block(int64_t sx, int lines_per_row, int nthr, size_t w) {
  const int64_t by_regs = (int64_t)32 * nthr / (sx * lines_per_row);
  const int64_t by_lds = (int64_t)kLdsRowBudget / ((sx + 1) * lines_per_row * 2 * (int64_t)w);
  return (int)std::max<int64_t>(1, std::min(by_regs, by_lds));
}

int ecap_for(int64_t elems, int nthr) {
  const int64_t e = (elems + nthr - 1) / nthr;
  return e <= 8 ? 8 : e <= 16 ? 16 : e <= 32 ? 32 : 64;
}

constexpr int kXcds = 8;   // accelerator complex dies of an MI355X, each with its own L2

// The dispatcher deals a launch's blocks to the XCDs round-robin (block b to
// XCD b mod 8).  Neighbouring column tiles share 128-byte lines of the
// spectrum and of the kernel tables, so the column list is reordered to give
// every XCD one contiguous run of tiles: XCD x takes q + (x < rem) tiles
// starting at x q + min(x, rem), q = n / 8, rem = n mod 8.  A permutation:
// every tile still runs exactly once.
template <typename B> std::vector<B> xcd_runs(const std::vector<B>& v) {
  const int64_t n = (int64_t)v.size(), q = n / kXcds, rem = n % kXcds;
  std::vector<B> out(v.size());
  for (int64_t b = 0; b < n; ++b) {
    const int64_t x = b % kXcds, j = b / kXcds;
    out[b] = v[x * q + std::min<int64_t>(x, rem) + j];
  }
  return out;
}

// Default tiles: 1024 threads per column block (512 if nothing fits) and
// the widest power-of-two tile whose longest column set fits 8 elements per
// thread (the lightest instantiation in registers) and the LDS; 512 threads
// per row block.
dt_batch_tiles default_tiles(dt_batch_plan p) {
  int64_t my = 0;
  for (const auto& I : p->inst) my = std::max<int64_t>(my, I.My);
  dt_batch_tiles t{1, 512, 512};
  for (int nt : {1024, 512})
    for (int nb : {16, 8, 4, 2, 1})
      if (my * nb <= 8 * nt && (size_t)(2 * my * nb + my) * 2 * p->wsz() <= (size_t)p->lds_max) {
        t.col_nb = nb;
        t.col_threads = nt;
        return t;
      }
  return t;
}

// -- plan log (DT_LOG) --------------------------------------------------------
std::string radices(const MixedPlan& mp) {
  std::string r;
  for (int s = 0; s < mp.n_st; ++s) r += (s ? "x" : "") + std::to_string(mp.radix[s]);
  return r;
}

void log_blocks(dt_batch_plan p) {
  if (!log_enabled()) return;
  static const char* pass[3] = {"rows", "columns", "epilogue rows"};
  logf("batch plan %p blocks: tiles col_nb %d, col_threads %d, row_threads %d", (void*)p, p->tiles.col_nb,
       p->tiles.col_threads, p->tiles.row_threads);
  for (int k = 0; k < 3; ++k)
    logf("  %s: %d blocks, up to %d points per thread, %zu B of LDS", pass[k], p->nblk[k], p->ecap[k], p->lds[k]);
  for (int i = 0; i < p->n; ++i) {
    const BatchInst& I = p->inst[i];
    logf("  inst %d: schedule families %d/%d/%d, radices rows %s, columns %s, inverse rows %s", i, p->sched[3 * i],
         p->sched[3 * i + 1], p->sched[3 * i + 2], radices(I.px).c_str(), radices(I.py).c_str(),
         radices(I.pxi).c_str());
  }
}

// Build the three block lists for the current tiles and upload them (only
// for the instances with keep[i] != 0 when keep is given: the autotuner times
// one pass over the instances of one length).
dt_status build_blocks(dt_batch_plan p, hipStream_t st, const std::vector<char>* keep = nullptr) {
  p->blocks_valid = false;
  const size_t w = p->wsz();
  std::vector<BatchBlock> lists[3];
  int64_t need[3] = {0, 0, 0};
  size_t lds[3] = {0, 0, 0};
  const int nt_row = p->tiles.row_threads, nt_col = p->tiles.col_threads, nb = p->tiles.col_nb;
  if (nt_row < 64 || nt_row > 512 || nt_col < 64 || nt_col > 1024 || nb < 1 || nb > 64) return DT_E_ARG;
  int64_t my_max = 0;
  for (const auto& I : p->inst) my_max = std::max<int64_t>(my_max, I.My);
  for (int i = 0; i < p->n; ++i) {
    if (keep && !(*keep)[i]) continue;
    const BatchInst& I = p->inst[i];
    const int64_t sx = I.sx;
    // row r2c: one line per row
    int r = std::min<int>(rows_per_block(sx, 1, nt_row, w), I.ny);
    for (int y = 0; y < I.ny; y += r) {
      const int c = std::min(r, I.ny - y);
      lists[P_R2C].push_back({i, y, c, (int)fastdiv_magic((uint32_t)c)});
      need[P_R2C] = std::max<int64_t>(need[P_R2C], sx * c);
      lds[P_R2C] = std::max<size_t>(lds[P_R2C], (size_t)(c * (sx + 1) + 2 * sx) * 2 * w);   // lines + twiddles
    }
    // column pass: the tile width applies to the longest columns; shorter
    // columns take proportionally more bins (the same elements per block,
    // at most 64 bins), so small instances still fill the block's threads
    // and read longer row segments
    const int nbi = (int)std::min<int64_t>(64, std::max<int64_t>(nb, nb * my_max / I.My));
    for (int kx = 0; kx <= sx; kx += nbi) {
      const int c = (int)std::min<int64_t>(nbi, sx + 1 - kx);
      lists[P_COL].push_back({i, kx, c, (int)fastdiv_magic((uint32_t)c)});
      need[P_COL] = std::max<int64_t>(need[P_COL], (int64_t)I.My * c);
      // spectrum + work column + the twiddle table
      lds[P_COL] = std::max<size_t>(lds[P_COL], (size_t)(2 * I.My * c + I.My) * 2 * w);
    }
    // epilogue: C lines per row
    r = std::min<int>(rows_per_block(sx, p->C, nt_row, w), I.ny);
    for (int y = 0; y < I.ny; y += r) {
      const int c = std::min(r, I.ny - y);
      lists[P_EPI].push_back({i, y, c, (int)fastdiv_magic((uint32_t)(c * p->C))});
      need[P_EPI] = std::max<int64_t>(need[P_EPI], sx * c * p->C);
      lds[P_EPI] = std::max<size_t>(lds[P_EPI], (size_t)(c * p->C * (sx + 1) + 2 * sx) * 2 * w);
    }
  }
  lists[P_COL] = xcd_runs(lists[P_COL]);
  const int nthr[3] = {nt_row, nt_col, nt_row};
  for (int k = 0; k < 3; ++k) {
    if ((int64_t)lists[k].size() > p->blk_cap[k]) return DT_E_UNSUPPORTED;
    const int e = ecap_for(need[k], nthr[k]);
    if (e > 32) return DT_E_UNSUPPORTED;
    if (e > 8 && nthr[k] > 512) return DT_E_UNSUPPORTED;
    if (lds[k] > (size_t)p->lds_max) return DT_E_UNSUPPORTED;
    p->ecap[k] = e;
    p->lds[k] = lds[k];
    p->nblk[k] = (int)lists[k].size();
    if (!lists[k].empty() &&
        hipMemcpyAsync(p->d_blk(k), lists[k].data(), lists[k].size() * sizeof(BatchBlock), hipMemcpyHostToDevice,
                       st) != hipSuccess)
      return DT_E_HIP;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
  p->blocks_valid = true;
  p->drop_graph();
  if (!keep) log_blocks(p);
  return DT_OK;
}

template <typename T> dt_status build_batch_tables(dt_batch_plan p, hipStream_t st) {
  // twiddles per distinct length
  for (auto& kv : p->tw_off) {
    std::vector<double> tw;
    make_twiddles((int)kv.first, tw);
    std::vector<T> twt(tw.size());
    for (size_t i = 0; i < tw.size(); ++i) twt[i] = (T)tw[i];
    if (hipMemcpyAsync(p->d_tw() + kv.second * 2 * sizeof(T), twt.data(), twt.size() * sizeof(T),
                       hipMemcpyHostToDevice, st) != hipSuccess)
      return DT_E_HIP;
    if (hipMemcpyAsync(p->d_tw64() + p->tw64_off[kv.first] * 2, tw.data(), tw.size() * sizeof(double),
                       hipMemcpyHostToDevice, st) != hipSuccess)
      return DT_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
  }
  double* buf0 = (double*)p->d_A();
  double* buf1 = (double*)p->d_B();
  std::vector<double> part(kPartialsB);
  for (auto& g : p->geos) {
    TabGeom tg{};
    tg.ndim = 2;
    tg.M[0] = (int)g.Mx; tg.M[1] = (int)g.My; tg.M[2] = 1;
    tg.H[0] = (int)(g.Mx / 2 + 1); tg.H[1] = (int)(g.My / 2 + 1); tg.H[2] = 1;
    tg.h[0] = g.hx; tg.h[1] = g.hy; tg.h[2] = 1.0;
    tg.cut[0] = g.cut[0]; tg.cut[1] = g.cut[1]; tg.cut[2] = 0;
    for (int c = 0; c < p->C; ++c) {
      TabKernel kd{};
      kd.kind = c == 0 ? KER_F : KER_U;
      kd.i = c == 0 ? 0 : c - 1;
      kd.tau = g.tau;
      const int nbp = launch_tab_sample(kd, tg, buf0, p->d_part(), st);
      if (hipMemcpyAsync(part.data(), p->d_part(), nbp * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
        return DT_E_HIP;
      if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
      double l1 = 0.0;
      for (int i = 0; i < nbp; ++i) l1 += part[i];
      if (c == 0) g.l1 = l1;
      g.e[c] = ceil_log2_d(l1);
      const int par[2] = {c == 1 ? 1 : 0, c == 2 ? 1 : 0};
      double* cur = buf0;
      double* nxt = buf1;
      for (int a = 0; a < 2; ++a) {
        const int64_t M = a == 0 ? g.Mx : g.My;
        launch_tab_axis(tg, a, par[a], p->d_tw64() + p->tw64_off[M] * 2, cur, nxt, st);
        std::swap(cur, nxt);
      }
      const double scale = std::ldexp(1.0, -g.e[c]) / ((double)g.Mx * (double)g.My);
      T* dst = (T*)p->d_tab() + g.tab_off + (int64_t)c * (g.My / 2 + 1) * g.pitch;
      launch_tab_store<T>(tg, cur, scale, dst, (int)g.pitch, 1, st);
    }
    if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
  }
  // per-instance scalars that depend on the tables
  for (int i = 0; i < p->n; ++i) {
    const auto& g = p->geos[p->geo_of[i]];
    BatchInst& I = p->inst[i];
    const double np = (double)g.Mx * (double)g.My;
    I.theta_coef = p->c_theta * p->unit() * std::log2(np) * g.l1 / std::sqrt(np);
    I.e_f = g.e[0];
    I.e_u[0] = p->C > 1 ? g.e[1] : 0;
    I.e_u[1] = p->C > 1 ? g.e[2] : 0;
    logf("batch plan %p inst %d: ||f||_1 = %.9g; one source: Theta = %.4g, S_max = %.3f tau", (void*)p, i, g.l1,
         I.theta_coef, -std::log(I.theta_coef));
  }
  if (hipMemcpyAsync(p->d_inst(), p->inst.data(), p->inst.size() * sizeof(BatchInst), hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return DT_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
  return hip_st(hipGetLastError());
}

// Radix schedules of every instance and pass from p->sched; the descriptors
// are uploaded again once the workspace is attached.
dt_status apply_schedule(dt_batch_plan p, hipStream_t st) {
  for (int i = 0; i < p->n; ++i) {
    BatchInst& I = p->inst[i];
    if (!mixed_plan_for(I.sx, p->sched[3 * i + P_R2C], I.px) || !mixed_plan_for(I.My, p->sched[3 * i + P_COL], I.py) ||
        !mixed_plan_for(I.sx, p->sched[3 * i + P_EPI], I.pxi))
      return DT_E_ARG;
  }
  if (p->ready) {
    if (hipMemcpyAsync(p->d_inst(), p->inst.data(), p->inst.size() * sizeof(BatchInst), hipMemcpyHostToDevice,
                       st) != hipSuccess)
      return DT_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
    p->drop_graph();
  }
  return DT_OK;
}

BatchArgs base_args(dt_batch_plan p) {
  BatchArgs a{};
  a.inst = p->d_inst();
  a.n_inst = p->n;
  a.koff = p->d_koff();
  a.scal = p->d_scal();
  a.err = p->d_err();
  a.tw = p->d_tw();
  a.tab = p->d_tab();
  a.C = p->C;
  return a;
}

// One pass alone over the current block list (the autotuner's timing unit;
// its input is whatever the buffers hold).
template <typename T> dt_status enqueue_pass(dt_batch_plan p, int k, void* S, void* grad, hipStream_t st) {
  BatchArgs a = base_args(p);
  a.blocks = p->d_blk(k);
  bool ok = false;
  if (k == P_R2C) {
    a.in = p->d_A();
    a.out = p->d_B();
    ok = launch_batch_row_r2c<T>(a, p->nblk[k], p->tiles.row_threads, p->ecap[k], p->lds[k], st);
  } else if (k == P_COL) {
    a.in = p->d_B();
    a.out = p->d_A();
    ok = launch_batch_col_fused<T>(a, p->nblk[k], p->tiles.col_threads, p->ecap[k], p->lds[k], st);
  } else {
    a.in = p->d_A();
    a.S = S;
    a.grad = grad;
    ok = launch_batch_row_c2r_epi<T>(a, p->nblk[k], p->tiles.row_threads, p->ecap[k], p->lds[k], st);
  }
  return ok ? hip_st(hipGetLastError()) : DT_E_UNSUPPORTED;
}

template <typename T> dt_status enqueue_forward(dt_batch_plan p, const float* Y, int64_t K_total, void* S,
                                                void* grad, hipStream_t st) {
  BatchArgs a = base_args(p);
  T* img = (T*)p->d_A();
  launch_fill_zero<T>(img, p->n_img, st);
  launch_fill_zero<double>(p->d_scal(), 4 * (int64_t)p->n, st);
  launch_batch_splat<T>(Y, K_total, a, img, st);
  launch_batch_finalize(a, st);
  a.blocks = p->d_blk(P_R2C);
  a.in = p->d_A();
  a.out = p->d_B();
  if (!launch_batch_row_r2c<T>(a, p->nblk[P_R2C], p->tiles.row_threads, p->ecap[P_R2C], p->lds[P_R2C], st))
    return DT_E_UNSUPPORTED;
  a.blocks = p->d_blk(P_COL);
  a.in = p->d_B();
  a.out = p->d_A();
  if (!launch_batch_col_fused<T>(a, p->nblk[P_COL], p->tiles.col_threads, p->ecap[P_COL], p->lds[P_COL], st))
    return DT_E_UNSUPPORTED;
  a.blocks = p->d_blk(P_EPI);
  a.in = p->d_A();
  a.out = nullptr;
  a.S = S;
  a.grad = grad;
  if (!launch_batch_row_c2r_epi<T>(a, p->nblk[P_EPI], p->tiles.row_threads, p->ecap[P_EPI], p->lds[P_EPI], st))
    return DT_E_UNSUPPORTED;
  return hip_st(hipGetLastError());
}

dt_status enqueue(dt_batch_plan p, const float* Y, int64_t K_total, void* S, void* grad, hipStream_t st) {
  return p->fp64 ? enqueue_forward<double>(p, Y, K_total, S, grad, st)
                 : enqueue_forward<float>(p, Y, K_total, S, grad, st);
}

// Validate and upload the source offsets (only when they changed).
dt_status prepare_call(dt_batch_plan p, const float* Y, const int64_t* K_offsets, void* S, void* grad,
                       hipStream_t st, int64_t& K_total) {
  if (!p->ready) return DT_E_WORKSPACE;
  if (!K_offsets) return DT_E_ARG;
  if (K_offsets[0] != 0) return DT_E_ARG;
  for (int i = 0; i < p->n; ++i)
    if (K_offsets[i + 1] < K_offsets[i]) return DT_E_ARG;
  for (int i = 0; i < p->n; ++i)   // reduced padding holds for at most k_max sources
    if (p->desc[i].k_max > 0 && K_offsets[i + 1] - K_offsets[i] > p->desc[i].k_max) return DT_E_ARG;
  K_total = K_offsets[p->n];
  if (K_total > 0 && !Y) return DT_E_ARG;
  if (K_total >= ((int64_t)1 << 31) * 256) return DT_E_UNSUPPORTED;
  if ((p->mask & DT_OUT_S) && !S) return DT_E_ARG;
  if ((p->mask & DT_OUT_GRAD) && !grad) return DT_E_ARG;
  if (!S && !grad) return DT_E_ARG;
  if (!p->blocks_valid) {
    const dt_status s = build_blocks(p, st);
    if (s != DT_OK) return s;
  }
  if (!p->koff_valid || !std::equal(p->koff.begin(), p->koff.end(), K_offsets)) {
    p->koff.assign(K_offsets, K_offsets + p->n + 1);
    if (hipMemcpyAsync(p->d_koff(), p->koff.data(), p->koff.size() * sizeof(int64_t), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return DT_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return DT_E_HIP;
    p->koff_valid = true;
    ++p->version;
  }
  return DT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" dt_status dt_create_batch_plan(dt_batch_plan* out, int n_inst, const dt_instance_desc* d, int precision,
                                          unsigned out_mask, double c_theta) {
  if (!out) return DT_E_ARG;
  *out = nullptr;
  if (n_inst < 1 || !d) return DT_E_ARG;
  if (precision != DT_FP32_SCALED && precision != DT_FP64) return DT_E_ARG;
  if (out_mask == 0 || (out_mask & ~(unsigned)(DT_OUT_S | DT_OUT_GRAD))) return DT_E_ARG;
  if (!(c_theta <= 0) && !finite_pos_b(c_theta)) return DT_E_ARG;
  for (int i = 0; i < n_inst; ++i) {
    const dt_instance_desc& q = d[i];
    if (!finite_pos_b(q.tau)) return DT_E_ARG;
    if (q.k_max < 0) return DT_E_ARG;
    for (int a = 0; a < 2; ++a) {
      if (q.dims[a] < 2) return DT_E_ARG;
      if (!finite_pos_b(q.spacing[a]) || !std::isfinite(q.origin[a])) return DT_E_ARG;
      if (q.dims[a] > 1024) return DT_E_UNSUPPORTED;
    }
  }
  dt_batch_plan p = new (std::nothrow) dt_batch_plan_s();
  if (!p) return DT_E_ARG;
  p->n = n_inst;
  p->fp64 = precision == DT_FP64;
  p->mask = out_mask;
  p->C = (out_mask & DT_OUT_GRAD) ? kBatchChan : 1;
  p->c_theta = c_theta > 0 ? c_theta : 256.0;
  p->desc.assign(d, d + n_inst);
  p->inst.resize(n_inst);
  p->geo_of.resize(n_inst);
  std::map<std::tuple<int64_t, int64_t, double, double, double, int, int>, int> geo_index;
  int64_t img = 0, spec = 0, outo = 0, tab = 0, scratch = 0, cols = 0, rows = 0;
  for (int i = 0; i < n_inst; ++i) {
    const dt_instance_desc& q = d[i];
    BatchInst& I = p->inst[i];
    std::memset(&I, 0, sizeof(I));
    I.nx = (int)q.dims[0];
    I.ny = (int)q.dims[1];
    int64_t sx = smooth7_at_least(q.dims[0]);
    int64_t My = 2 * smooth7_at_least(q.dims[1]);
    int cut[2] = {0, 0};
    if (q.k_max > 0) {
      // Reduced padding: a call with K <= k_max sources in the instance has
      // Theta >= sqrt(K) Theta_low, Theta_low the validity threshold of one
      // source on the full padding (||g||_2 >= sqrt(K) for integer
      // multiplicities, ||f||_1 >= f(0) = 1, log2(N)/sqrt(N) falls with N);
      // the truncation distance then keeps the K dropped tails below
      // sqrt(K) Theta_low / c_theta <= Theta / c_theta.
      const double np_full = (double)(2 * sx) * (double)My;
      const double theta_low = p->c_theta * (p->fp64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24)) *
                               std::log2(np_full) / std::sqrt(np_full);
      const double d_cut = q.tau * (std::log(p->c_theta * std::sqrt((double)q.k_max)) - std::log(theta_low));
      for (int a = 0; a < 2; ++a) {
        const double c = std::ceil(d_cut / q.spacing[a]);
        cut[a] = c < 1e9 ? (int)c : 1000000000;
      }
      // an axis whose box reaches n cells cannot gain: full padding, no truncation
      const int64_t sx_r = cut[0] < q.dims[0] ? smooth7_at_least((q.dims[0] + cut[0] + 1) / 2) : sx;
      const int64_t my_r = cut[1] < q.dims[1] ? 2 * smooth7_at_least((q.dims[1] + cut[1] + 1) / 2) : My;
      if (sx_r < sx) sx = sx_r; else cut[0] = 0;
      if (my_r < My) My = my_r; else cut[1] = 0;
    }
    I.sx = (int)sx;
    I.My = (int)My;
    I.pitch = (int)((sx + 1 + 15) / 16 * 16);
    I.ox = q.origin[0]; I.oy = q.origin[1];
    I.hx = q.spacing[0]; I.hy = q.spacing[1];
    I.tau = q.tau;
    if (!mixed_plan_for(sx, kDefaultFamily, I.px) || !mixed_plan_for(My, kDefaultFamily, I.py) ||
        !mixed_plan_for(sx, kDefaultFamily, I.pxi)) {
      delete p;
      return DT_E_UNSUPPORTED;
    }
    p->sched.insert(p->sched.end(), {kDefaultFamily, kDefaultFamily, kDefaultFamily});
    I.m_sx = fastdiv_magic((uint32_t)sx);
    I.m_sx1 = fastdiv_magic((uint32_t)(sx + 1));
    I.m_nx = fastdiv_magic((uint32_t)I.nx);
    I.img_off = img;
    img += (int64_t)I.nx * I.ny;
    I.spec_off = spec;
    spec += (int64_t)I.ny * I.pitch;
    I.out_off = outo;
    outo += (int64_t)I.nx * I.ny;
    for (int64_t M : {2 * sx, My}) {
      if (!p->tw_off.count(M)) {
        p->tw_off[M] = p->n_tw;
        p->n_tw += M;
        p->tw64_off[M] = p->n_tw64;
        p->n_tw64 += M;
      }
    }
    I.twx_off = p->tw_off[2 * sx];
    I.twy_off = p->tw_off[My];
    const auto key = std::make_tuple(2 * sx, My, q.spacing[0], q.spacing[1], q.tau, cut[0], cut[1]);
    auto it = geo_index.find(key);
    if (it == geo_index.end()) {
      dt_batch_plan_s::Geo g{};
      g.Mx = 2 * sx; g.My = My; g.pitch = I.pitch;
      g.cut[0] = cut[0]; g.cut[1] = cut[1];
      g.hx = q.spacing[0]; g.hy = q.spacing[1]; g.tau = q.tau;
      g.tab_off = tab;
      tab += (int64_t)p->C * (My / 2 + 1) * I.pitch;
      scratch = std::max<int64_t>(scratch, (sx + 1) * (My / 2 + 1));
      p->geos.push_back(g);
      it = geo_index.emplace(key, (int)p->geos.size() - 1).first;
    }
    p->geo_of[i] = it->second;
    I.tab_off = p->geos[it->second].tab_off;
    I.tab_stride = (int64_t)(My / 2 + 1) * I.pitch;
    rows += I.ny;
    cols += sx + 1;
  }
  // the column-pass outputs follow the same per-instance order
  int64_t fused = 0;
  for (int i = 0; i < n_inst; ++i) {
    p->inst[i].fused_off = fused;
    fused += (int64_t)p->C * p->inst[i].ny * p->inst[i].pitch;
  }
  p->n_img = img;
  p->n_spec = spec;
  p->n_fused = fused;
  p->n_tab = tab;
  p->n_scratch = scratch;
  p->total_nodes = outo;
  p->blk_cap[P_R2C] = rows;
  p->blk_cap[P_COL] = cols;
  p->blk_cap[P_EPI] = rows;
  const size_t w = p->wsz();
  size_t off = 0;
  p->off_inst = off; off = align_b(off + (size_t)n_inst * sizeof(BatchInst));
  for (int k = 0; k < 3; ++k) { p->off_blk[k] = off; off = align_b(off + (size_t)p->blk_cap[k] * sizeof(BatchBlock)); }
  p->off_koff = off; off = align_b(off + (size_t)(n_inst + 1) * sizeof(int64_t));
  p->off_scal = off; off = align_b(off + (size_t)4 * n_inst * sizeof(double));
  p->off_err = off; off = align_b(off + sizeof(uint64_t));
  p->off_part = off; off = align_b(off + kPartialsB * sizeof(double));
  p->off_tw = off; off = align_b(off + (size_t)p->n_tw * 2 * w);
  p->off_tw64 = off; off = align_b(off + (size_t)p->n_tw64 * 2 * sizeof(double));
  p->off_tab = off; off = align_b(off + (size_t)p->n_tab * w);
  const size_t a_bytes = std::max({(size_t)img * w, (size_t)fused * 2 * w, (size_t)scratch * sizeof(double)});
  const size_t b_bytes = std::max((size_t)spec * 2 * w, (size_t)scratch * sizeof(double));
  p->off_A = off; off = align_b(off + a_bytes);
  p->off_B = off; off = align_b(off + b_bytes);
  p->ws_bytes = off;
  if (log_enabled()) {
    char mb[64];
    logf("batch plan %p created: %d 2D instances, precision %s, outputs %s, c_theta = %g, workspace %.1f MB",
         (void*)p, n_inst, precision_name(precision), mask_names(out_mask, mb, sizeof(mb)), p->c_theta,
         p->ws_bytes / 1e6);
    for (int i = 0; i < n_inst; ++i) {
      const BatchInst& I = p->inst[i];
      const auto& g = p->geos[p->geo_of[i]];
      logf("  inst %d: grid %dx%d, h = %.6g %.6g, tau = %.6g, padded %lldx%lld, kernels truncated to %dx%d cells "
           "(0: none), k_max %lld",
           i, I.nx, I.ny, I.hx, I.hy, I.tau, (long long)g.Mx, (long long)g.My, g.cut[0], g.cut[1],
           (long long)d[i].k_max);
    }
  }
  *out = p;
  return DT_OK;
}

extern "C" dt_status dt_batch_workspace_size(dt_batch_plan p, size_t* bytes) {
  if (!p || !bytes) return DT_E_ARG;
  *bytes = p->ws_bytes;
  return DT_OK;
}

extern "C" dt_status dt_batch_set_workspace(dt_batch_plan p, void* dev_ptr, size_t bytes, void* stream) {
  if (!p || !dev_ptr) return DT_E_ARG;
  if (bytes < p->ws_bytes || ((uintptr_t)dev_ptr % kAlignB) != 0) return DT_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  p->drop_graph();
  p->ws = (char*)dev_ptr;
  p->stream = st;
  p->ready = false;
  p->koff_valid = false;
  p->blocks_valid = false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DT_E_HIP;
  if (hipDeviceGetAttribute(&p->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return DT_E_HIP;
  const bool ok = p->fp64 ? batch_set_lds_limit<double>(p->lds_max) : batch_set_lds_limit<float>(p->lds_max);
  if (!ok) p->lds_max = 65536;
  launch_fill_zero<double>((double*)p->ws, (int64_t)(p->off_tw / sizeof(double)), st);
  const dt_status s = p->fp64 ? build_batch_tables<double>(p, st) : build_batch_tables<float>(p, st);
  if (s != DT_OK) return s;
  p->ready = true;
  if (!p->tiles_set) p->tiles = default_tiles(p);
  return build_blocks(p, st);
}

extern "C" dt_status dt_batch_instance_info(dt_batch_plan p, int i, dt_batch_instance_info_t* info) {
  if (!p || !info || i < 0 || i >= p->n) return DT_E_ARG;
  const BatchInst& I = p->inst[i];
  info->padded[0] = 2 * (int64_t)I.sx;
  info->padded[1] = I.My;
  info->node_offset = I.out_off;
  info->total_nodes = p->total_nodes;
  info->precision = p->fp64 ? DT_FP64 : DT_FP32_SCALED;
  const auto& g = p->geos[p->geo_of[i]];
  info->kernel_l1 = g.l1;
  return DT_OK;
}

extern "C" dt_status dt_batch_set_tiles(dt_batch_plan p, const dt_batch_tiles* t) {
  if (!p || !t) return DT_E_ARG;
  const dt_batch_tiles old = p->tiles;
  p->tiles = *t;
  p->tiles_set = true;
  if (p->ready) {
    const dt_status s = build_blocks(p, p->stream);
    if (s != DT_OK) {
      p->tiles = old;
      (void)build_blocks(p, p->stream);
      return s;
    }
  } else {
    p->blocks_valid = false;
  }
  return DT_OK;
}

extern "C" dt_status dt_batch_get_tiles(dt_batch_plan p, dt_batch_tiles* t) {
  if (!p || !t) return DT_E_ARG;
  *t = p->tiles;
  return DT_OK;
}

extern "C" dt_status dt_batch_set_graph(dt_batch_plan p, int enable) {
  if (!p) return DT_E_ARG;
  p->use_graph = enable != 0;
  if (!p->use_graph) p->drop_graph();
  return DT_OK;
}

extern "C" dt_status dt_forward_batched(dt_batch_plan p, const float* Y, const int64_t* K_offsets, void* S,
                                        void* grad, void* stream) {
  if (!p) return DT_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  int64_t K_total = 0;
  dt_status s = prepare_call(p, Y, K_offsets, S, grad, st, K_total);
  if (s != DT_OK) return s;
  if (!(p->mask & DT_OUT_S)) S = nullptr;
  if (!(p->mask & DT_OUT_GRAD)) grad = nullptr;
  if (!p->use_graph) return enqueue(p, Y, K_total, S, grad, st);
  if (!(p->exec && p->g_version == p->version && p->g_Y == Y && p->g_S == S && p->g_grad == grad)) {
    p->drop_graph();
    if (!p->cap_stream && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return DT_E_HIP;
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return DT_E_HIP;
    s = enqueue(p, Y, K_total, S, grad, p->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->cap_stream, &g);
    if (s != DT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (ec != hipSuccess || !g) return DT_E_HIP;
    const hipError_t ei = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      p->exec = nullptr;
      return DT_E_HIP;
    }
    p->g_version = p->version;
    p->g_Y = Y;
    p->g_S = S;
    p->g_grad = grad;
  }
  return hip_st(hipGraphLaunch(p->exec, st));
}

extern "C" dt_status dt_batch_autotune(dt_batch_plan p, const float* Y, const int64_t* K_offsets, void* S,
                                       void* grad, int reps, void* stream, dt_batch_tiles* best) {
  if (!p || reps < 1) return DT_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  int64_t K_total = 0;
  dt_status s = prepare_call(p, Y, K_offsets, S, grad, st, K_total);
  if (s != DT_OK) return s;
  if (!(p->mask & DT_OUT_S)) S = nullptr;
  if (!(p->mask & DT_OUT_GRAD)) grad = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return DT_E_HIP;
  auto time_cfg = [&](const dt_batch_tiles& t, float& ms) -> bool {
    p->tiles = t;
    if (build_blocks(p, st) != DT_OK) return false;
    if (enqueue(p, Y, K_total, S, grad, st) != DT_OK) return false;   // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r)
      if (enqueue(p, Y, K_total, S, grad, st) != DT_OK) return false;
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) return false;
    return hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  };
  dt_batch_tiles cur = p->tiles, win = p->tiles;
  float best_ms = 1e30f;
  {
    float ms;
    if (time_cfg(cur, ms)) best_ms = ms;
  }
  // column pass first (tile width and threads), then the row passes
  auto sweep_tiles = [&]() {
    for (int nb : {2, 4, 8, 16, 32})
      for (int nt : {128, 256, 512, 1024}) {
        dt_batch_tiles t = win;
        t.col_nb = nb;
        t.col_threads = nt;
        float ms;
        if (time_cfg(t, ms) && ms < best_ms) { best_ms = ms; win = t; }
      }
    for (int nt : {128, 256, 512}) {
      dt_batch_tiles t = win;
      t.row_threads = nt;
      float ms;
      if (time_cfg(t, ms) && ms < best_ms) { best_ms = ms; win = t; }
    }
    p->tiles = win;
  };
  sweep_tiles();
  // Radix schedule per (pass, length): every candidate schedule of a length
  // is timed on that pass alone over the instances of that length.
  auto time_pass = [&](int k, float& ms) -> bool {
    const bool f64 = p->fp64;
    auto run = [&]() { return f64 ? enqueue_pass<double>(p, k, S, grad, st) : enqueue_pass<float>(p, k, S, grad, st); };
    if (run() != DT_OK) return false;   // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r)
      if (run() != DT_OK) return false;
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) return false;
    return hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  };
  for (int k : {P_R2C, P_COL, P_EPI}) {
    std::map<int64_t, std::vector<int>> by_len;
    for (int i = 0; i < p->n; ++i) by_len[k == P_COL ? p->inst[i].My : p->inst[i].sx].push_back(i);
    for (const auto& kv : by_len) {
      std::vector<char> keep(p->n, 0);
      for (int i : kv.second) keep[i] = 1;
      int best_f = p->sched[3 * kv.second[0] + k];
      float best_k = 1e30f;
      std::vector<MixedPlan> seen;
      for (int f = 0; f < kMixedFamilies; ++f) {
        MixedPlan mp;
        if (!mixed_plan_for(kv.first, f, mp)) continue;
        bool dup = false;
        for (const auto& q : seen) dup = dup || same_plan(q, mp);
        if (dup) continue;
        seen.push_back(mp);
        for (int i : kv.second) p->sched[3 * i + k] = f;
        float ms;
        if (apply_schedule(p, st) == DT_OK && build_blocks(p, st, &keep) == DT_OK && time_pass(k, ms) &&
            ms < best_k) {
          best_k = ms;
          best_f = f;
        }
      }
      for (int i : kv.second) p->sched[3 * i + k] = best_f;
    }
  }
  // the tiles again, under the chosen schedules (the best tiles depend on them)
  s = apply_schedule(p, st);
  if (s == DT_OK) {
    float ms;
    best_ms = time_cfg(win, ms) ? ms : 1e30f;
    sweep_tiles();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGetLastError();
  s = apply_schedule(p, st);
  if (s != DT_OK) return s;
  s = build_blocks(p, st);
  if (s != DT_OK) return s;
  if (best) *best = win;
  return DT_OK;
}

extern "C" dt_status dt_batch_set_schedule(dt_batch_plan p, const int* fams) {
  if (!p || !fams) return DT_E_ARG;
  for (int i = 0; i < 3 * p->n; ++i)
    if (fams[i] < 0 || fams[i] >= kMixedFamilies) return DT_E_ARG;
  const std::vector<int> old = p->sched;
  std::copy(fams, fams + 3 * p->n, p->sched.begin());
  const dt_status s = apply_schedule(p, p->stream);
  if (s != DT_OK) {
    p->sched = old;
    (void)apply_schedule(p, p->stream);
  }
  return s;
}

extern "C" dt_status dt_batch_get_schedule(dt_batch_plan p, int* fams) {
  if (!p || !fams) return DT_E_ARG;
  for (int i = 0; i < 3 * p->n; ++i) fams[i] = p->sched[i];
  return DT_OK;
}

extern "C" dt_status dt_batch_last_error(dt_batch_plan p) {
  if (!p || !p->ready) return DT_E_ARG;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return DT_E_HIP;
  uint32_t e = 0;
  if (hipMemcpy(&e, p->d_err(), sizeof(e), hipMemcpyDeviceToHost) != hipSuccess) return DT_E_HIP;
  if (e) {
    launch_fill_zero<float>((float*)p->d_err(), 1, p->stream);
    if (hipStreamSynchronize(p->stream) != hipSuccess) return DT_E_HIP;
  }
  return e ? DT_E_RANGE : DT_OK;
}

extern "C" dt_status dt_batch_stats(dt_batch_plan p, int i, dt_call_stats* out) {
  if (!p || !out || !p->ready || i < 0 || i >= p->n) return DT_E_ARG;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return DT_E_HIP;
  double s[4];
  if (hipMemcpy(s, p->d_scal() + 4 * i, sizeof(s), hipMemcpyDeviceToHost) != hipSuccess) return DT_E_HIP;
  std::memset(out, 0, sizeof(*out));
  out->theta = s[0];
  out->s_max = s[1];
  out->g_l2 = s[2];
  logf("batch plan %p inst %d last call: ||g||_2 = %.6g, Theta = %.4g, S_max = %.3f tau", (void*)p, i, out->g_l2,
       out->theta, out->s_max / p->inst[i].tau);
  return DT_OK;
}

extern "C" dt_status dt_destroy_batch_plan(dt_batch_plan p) {
  if (!p) return DT_E_ARG;
  p->drop_graph();
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
  return DT_OK;
}
