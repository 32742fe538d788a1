// Host-only checks of libdt's C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_host_asan.py compiles the library's
// host code and this driver without device code and runs it on the CPU).
//
// Every path exercised here returns before any device call: plan creation
// and validation, the workspace layout, the reduced-padding rule, the batched
// plan's instance table, padding and radix schedules, and the refusals of
// compute calls that have no workspace.  Random arguments come from a seeded
// splitmix64 stream; each check prints the failing case and exits nonzero.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "dt.h"

namespace {

uint64_t g_state = 0x1112301000000001ull;
uint64_t next_u64() {
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }
double unit() { return (double)(next_u64() >> 11) * 0x1.0p-53; }
int64_t log_uniform(int64_t lo, int64_t hi) {
  const double v = std::exp(std::log((double)lo) + unit() * (std::log((double)hi + 1) - std::log((double)lo)));
  return std::min<int64_t>(hi, std::max<int64_t>(lo, (int64_t)v));
}

int g_fail = 0;
#define CHECK(cond, ...)                                          \
  do {                                                            \
    if (!(cond)) {                                                \
      std::fprintf(stderr, "FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond); \
      std::fprintf(stderr, __VA_ARGS__);                          \
      std::fprintf(stderr, "\n");                                 \
      if (++g_fail > 20) std::exit(1);                            \
    }                                                             \
  } while (0)

bool is_pow2(int64_t m) { return m > 0 && (m & (m - 1)) == 0; }
bool is_smooth7(int64_t m) {
  for (int p : {2, 3, 5, 7})
    while (m % p == 0) m /= p;
  return m == 1;
}

const double kNaN = std::numeric_limits<double>::quiet_NaN();
const double kInf = std::numeric_limits<double>::infinity();

// ---------------------------------------------------------------------------
// Single plans
// ---------------------------------------------------------------------------
void check_plan(dt_plan p, int ndim, const int64_t* dims, int64_t k_max, int prec_req) {
  dt_plan_info_t info;
  CHECK(dt_plan_info(p, &info) == DT_OK, "info");
  CHECK(info.ndim == ndim, "ndim %d", info.ndim);
  CHECK(info.k_max == k_max, "k_max %lld", (long long)info.k_max);
  if (prec_req != DT_AUTO) CHECK(info.precision == prec_req, "precision %d vs %d", info.precision, prec_req);
  for (int a = 0; a < ndim; ++a) {
    const int64_t n = dims[a], M = info.padded[a], c = info.cut[a];
    CHECK(info.dims[a] == n, "dims");
    if (k_max == 0 || c == 0) {
      // full padding: the smallest power of two >= max(64, 2n)
      CHECK(is_pow2(M) && M >= 2 * n && M >= 64 && (M == 64 || M / 2 < 2 * n), "axis %d n %lld M %lld", a,
            (long long)n, (long long)M);
      CHECK(c == 0, "cut without reduction");
    } else {
      // reduced: an engine length that holds n + c and is below the full padding
      CHECK(is_pow2(M) || M == 288 || M == 392, "reduced length %lld", (long long)M);
      CHECK(M >= n + c && M >= 64, "axis %d n %lld c %lld M %lld", a, (long long)n, (long long)c, (long long)M);
      int64_t full = 64;
      while (full < 2 * n) full *= 2;
      CHECK(M < full, "reduced %lld not below full %lld", (long long)M, (long long)full);
    }
  }
  for (int a = ndim; a < 3; ++a) CHECK(info.padded[a] == 1 && info.dims[a] == 1, "unused axis");
  size_t ws = 0;
  CHECK(dt_plan_workspace_size(p, &ws) == DT_OK && ws == info.workspace_bytes, "workspace size");
  CHECK(ws > 0 && ws % 256 == 0, "workspace %zu", ws);
  CHECK(info.n_tables >= 0 && info.n_tables <= 16, "tables %d", info.n_tables);
  // compute calls without a workspace, and with bad arguments
  float dummy[6] = {0};
  CHECK(dt_distance(p, dummy, 1, dummy, nullptr) != DT_OK, "distance without workspace");
  CHECK(dt_distance(p, dummy, 0, dummy, nullptr) == DT_E_ARG, "K = 0");
  CHECK(dt_distance(p, nullptr, 3, dummy, nullptr) == DT_E_ARG, "Y = NULL");
  CHECK(dt_backward(p, dummy, 0, dummy, dummy, dummy, nullptr, nullptr) == DT_E_ARG, "backward K = 0");
  CHECK(dt_last_error(p) == DT_E_WORKSPACE, "last_error without workspace");
  dt_call_stats cs;
  CHECK(dt_last_stats(p, &cs) == DT_E_WORKSPACE, "stats without workspace");
  CHECK(dt_plan_set_workspace(p, nullptr, ws, nullptr) == DT_E_ARG, "null workspace");
  CHECK(dt_plan_set_workspace(p, (void*)(uintptr_t)4096, ws - 1, nullptr) == DT_E_WORKSPACE, "short workspace");
  CHECK(dt_plan_set_workspace(p, (void*)(uintptr_t)(4096 + 64), ws, nullptr) == DT_E_WORKSPACE, "misaligned");
  CHECK(dt_plan_set_timing(p, 1) == DT_OK && dt_plan_set_timing(p, 0) == DT_OK, "timing switch");
  int n_ent = -1;
  dt_pass_timing tim[4];
  CHECK(dt_plan_timings(p, tim, 4, &n_ent) == DT_OK && n_ent == 0, "no timings yet (%d)", n_ent);
}

void plans_random(int count) {
  static const unsigned masks[] = {DT_OUT_S, DT_OUT_GRAD, DT_OUT_S | DT_OUT_GRAD, DT_OUT_HESS, DT_OUT_SIGN,
                                   DT_OUT_S | DT_OUT_SIGN, DT_OUT_BACKWARD, DT_OUT_CURV, 63u};
  int made = 0;
  for (int it = 0; it < count; ++it) {
    const int ndim = (int)uniform(2, 3);
    int64_t dims[3];
    // 3D stays moderate: DT_AUTO estimates ||f||_1 on the host over M^3 / 8 nodes
    for (int a = 0; a < ndim; ++a) dims[a] = log_uniform(2, ndim == 3 ? 300 : 1024);
    double h[3], o[3];
    for (int a = 0; a < ndim; ++a) {
      h[a] = 1.0 / (double)dims[a] * (0.5 + unit());
      o[a] = unit() - 0.5;
    }
    const double tau = h[0] * (0.25 + 8 * unit());
    const int prec = (int)uniform(0, 4);
    const unsigned mask = masks[uniform(0, 8)];
    const bool reduced = uniform(0, 2) == 0;
    const int64_t k_max = reduced ? log_uniform(1, 1000000) : 0;
    const double c_theta = uniform(0, 3) == 0 ? 16 + 2048 * unit() : 0.0;
    dt_plan p = nullptr;
    dt_status st;
    if (reduced)
      st = dt_create_plan_reduced(&p, ndim, dims, h, o, tau, prec, mask, k_max, c_theta);
    else
      st = dt_create_plan(&p, ndim, dims, h, o, tau, prec, mask, tau * (2 + 30 * unit()), log_uniform(1, 100000),
                          c_theta);
    // what the header promises for these arguments
    if (reduced && (mask & DT_OUT_SIGN)) {
      CHECK(st == DT_E_UNSUPPORTED || st == DT_E_ARG, "reduced sign plan: %d", st);
    } else if (reduced && prec != DT_FP32_SCALED && prec != DT_FP64) {
      CHECK(st == DT_E_ARG, "reduced precision %d: %d", prec, st);
    } else if (prec == DT_FP64X2 || prec == DT_FP64X4) {
      bool ok = !(mask & DT_OUT_SIGN);
      const int64_t cap = prec == DT_FP64X4 ? 128 : 256;
      for (int a = 0; a < ndim && ndim == 3; ++a) ok = ok && dims[a] <= cap;
      CHECK(ok ? st == DT_OK : st == DT_E_UNSUPPORTED, "extended precision %d mask %u: %d", prec, mask, st);
    } else if (prec == DT_AUTO) {
      CHECK(st == DT_OK || st == DT_E_PRECISION, "auto: %d", st);
    } else {
      CHECK(st == DT_OK, "ndim %d dims %lld %lld prec %d mask %u reduced %d: %d", ndim, (long long)dims[0],
            (long long)dims[1], prec, mask, (int)reduced, st);
    }
    CHECK((st == DT_OK) == (p != nullptr), "handle on status %d", st);
    if (st != DT_OK) continue;
    ++made;
    check_plan(p, ndim, dims, reduced ? k_max : 0, prec);
    CHECK(dt_destroy_plan(p) == DT_OK, "destroy");
  }
  std::printf("single plans: %d of %d created and checked\n", made, count);
}

void plans_refused() {
  const int64_t d2[2] = {64, 48}, d3[3] = {32, 40, 24};
  const double h[3] = {0.01, 0.01, 0.01}, o[3] = {0, 0, 0};
  dt_plan p = nullptr;
  CHECK(dt_create_plan(nullptr, 2, d2, h, o, 0.02, 0, 1, 0, 0, 0) == DT_E_ARG, "null out");
  CHECK(dt_create_plan(&p, 1, d2, h, o, 0.02, 0, 1, 0, 0, 0) == DT_E_ARG && !p, "ndim 1");
  CHECK(dt_create_plan(&p, 4, d2, h, o, 0.02, 0, 1, 0, 0, 0) == DT_E_ARG && !p, "ndim 4");
  CHECK(dt_create_plan(&p, 2, nullptr, h, o, 0.02, 0, 1, 0, 0, 0) == DT_E_ARG, "null dims");
  CHECK(dt_create_plan(&p, 2, d2, nullptr, o, 0.02, 0, 1, 0, 0, 0) == DT_E_ARG, "null spacing");
  CHECK(dt_create_plan(&p, 2, d2, h, nullptr, 0.02, 0, 1, 0, 0, 0) == DT_E_ARG, "null origin");
  for (double tau : {0.0, -1.0, kNaN, kInf})
    CHECK(dt_create_plan(&p, 2, d2, h, o, tau, 0, 1, 0, 0, 0) == DT_E_ARG && !p, "tau %g", tau);
  for (int prec : {-1, 5, 99}) CHECK(dt_create_plan(&p, 2, d2, h, o, 0.02, prec, 1, 0, 0, 0) == DT_E_ARG, "prec");
  for (unsigned m : {0u, 64u, 128u | 1u}) CHECK(dt_create_plan(&p, 2, d2, h, o, 0.02, 0, m, 0, 0, 0) == DT_E_ARG, "mask");
  for (double c : {kNaN, kInf}) CHECK(dt_create_plan(&p, 2, d2, h, o, 0.02, 0, 1, 0, 0, c) == DT_E_ARG, "c_theta");
  const int64_t small[2] = {1, 48}, big[3] = {32, 1025, 24};
  CHECK(dt_create_plan(&p, 2, small, h, o, 0.02, 0, 1, 0, 0, 0) == DT_E_ARG, "n = 1");
  CHECK(dt_create_plan(&p, 3, big, h, o, 0.02, 0, 1, 0, 0, 0) == DT_E_UNSUPPORTED, "n > 1024");
  const double hbad[3] = {0.01, kNaN, 0.01}, obad[3] = {0, kInf, 0};
  CHECK(dt_create_plan(&p, 3, d3, hbad, o, 0.02, 0, 1, 0, 0, 0) == DT_E_ARG, "spacing NaN");
  CHECK(dt_create_plan(&p, 3, d3, h, obad, 0.02, 0, 1, 0, 0, 0) == DT_E_ARG, "origin inf");
  // DT_AUTO needs a finite truncation distance and k_hint >= 1
  CHECK(dt_create_plan(&p, 2, d2, h, o, 0.02, DT_AUTO, 1, kNaN, 10, 0) == DT_E_ARG, "auto trunc NaN");
  CHECK(dt_create_plan(&p, 2, d2, h, o, 0.02, DT_AUTO, 1, 0.1, 0, 0) == DT_E_ARG, "auto k_hint 0");
  CHECK(dt_create_plan_reduced(&p, 2, d2, h, o, 0.02, 0, 1, 0, 0) == DT_E_ARG, "k_max 0");
  CHECK(dt_create_plan_reduced(&p, 2, d2, h, o, 0.02, 0, 1, -5, 0) == DT_E_ARG, "k_max < 0");
  CHECK(dt_create_plan_reduced(&p, 2, d2, h, o, 0.02, 0, 1, INT64_MAX, 0) == DT_OK, "k_max huge");
  if (p) {
    dt_plan_info_t info;
    CHECK(dt_plan_info(p, &info) == DT_OK && info.padded[0] == 128 && info.cut[0] == 0, "huge k_max: full padding");
    CHECK(dt_destroy_plan(p) == DT_OK, "destroy");
    p = nullptr;
  }
  // calls on a null plan
  dt_plan_info_t info;
  size_t ws = 0;
  CHECK(dt_plan_info(nullptr, &info) == DT_E_ARG, "info null");
  CHECK(dt_plan_workspace_size(nullptr, &ws) == DT_E_ARG, "ws null");
  CHECK(dt_destroy_plan(nullptr) == DT_E_ARG, "destroy null");
  CHECK(dt_last_error(nullptr) == DT_E_ARG, "last_error null");
  CHECK(dt_plan_set_static_workspace(nullptr, nullptr) == DT_E_ARG, "static null");
  for (int s = -3; s < 12; ++s) {
    const char* m = dt_status_str((dt_status)s);
    CHECK(m != nullptr && std::strlen(m) > 0, "status string %d", s);
  }
}

// ---------------------------------------------------------------------------
// Batched plans
// ---------------------------------------------------------------------------
void batch_random(int count) {
  int made = 0;
  for (int it = 0; it < count; ++it) {
    const int n = (int)log_uniform(1, 200);
    std::vector<dt_instance_desc> d(n);
    bool any_bad = false, any_big = false;
    for (int i = 0; i < n; ++i) {
      auto& q = d[i];
      std::memset(&q, 0, sizeof(q));
      q.dims[0] = log_uniform(2, 1100);
      q.dims[1] = log_uniform(2, 1100);
      any_big = any_big || q.dims[0] > 1024 || q.dims[1] > 1024;
      q.spacing[0] = 1.0 / (double)q.dims[0];
      q.spacing[1] = 1.0 / (double)q.dims[1] * (0.5 + unit());
      q.origin[0] = unit();
      q.origin[1] = -unit();
      q.tau = q.spacing[0] * (0.5 + 4 * unit());
      q.k_max = uniform(0, 1) ? log_uniform(1, 50000) : 0;
      if (uniform(0, 60) == 0) {   // a bad instance
        q.tau = uniform(0, 1) ? -1.0 : kNaN;
        any_bad = true;
      }
    }
    const int prec = (int)uniform(0, 1);
    const unsigned mask = (unsigned)uniform(1, 3);
    dt_batch_plan p = nullptr;
    const dt_status st = dt_create_batch_plan(&p, n, d.data(), prec, mask, 0.0);
    if (any_bad) {
      CHECK(st == DT_E_ARG || (any_big && st == DT_E_UNSUPPORTED), "bad instance accepted: %d", st);
    } else if (any_big) {
      CHECK(st == DT_E_UNSUPPORTED, "n > 1024 accepted: %d", st);
    } else {
      CHECK(st == DT_OK, "batch of %d: %d", n, st);
    }
    CHECK((st == DT_OK) == (p != nullptr), "handle on status %d", st);
    if (st != DT_OK) continue;
    ++made;
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
      dt_batch_instance_info_t bi;
      CHECK(dt_batch_instance_info(p, i, &bi) == DT_OK, "instance info");
      CHECK(bi.node_offset == off, "offset of %d", i);
      off += d[i].dims[0] * d[i].dims[1];
      for (int a = 0; a < 2; ++a) {
        const int64_t M = bi.padded[a], nn = d[i].dims[a];
        CHECK(M % 2 == 0 && is_smooth7(M / 2), "length %lld", (long long)M);
        if (d[i].k_max == 0) {
          // full: twice the smallest 7-smooth length >= n
          CHECK(M >= 2 * nn, "full padding %lld for n %lld", (long long)M, (long long)nn);
          for (int64_t s = nn; s < M / 2; ++s) CHECK(!is_smooth7(s), "not the smallest: %lld", (long long)s);
        } else {
          CHECK(M >= nn, "reduced padding %lld for n %lld", (long long)M, (long long)nn);
        }
      }
      CHECK(bi.precision == prec, "precision");
    }
    dt_batch_instance_info_t bi;
    CHECK(dt_batch_instance_info(p, -1, &bi) == DT_E_ARG && dt_batch_instance_info(p, n, &bi) == DT_E_ARG,
          "instance index range");
    CHECK(dt_batch_instance_info(p, 0, &bi) == DT_OK && bi.total_nodes == off, "total nodes");
    size_t ws = 0;
    CHECK(dt_batch_workspace_size(p, &ws) == DT_OK && ws > 0 && ws % 256 == 0, "workspace %zu", ws);
    // radix schedules: default 4; out-of-range values change nothing
    std::vector<int> f(3 * n), g(3 * n);
    CHECK(dt_batch_get_schedule(p, f.data()) == DT_OK, "get schedule");
    for (int v : f) CHECK(v == 4, "default family %d", v);
    for (auto& v : g) v = (int)uniform(0, 5);
    CHECK(dt_batch_set_schedule(p, g.data()) == DT_OK, "set schedule");
    std::vector<int> h2(3 * n);
    CHECK(dt_batch_get_schedule(p, h2.data()) == DT_OK && h2 == g, "schedule round trip");
    std::vector<int> bad = g;
    bad[uniform(0, 3 * n - 1)] = uniform(0, 1) ? 6 : -1;
    CHECK(dt_batch_set_schedule(p, bad.data()) == DT_E_ARG, "bad family accepted");
    CHECK(dt_batch_get_schedule(p, h2.data()) == DT_OK && h2 == g, "schedule changed by a refused call");
    // tiles and graph switch before the workspace is attached
    dt_batch_tiles t{4, 256, 128}, t2{};
    CHECK(dt_batch_set_tiles(p, &t) == DT_OK, "set tiles");
    CHECK(dt_batch_get_tiles(p, &t2) == DT_OK && t2.col_nb == 4 && t2.col_threads == 256 && t2.row_threads == 128,
          "tiles round trip");
    CHECK(dt_batch_set_graph(p, 1) == DT_OK && dt_batch_set_graph(p, 0) == DT_OK, "graph switch");
    // calls without a workspace
    std::vector<int64_t> koff(n + 1, 0);
    float y[2] = {0.5f, 0.5f};
    CHECK(dt_forward_batched(p, y, koff.data(), y, y, nullptr) == DT_E_WORKSPACE, "forward without workspace");
    CHECK(dt_batch_set_workspace(p, (void*)(uintptr_t)4096, ws - 1, nullptr) == DT_E_WORKSPACE, "short ws");
    CHECK(dt_batch_set_workspace(p, nullptr, ws, nullptr) == DT_E_ARG, "null ws");
    dt_call_stats cs;
    CHECK(dt_batch_stats(p, 0, &cs) == DT_E_ARG, "stats before attach");
    CHECK(dt_destroy_batch_plan(p) == DT_OK, "destroy");
  }
  std::printf("batch plans: %d of %d created and checked\n", made, count);
}

void batch_refused() {
  dt_instance_desc q;
  std::memset(&q, 0, sizeof(q));
  q.dims[0] = 64;
  q.dims[1] = 40;
  q.spacing[0] = q.spacing[1] = 0.01;
  q.tau = 0.02;
  dt_batch_plan p = nullptr;
  CHECK(dt_create_batch_plan(nullptr, 1, &q, 0, 3, 0) == DT_E_ARG, "null out");
  CHECK(dt_create_batch_plan(&p, 0, &q, 0, 3, 0) == DT_E_ARG && !p, "no instances");
  CHECK(dt_create_batch_plan(&p, 1, nullptr, 0, 3, 0) == DT_E_ARG, "null desc");
  for (int prec : {(int)DT_AUTO, (int)DT_FP64X2, (int)DT_FP64X4, 9})
    CHECK(dt_create_batch_plan(&p, 1, &q, prec, 3, 0) == DT_E_ARG, "prec");
  for (unsigned m : {0u, (unsigned)DT_OUT_HESS, 7u}) CHECK(dt_create_batch_plan(&p, 1, &q, 0, m, 0) == DT_E_ARG, "mask");
  CHECK(dt_create_batch_plan(&p, 1, &q, 0, 3, kNaN) == DT_E_ARG, "c_theta NaN");
  q.dims[1] = 1;
  CHECK(dt_create_batch_plan(&p, 1, &q, 0, 3, 0) == DT_E_ARG, "n = 1");
  dt_batch_tiles t{};
  CHECK(dt_batch_get_tiles(nullptr, &t) == DT_E_ARG && dt_batch_set_graph(nullptr, 1) == DT_E_ARG, "null plan");
  CHECK(dt_destroy_batch_plan(nullptr) == DT_E_ARG, "destroy null");
}

}  // namespace

int main(int argc, char** argv) {
  const int n_single = argc > 1 ? std::atoi(argv[1]) : 3000;
  const int n_batch = argc > 2 ? std::atoi(argv[2]) : 300;
  plans_refused();
  batch_refused();
  plans_random(n_single);
  batch_random(n_batch);
  if (g_fail) {
    std::fprintf(stderr, "%d check(s) failed\n", g_fail);
    return 1;
  }
  std::printf("all host checks passed\n");
  return 0;
}
