// Column passes on the two-step register FFT engine (see fft_twostep.hpp):
// the strided C2C pass and the fused forward / kernel-spectrum product /
// inverse pass of the last axis (Sec. 3, Table 1 steps 3-5).  Used for the
// transform lengths whose register footprint fits; the Stockham kernels in
// k_fft.hip cover the rest.
#include "dt_launch.hpp"
#include <type_traits>

#include "fft_twostep.hpp"

namespace dt {

// Factorisation N = E * P per length and precision (0 = not provided).
template <typename T, bool FUSED> constexpr int twostep_E(int N) {
  if (sizeof(T) == 4) {
    if (FUSED) return N == 64 ? 8 : N == 128 ? 16 : N == 256 ? 16 : N == 512 ? 32 : 0;
    return N == 64 ? 8 : N == 128 ? 16 : N == 256 ? 16 : N == 512 ? 32 : N == 1024 ? 32 : 0;
  }
  // float64: a fused pass keeps two copies of the column in registers
  if (FUSED) return N == 64 ? 8 : N == 128 ? 16 : N == 256 ? 16 : 0;
  return N == 64 ? 8 : N == 128 ? 16 : N == 256 ? 16 : N == 512 ? 32 : 0;
}
template <typename T, bool FUSED = false> constexpr int twostep_NB() {
  return sizeof(T) == 4 ? (FUSED ? 8 : 16) : 8;
}

template <typename T, int N, int E, int NB, int DIR, bool HALF>
__global__ void __launch_bounds__((N / E) * NB) k_col2_c2c(const Cx<T>* __restrict__ in, Cx<T>* __restrict__ out,
                                                          ColParams p) {
  using V = Cx<T>;
  using TS = TwoStep<T, N, E, NB>;
  constexpr int P = TS::P;
  __shared__ V lds[TS::LDS];
  const int tid = threadIdx.x;
  const int b = tid % NB, pt = tid / NB;
  const int kx = blockIdx.x * NB + b;
  const bool active = kx < p.inner;
  const int kxs = active ? kx : 0;
  ThreadTwiddles<T, N, E> tw;
  tw.load((const V*)p.tw, pt);
  const int64_t in_line = p.in_line, out_line = p.out_line;
  const V* src = in + blockIdx.z * p.in_ch + (int64_t)blockIdx.y * p.in_outer + kxs;
  V* dst = out + blockIdx.z * p.out_ch + (int64_t)blockIdx.y * p.out_outer + kxs;
  V v[E];
  if constexpr (DIR > 0) {
    // natural input rows pt + P e (pruned), outputs in slot order
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = pt + P * e;
      if (HALF && e >= E / 2) v[e] = mk<V>(T(0), T(0));
      else v[e] = (active && n < p.n_in) ? src[(int64_t)n * in_line] : mk<V>(T(0), T(0));
    }
    TS::forward(v, lds, pt, b, tw);
    if (!active) return;
#pragma unroll
    for (int t = 0; t < E / P; ++t)
#pragma unroll
      for (int k2 = 0; k2 < P; ++k2) {
        const int k = TS::slot_index(pt, t, k2);
        if (k < p.n_out) dst[(int64_t)k * out_line] = v[t * P + k2];
      }
  } else {
    // inputs in slot order, natural output rows pt + P n2 (pruned)
#pragma unroll
    for (int t = 0; t < E / P; ++t)
#pragma unroll
      for (int k2 = 0; k2 < P; ++k2) {
        const int k = TS::slot_index(pt, t, k2);
        v[t * P + k2] = (active && k < p.n_in) ? src[(int64_t)k * in_line] : mk<V>(T(0), T(0));
      }
    TS::inverse(v, lds, pt, b, tw);
    if (!active) return;
#pragma unroll
    for (int n2 = 0; n2 < E; ++n2) {
      if (HALF && n2 >= E / 2) continue;
      const int n = pt + P * n2;
      if (n < p.n_out) dst[(int64_t)n * out_line] = v[n2];
    }
  }
}

// The same strided pass on the pair-split engine (N = 2 E^2).
template <typename T, int N, int NB, int DIR, bool HALF>
__global__ void __launch_bounds__(2 * pair_E(N) * NB) k_col2_c2c_pair(const Cx<T>* __restrict__ in,
                                                                     Cx<T>* __restrict__ out, ColParams p) {
  using V = Cx<T>;
  using ENG = PairFFT<T, N, NB>;
  constexpr int E = ENG::E, P = ENG::P;
  __shared__ __align__(16) T xch[ENG::LDS];
  const int tid = threadIdx.x;
  const int b = tid % NB, pt = tid / NB;
  const int kx = blockIdx.x * NB + b;
  const bool active = kx < p.inner;
  const int kxs = active ? kx : 0;
  typename ENG::Tw tw;
  tw.load((const V*)p.tw, pt);
  const V* src = in + blockIdx.z * p.in_ch + blockIdx.y * p.in_outer + kxs;
  V* dst = out + blockIdx.z * p.out_ch + blockIdx.y * p.out_outer + kxs;
  V v[E];
  if constexpr (DIR > 0) {
    // natural input rows pt + P e (pruned), outputs in slot order
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = pt + P * e;
      if (HALF && e >= E / 2) v[e] = mk<V>(T(0), T(0));
      else v[e] = (active && n < p.n_in) ? src[(int64_t)n * p.in_line] : mk<V>(T(0), T(0));
    }
    ENG::forward_split(v, xch, pt, b, tw);
    if (!active) return;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = ENG::slot(pt, j);
      if (k < p.n_out) dst[(int64_t)k * p.out_line] = v[j];
    }
  } else {
    // inputs in slot order, natural output rows pt + P n2 (pruned)
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = ENG::slot(pt, j);
      v[j] = (active && k < p.n_in) ? src[(int64_t)k * p.in_line] : mk<V>(T(0), T(0));
    }
    ENG::inverse_split(v, xch, pt, b, tw);
    if (!active) return;
#pragma unroll
    for (int n2 = 0; n2 < E; ++n2) {
      if (HALF && n2 >= E / 2) continue;
      const int n = pt + P * n2;
      if (n < p.n_out) dst[(int64_t)n * p.out_line] = v[n2];
    }
  }
}

template <typename T, int N, int E, int NB, bool HALF>
__global__ void __launch_bounds__((N / E) * NB) k_col2_fused(const Cx<T>* __restrict__ in, Cx<T>* __restrict__ out,
                                                            ColParams p, FusedSpec fs) {
  using V = Cx<T>;
  using TS = TwoStep<T, N, E, NB>;
  constexpr int P = TS::P;
  __shared__ V lds[TS::LDS];
  const int tid = threadIdx.x;
  const int b = tid % NB, pt = tid / NB;
  const int kx = blockIdx.x * NB + b;
  const bool active = kx < p.inner;
  const int kxs = active ? kx : 0;
  const int o = blockIdx.y;
  const bool o_neg = 2 * o > p.outer_len;
  const int of = o_neg ? p.outer_len - o : o;
  const FusedItem& IT = fs.items[blockIdx.z];
  const FusedGroup& G = fs.g[IT.group];
  ThreadTwiddles<T, N, E> tw;
  tw.load((const V*)p.tw, pt);

  auto load_fwd = [&](int ch, V* v) {
    const V* src = in + (int64_t)ch * p.in_ch + (int64_t)o * p.in_outer + kxs;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = pt + P * e;
      if (HALF && e >= E / 2) v[e] = mk<V>(T(0), T(0));
      else v[e] = (active && n < p.n_in) ? src[(int64_t)n * p.in_line] : mk<V>(T(0), T(0));
    }
    TS::forward(v, lds, pt, b, tw);
  };
  // kernel-spectrum values of table tab at this thread's slots (sign folded in)
  auto load_tab = [&](int tab, T* tv) {
    const TabRef& t = fs.tabs[tab];
    const T* base = (const T*)t.ptr + (int64_t)of * fs.tab_outer_stride + (int64_t)blockIdx.x * fs.tab_tile_stride + b;
    const bool flip_o = t.odd_outer && o_neg;
#pragma unroll
    for (int tt = 0; tt < E / P; ++tt)
#pragma unroll
      for (int k2 = 0; k2 < P; ++k2) {
        const int l = TS::slot_index(pt, tt, k2);
        const bool l_neg = 2 * l > N;
        const int lf = l_neg ? N - l : l;
        const T val = base[(int64_t)lf * fs.tab_line_stride];
        tv[tt * P + k2] = (flip_o != (t.odd_line && l_neg)) ? -val : val;
      }
  };
  auto times = [&](const T* tv, int phase, const V* v, V* res, bool accumulate) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const V prod = mul_mi_pow(cscale(v[e], tv[e]), phase);
      res[e] = accumulate ? cadd(res[e], prod) : prod;
    }
  };
  auto inv_store = [&](V* v, int ch) {
    TS::inverse(v, lds, pt, b, tw);
    if (!active) return;
    V* dst = out + (int64_t)ch * p.out_ch + (int64_t)o * p.out_outer + kx;
#pragma unroll
    for (int n2 = 0; n2 < E; ++n2) {
      if (HALF && n2 >= E / 2) continue;
      const int n = pt + P * n2;
      if (n < p.n_out) dst[(int64_t)n * p.out_line] = v[n2];
    }
  };

  if (G.mode == 0) {
    T tv[E];
    load_tab(G.tab[IT.c0], tv);       // issued before the forward transform
    V spec[E];
    load_fwd(G.in_ch[0], spec);
    for (int c = IT.c0; c < IT.c1; ++c) {
      V v[E];
      times(tv, fs.tabs[G.tab[c]].phase, spec, v, false);
      if (c + 1 < IT.c1) load_tab(G.tab[c + 1], tv);   // prefetch the next channel's table
      inv_store(v, G.out_ch[c]);
    }
  } else {
    V acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = mk<V>(T(0), T(0));
    for (int i = 0; i < G.n_in; ++i) {
      T tv[E];
      load_tab(G.tab[i], tv);
      V v[E];
      load_fwd(G.in_ch[i], v);
      times(tv, fs.tabs[G.tab[i]].phase, v, acc, true);
    }
    inv_store(acc, G.out_ch[0]);
  }
}

// 3D variant of the fused pass with the kernel tables staged in LDS.  The
// tables are stored tile-major, so the slice a block needs (all folded kz of
// one kx tile at one |ky|) is a contiguous run that is copied with 16-byte
// loads.  The block owns the column pair (ky, M_y - ky), which share the
// slice: every folded table entry then serves all four spectral points
// (+-ky, +-kz) from one read.  The transform engine ENG is PairFFT
// (one complex LDS exchange) or TwoStep (real and imaginary parts exchanged in
// two rounds through a real LDS buffer); the tables are staged kTabChunk
// channels at a time.  Per precision: float32 stages all four slices at once
// with one complex exchange and register twiddles (68 KB of LDS, two blocks
// per CU).  float64 stages one slice at a time, exchanges in two rounds and
// keeps the twiddles in LDS: 60 KB of LDS and at most 256 registers, so two
// blocks share a CU instead of one.
template <typename T> constexpr int tab_chunk() { return sizeof(T) == 8 ? 1 : 4; }
template <typename T> constexpr int fused_split() { return sizeof(T) == 8 ? 1 : 0; }
template <typename T> constexpr bool fused_twl() { return sizeof(T) == 8; }
// the float64 hint applies to the 512-point pair engine (the 256^3 grids)
template <typename T, int N> constexpr int fused_minwaves() { return sizeof(T) == 8 && (N == 512 || N == 392) ? 2 : 1; }

// The float64 strided C2C passes use the pair-split engine at these lengths
// (in float32 the two-step kernel with 16-column tiles streams faster); 288
// and 392 have only the pair-split factorisation.
template <typename T> constexpr bool c2c_pair(int N) {
  return N == 288 || N == 392 || (sizeof(T) == 8 && (N == 128 || N == 512));
}
// column tile of the strided pair-split pass: 128-byte row segments
template <typename T> constexpr int c2c_pair_NB() { return sizeof(T) == 4 ? 16 : 8; }
// The pair-split engine serves the 3D fused pass where N = 2 E^2.
template <typename T> constexpr bool fused_pair(int N) { return pair_E(N) > 0 && N >= 128 && N <= 512; }

template <typename T, int N, class ENG, int NB, bool HALF>
__global__ void __launch_bounds__(ENG::P * NB, (fused_minwaves<T, N>())) k_col2_fused_staged(const Cx<T>* __restrict__ in,
                                                                                     Cx<T>* __restrict__ out,
                                                                                     ColParams p, FusedSpec fs) {
  using V = Cx<T>;
  constexpr int E = ENG::E;
  constexpr int P = ENG::P;
  constexpr int kTabChunk = tab_chunk<T>();
  constexpr int H = N / 2 + 1;                     // folded rows along the transform axis
  constexpr int SLICE = H * NB;                    // table elements per channel slice
  constexpr int SLICE16 = SLICE * (int)sizeof(T) / 16;
  static_assert((SLICE * sizeof(T)) % 16 == 0, "slice must be a whole number of 16-byte words");
  __shared__ __align__(16) T xch[ENG::LDS];
  __shared__ __align__(16) T tab_lds[kTabChunk * SLICE];
  const int tid = threadIdx.x;
  constexpr int NT = P * NB;
  const int b = tid % NB, pt = tid / NB;
  const int kx = blockIdx.x * NB + b;
  const bool active = kx < p.inner;
  const int kxs = active ? kx : 0;
  // block y serves the column pair (of, outer_len - of): one folded table slice
  const int of = blockIdx.y;
  const int n_cols = (of == 0 || 2 * of == p.outer_len) ? 1 : 2;
  const FusedItem& IT = fs.items[blockIdx.z];
  const FusedGroup& G = fs.g[IT.group];
  typename ENG::Tw tw;
  tw.load((const V*)p.tw, pt);
  // complete the twiddle loads now: a wait at their first use would also
  // wait for the asynchronous table copy issued below
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  if constexpr (ENG::Tw::NEEDS_BARRIER) __syncthreads();

  // Copy the contiguous table slices of tabs[0..nt) into LDS.  Each wave
  // moves 1 KiB runs with direct global-to-LDS loads, which do not pass
  // through registers and complete asynchronously: the copy overlaps the
  // column loads that follow.  It is complete for the whole block once every
  // wave has waited for its loads and passed a barrier: load_fwd waits for
  // all loads before its first exchange barrier, stage_wait does both.
  auto stage = [&](const int* tabs, int nt) {
    // slice addresses first: a wait for these loads would also wait for copies already issued
    const uint4* src[kTabChunk];
#pragma unroll
    for (int c = 0; c < kTabChunk; ++c)
      src[c] = c < nt ? (const uint4*)((const T*)fs.tabs[tabs[c]].ptr + (int64_t)of * fs.tab_outer_stride +
                                       (int64_t)blockIdx.x * fs.tab_tile_stride)
                      : nullptr;
    __syncthreads();                                  // earlier readers of tab_lds are done
    constexpr int RUNS = (SLICE16 + 63) / 64;         // 64-lane runs per slice
    constexpr int NW = NT / 64;                       // whole waves (a partial last wave does not copy)
    static_assert(NW >= 1, "the block needs a whole wave");
    const int lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int c = 0; c < kTabChunk; ++c) {
      if (c >= nt) break;
      for (int r = w; w < NW && r < RUNS; r += NW) {
        const int idx = r * 64 + lane;
        if (idx < SLICE16)
          __builtin_amdgcn_global_load_lds(
              (__attribute__((address_space(1))) void*)(src[c] + idx),
              (__attribute__((address_space(3))) void*)((uint4*)tab_lds + c * SLICE16 + r * 64), 16, 0, 0);
      }
    }
  };
  auto stage_wait = [&]() {
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
  };
  auto issue_load = [&](int ch, int o, V* v) {
    const V* src = in + (int64_t)ch * p.in_ch + (int64_t)o * p.in_outer + kxs;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = pt + P * e;
      if (HALF && e >= E / 2) v[e] = mk<V>(T(0), T(0));
      else v[e] = (active && n < p.n_in) ? src[(int64_t)n * p.in_line] : mk<V>(T(0), T(0));
    }
  };
  // Forward transform of a loaded column.  With the pair-basis product the
  // transform stops before the lane butterfly and cr receives the partner's
  // twiddled half (PairFFT::cross); otherwise cr is unused.
  auto fwd = [&](V* v, V* cr) {
    if constexpr (ENG::PAIR_PRODUCT) {
      ENG::forward_half(v, xch, pt, b, tw);     // starts with a barrier
      ENG::cross(v, cr, pt);
    } else {
      ENG::forward_split(v, xch, pt, b, tw);
    }
  };
  auto load_fwd = [&](int ch, int o, V* v, V* cr) {
    issue_load(ch, o, v);
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);   // the column and any table copy issued before it
    fwd(v, cr);
  };
  // res[i] (+)= v[i] * kernel spectrum at slot i: the folded table entry with
  // the signs of the odd axes and the factor (-i)^phase
  auto times = [&](int slot, int tab, bool o_neg, const V* v, V* res, bool accumulate) {
    const TabRef& t = fs.tabs[tab];
    const bool flip_o = t.odd_outer && o_neg;
    if constexpr (ENG::LINEAR_FOLD) {
      // one sign per lane and a linear walk through the table column
      const bool flip = flip_o != (t.odd_line && ENG::fold_neg(pt));
      const T* tl = tab_lds + slot * SLICE + b + ENG::fold_base(pt) * NB;
      const int step = ENG::fold_step(pt) * NB;
      const T sgn = flip ? T(-1) : T(1);
      auto apply = [&](auto rot) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const V prod = rot(cscale(v[i], sgn * tl[i * step]));
          res[i] = accumulate ? cadd(res[i], prod) : prod;
        }
      };
      switch (t.phase & 3) {   // uniform: one branch per call, not per element
        case 0: apply([](V a) { return a; }); break;
        case 1: apply([](V a) { return mul_mi(a); }); break;
        case 2: apply([](V a) { return mk<V>(-a.x, -a.y); }); break;
        default: apply([](V a) { return mul_pi(a); }); break;
      }
    } else {
      const T* tl = tab_lds + slot * SLICE + b;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int l = ENG::slot(pt, i);
        const bool l_neg = 2 * l > N;
        const int lf = l_neg ? N - l : l;
        T val = tl[lf * NB];
        if (flip_o != (t.odd_line && l_neg)) val = -val;
        const V prod = mul_mi_pow(cscale(v[i], val), t.phase);
        res[i] = accumulate ? cadd(res[i], prod) : prod;
      }
    }
  };
  // res[j] (+)= the product in the pair basis (PairFFT): (K0 + K1) z[j] +
  // (K0 - K1) cr[j], K0 and K1 the kernel spectrum at the slots k1 + E j and
  // k1 + E j + N/2 of the lane pair k1; their folded table rows are k1 + E j
  // and N/2 - k1 - E j.  A kernel odd along the line axis negates K1, which
  // swaps the two coefficients; odd along the outer axis at a negative
  // outer frequency negates both (a half turn of the phase).
  auto pair_times = [&](int slot, int tab, bool o_neg, const V* z, const V* cr, V* res, bool accumulate) {
    const TabRef& t = fs.tabs[tab];
    const int k1 = pt >> 1;
    const T* t0 = tab_lds + slot * SLICE + b + k1 * NB;
    const T* t1 = tab_lds + slot * SLICE + b + (N / 2 - k1) * NB;
    const int ph = (t.phase + ((t.odd_outer && o_neg) ? 2 : 0)) & 3;
    auto apply = [&](auto rot, auto odd) {
      constexpr bool ODD = decltype(odd)::value;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const T a0 = t0[j * E * NB];
        const T a1 = t1[-j * E * NB];
        const T cA = ODD ? a0 - a1 : a0 + a1;
        const T cD = ODD ? a0 + a1 : a0 - a1;
        const V prod = rot(mk<V>(fma(cA, z[j].x, cD * cr[j].x), fma(cA, z[j].y, cD * cr[j].y)));
        res[j] = accumulate ? cadd(res[j], prod) : prod;
      }
    };
    auto by_phase = [&](auto odd) {
      switch (ph) {   // uniform: one branch per call, not per element
        case 0: apply([](V a) { return a; }, odd); break;
        case 1: apply([](V a) { return mul_mi(a); }, odd); break;
        case 2: apply([](V a) { return mk<V>(-a.x, -a.y); }, odd); break;
        default: apply([](V a) { return mul_pi(a); }, odd); break;
      }
    };
    if (t.odd_line) by_phase(std::true_type{});
    else by_phase(std::false_type{});
  };
  auto product = [&](int slot, int tab, bool o_neg, const V* z, const V* cr, V* res, bool accumulate) {
    if constexpr (ENG::PAIR_PRODUCT) pair_times(slot, tab, o_neg, z, cr, res, accumulate);
    else times(slot, tab, o_neg, z, res, accumulate);
  };
  auto inv_store = [&](V* v, int ch, int o) {
    if constexpr (ENG::PAIR_PRODUCT) ENG::inverse_half(v, xch, pt, b, tw);
    else ENG::inverse_split(v, xch, pt, b, tw);
    if (!active) return;
    V* dst = out + (int64_t)ch * p.out_ch + (int64_t)o * p.out_outer + kx;
#pragma unroll
    for (int n2 = 0; n2 < E; ++n2) {
      if (HALF && n2 >= E / 2) continue;
      const int n = pt + P * n2;
      if (n < p.n_out) dst[(int64_t)n * p.out_line] = v[n2];
    }
  };
  auto column = [&](int col) { return col == 0 ? of : p.outer_len - of; };

  if (G.mode == 0) {
    if (IT.c1 - IT.c0 <= kTabChunk) {
      // every table of the item fits: stage once for both columns.  The
      // second column's input is loaded before the first column's stores, so
      // waiting for it does not wait for those stores (the vector memory
      // counter covers loads and stores in issue order).
      stage(&G.tab[IT.c0], IT.c1 - IT.c0);
      V spec[E], cr[E];
      load_fwd(G.in_ch[0], column(0), spec, cr);
      for (int col = 0; col < n_cols; ++col) {
        const int o = column(col);
        const bool o_neg = 2 * o > p.outer_len;
        V nxt[E];
        if (col + 1 < n_cols) issue_load(G.in_ch[0], column(col + 1), nxt);
        for (int c = IT.c0; c < IT.c1; ++c) {
          V v[E];
          product(c - IT.c0, G.tab[c], o_neg, spec, cr, v, false);
          inv_store(v, G.out_ch[c], o);
        }
        if (col + 1 < n_cols) {
#pragma unroll
          for (int e = 0; e < E; ++e) spec[e] = nxt[e];
          fwd(spec, cr);
        }
      }
    } else {
      // one forward transform per column; the table chunks are restaged per
      // column (the second time from L2)
      for (int col = 0; col < n_cols; ++col) {
        const int o = column(col);
        const bool o_neg = 2 * o > p.outer_len;
        V spec[E], cr[E];
        load_fwd(G.in_ch[0], o, spec, cr);
        for (int c0 = IT.c0; c0 < IT.c1; c0 += kTabChunk) {
          const int nc = IT.c1 - c0 < kTabChunk ? IT.c1 - c0 : kTabChunk;
          stage(&G.tab[c0], nc);
          stage_wait();
          for (int c = 0; c < nc; ++c) {
            V v[E];
            product(c, G.tab[c0 + c], o_neg, spec, cr, v, false);
            inv_store(v, G.out_ch[c0 + c], o);
          }
        }
      }
    }
  } else {
    const bool once = G.n_in <= kTabChunk;
    if (once) stage(G.tab, G.n_in);
    for (int col = 0; col < n_cols; ++col) {
      const int o = column(col);
      const bool o_neg = 2 * o > p.outer_len;
      V acc[E];
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] = mk<V>(T(0), T(0));
      for (int i = 0; i < G.n_in; ++i) {
        V v[E], cr[E];
        load_fwd(G.in_ch[i], o, v, cr);
        if (!once) {
          stage(&G.tab[i], 1);
          stage_wait();
        }
        product(once ? i : 0, G.tab[i], o_neg, v, cr, acc, true);
      }
      inv_store(acc, G.out_ch[0], o);
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers (return false when the length has no two-step factorisation)
// ---------------------------------------------------------------------------
int col2_tile_width(int N, bool fp64, bool fused) {
  int E = fp64 ? (fused ? twostep_E<double, true>(N) : twostep_E<double, false>(N))
               : (fused ? twostep_E<float, true>(N) : twostep_E<float, false>(N));
  if (fused && (fp64 ? fused_pair<double>(N) : fused_pair<float>(N))) E = pair_E(N);
  if (!fused && (fp64 ? c2c_pair<double>(N) : c2c_pair<float>(N)))
    return fp64 ? c2c_pair_NB<double>() : c2c_pair_NB<float>();
  if (E == 0) return 0;
  if (fused) return fp64 ? twostep_NB<double, true>() : twostep_NB<float, true>();
  return fp64 ? twostep_NB<double>() : twostep_NB<float>();
}

#define DT_FOR_EACH_COL2_N(X) X(64) X(128) X(256) X(288) X(392) X(512) X(1024)

template <typename T> bool launch_col2_c2c(const void* in, void* out, const ColParams& p, int N, int dir, int tiles,
                                           int outer, int chans, hipStream_t st) {
  const dim3 grid1(tiles, outer, chans);
  const bool half = dir > 0 ? (2 * p.n_in == N) : (2 * p.n_out == N);
  if (c2c_pair<T>(N)) {
    const Cx<T>* i_ = (const Cx<T>*)in;
    Cx<T>* o_ = (Cx<T>*)out;
    switch (N) {
#define CASEP(NN)                                                                                         \
  case NN: {                                                                                              \
    constexpr int NB = c2c_pair_NB<T>();                                                                  \
    constexpr int NT = 2 * pair_E(NN) * NB;                                                               \
    if (dir > 0 && half) hipLaunchKernelGGL((k_col2_c2c_pair<T, NN, NB, 1, true>), grid1, dim3(NT), 0, st, i_, o_, p);  \
    else if (dir > 0) hipLaunchKernelGGL((k_col2_c2c_pair<T, NN, NB, 1, false>), grid1, dim3(NT), 0, st, i_, o_, p);    \
    else if (half) hipLaunchKernelGGL((k_col2_c2c_pair<T, NN, NB, -1, true>), grid1, dim3(NT), 0, st, i_, o_, p);       \
    else hipLaunchKernelGGL((k_col2_c2c_pair<T, NN, NB, -1, false>), grid1, dim3(NT), 0, st, i_, o_, p);                \
    return true;                                                                                          \
  }
      CASEP(128) CASEP(288) CASEP(392) CASEP(512)
#undef CASEP
      default: break;
    }
  }
  switch (N) {
#define CASE(NN)                                                                                          \
  case NN: {                                                                                              \
    constexpr int E = twostep_E<T, false>(NN);                                                            \
    if constexpr (E == 0) {                                                                               \
      return false;                                                                                       \
    } else {                                                                                              \
      constexpr int NB = twostep_NB<T>();                                                                 \
      constexpr int NT = (NN / E) * NB;                                                                   \
      const Cx<T>* i_ = (const Cx<T>*)in;                                                                 \
      Cx<T>* o_ = (Cx<T>*)out;                                                                            \
      if (dir > 0 && half) hipLaunchKernelGGL((k_col2_c2c<T, NN, E, NB, 1, true>), grid1, dim3(NT), 0, st, i_, o_, p);  \
      else if (dir > 0) hipLaunchKernelGGL((k_col2_c2c<T, NN, E, NB, 1, false>), grid1, dim3(NT), 0, st, i_, o_, p);    \
      else if (half) hipLaunchKernelGGL((k_col2_c2c<T, NN, E, NB, -1, true>), grid1, dim3(NT), 0, st, i_, o_, p);       \
      else hipLaunchKernelGGL((k_col2_c2c<T, NN, E, NB, -1, false>), grid1, dim3(NT), 0, st, i_, o_, p);                \
      return true;                                                                                        \
    }                                                                                                     \
  }
    DT_FOR_EACH_COL2_N(CASE)
#undef CASE
    default: return false;
  }
}

template <typename T> bool launch_col2_fused(const void* in, void* out, const ColParams& p, const FusedSpec& fs,
                                             int N, int tiles, int outer, hipStream_t st) {
  const dim3 grid(tiles, outer, fs.n_items);
  const bool half = 2 * p.n_in == N && 2 * p.n_out == N;
  const Cx<T>* i_ = (const Cx<T>*)in;
  Cx<T>* o_ = (Cx<T>*)out;
  const dim3 gm(tiles, p.outer_len / 2 + 1, fs.n_items);
  switch (N) {
#define CASE(NN)                                                                                          \
  case NN: {                                                                                              \
    constexpr int E = twostep_E<T, true>(NN);                                                             \
    constexpr int NB = twostep_NB<T, true>();                                                             \
    if (p.outer_len > 1 || (E == 0 && fused_pair<T>(NN))) {                                              \
      if constexpr (fused_pair<T>(NN)) {                                                                     \
        using ENG = PairFFT<T, NN, NB, fused_split<T>(), fused_twl<T>()>;                                 \
        constexpr int NT = ENG::P * NB;                                                                   \
        if (half) hipLaunchKernelGGL((k_col2_fused_staged<T, NN, ENG, NB, true>), gm, dim3(NT), 0, st, i_, o_, p, fs); \
        else hipLaunchKernelGGL((k_col2_fused_staged<T, NN, ENG, NB, false>), gm, dim3(NT), 0, st, i_, o_, p, fs);     \
        return true;                                                                                      \
      } else if constexpr (E > 0) {                                                                       \
        using ENG = TwoStep<T, NN, E, NB>;                                                                \
        constexpr int NT = ENG::P * NB;                                                                   \
        if (half) hipLaunchKernelGGL((k_col2_fused_staged<T, NN, ENG, NB, true>), gm, dim3(NT), 0, st, i_, o_, p, fs); \
        else hipLaunchKernelGGL((k_col2_fused_staged<T, NN, ENG, NB, false>), gm, dim3(NT), 0, st, i_, o_, p, fs);     \
        return true;                                                                                      \
      } else {                                                                                            \
        return false;                                                                                     \
      }                                                                                                   \
    }                                                                                                     \
    if constexpr (E > 0) {                                                                                \
      constexpr int NT = (NN / E) * NB;                                                                   \
      if (half) hipLaunchKernelGGL((k_col2_fused<T, NN, E, NB, true>), grid, dim3(NT), 0, st, i_, o_, p, fs); \
      else hipLaunchKernelGGL((k_col2_fused<T, NN, E, NB, false>), grid, dim3(NT), 0, st, i_, o_, p, fs);     \
      return true;                                                                                        \
    } else {                                                                                              \
      return false;                                                                                       \
    }                                                                                                     \
  }
    DT_FOR_EACH_COL2_N(CASE)
#undef CASE
    default: return false;
  }
}

template bool launch_col2_c2c<float>(const void*, void*, const ColParams&, int, int, int, int, int, hipStream_t);
template bool launch_col2_c2c<double>(const void*, void*, const ColParams&, int, int, int, int, int, hipStream_t);
template bool launch_col2_fused<float>(const void*, void*, const ColParams&, const FusedSpec&, int, int, int,
                                       hipStream_t);
template bool launch_col2_fused<double>(const void*, void*, const ColParams&, const FusedSpec&, int, int, int,
                                        hipStream_t);

}  // namespace dt
