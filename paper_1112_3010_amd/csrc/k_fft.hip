// FFT passes of the zero-padded convolution (Sec. 3, Table 1 steps 3-6):
//
//   row_r2c      x pass, real -> half spectrum (input rows zero-padded from
//                n_x to M_x; a length-M_x real transform done as a length
//                M_x/2 complex transform of packed even/odd samples).
//   col_c2c      strided pass along y (3D forward or inverse), with the
//                zero input rows (forward) or unused output rows (inverse)
//                pruned.
//   col_fused    last axis: forward transform of the source images, pointwise
//                product with the kernel spectra (Table 1 step 4) for every
//                output channel, inverse transform, keep only the n rows of
//                the unpadded grid.  The source spectrum never leaves
//                registers.
//   row_c2r_epi  x pass, half spectrum -> real, fused with the epilogue:
//                S = -tau log phi (step 6), the derivative ratios of Sec. 5
//                and the winding number / degree label of Sec. 4.
#include <math.h>

#include <algorithm>

#include "dt_launch.hpp"
#include "fft_engine.hpp"
#include "fft_twostep.hpp"
#include "epilogue.hpp"

namespace dt {

// LDS position of element i of a row line: XOR-swizzling the low five bits
// with bits 3..7 spreads the strided Stockham accesses over the 64 banks
// (a bijection on [0, N) for power-of-two N >= 256; other lengths keep the
// natural order).
template <int N> __device__ __forceinline__ int row_swz(int i) {
  if constexpr ((N & (N - 1)) == 0) return i ^ ((i >> 3) & 31);
  else return i;
}
// bin k of a half-spectrum line read from the length-N complex transform (bin N is bin 0)
template <int N> __device__ __forceinline__ int row_wrap(int k) { return k == N ? 0 : k; }

// ---------------------------------------------------------------------------
// Row pass: real -> half spectrum
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(256) k_row_r2c(const T* __restrict__ in, Cx<T>* __restrict__ out, RowParams p) {
  using V = Cx<T>;
  constexpr int E = row_E(N);
  constexpr int Q = N / E;
  constexpr int LPB = Q >= 256 ? 1 : 256 / Q;
  constexpr int LP = N + 1;
  constexpr int R0 = fft_radix(N, 0);
  using F = Stockham<T, N, E, +1>;
  __shared__ __align__(16) V lds[LPB * LP];
  const int tid = threadIdx.x;
  const int q = tid % Q, b = tid / Q;
  const int64_t line = (int64_t)blockIdx.x * LPB + b;
  const bool active = line < p.n_lines;
  const V* tw = (const V*)p.tw;  // exp(-2 pi i m / M), M = 2N
  V v[E];
  if ((p.nx * (int)sizeof(T)) % 16 == 0) {
    // The block's rows are one contiguous run of LPB * nx reals: copy it
    // into LDS with direct global-to-LDS loads (16-byte words), then take
    // each thread's sample pairs from there.  The rows (nx <= 2N reals)
    // fit the exchange buffer, which B::run writes only after a barrier.
    const int wpl = p.nx * (int)sizeof(T) / 16;   // words per row
    const int64_t line0 = (int64_t)blockIdx.x * LPB;
    const int64_t rows = p.n_lines - line0 < LPB ? p.n_lines - line0 : LPB;
    const int words = (int)rows * wpl;
    const uint4* g = reinterpret_cast<const uint4*>(in + line0 * (int64_t)p.nx);
    const int lane = tid & 63, w = tid >> 6, nfw = blockDim.x >> 6;   // whole waves only
    for (int r = w; w < nfw && r * 64 < words; r += nfw) {
      const int u = r * 64 + lane;
      if (u < words)
        __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(g + u),
                                         (__attribute__((address_space(3))) void*)((uint4*)lds + r * 64), 16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    const T* raw = reinterpret_cast<const T*>(lds) + b * p.nx;
#pragma unroll
    for (int s = 0; s < E / R0; ++s)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int m = 2 * F::template in_index<0>(q, s, r);
        const T a = (active && m < p.nx) ? raw[m] : T(0);
        const T c = (active && m + 1 < p.nx) ? raw[m + 1] : T(0);
        v[s * R0 + r] = mk<V>(a, c);
      }
  } else {
    const T* src = in + (active ? line : 0) * (int64_t)p.nx;
#pragma unroll
    for (int s = 0; s < E / R0; ++s)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int m = 2 * F::template in_index<0>(q, s, r);
        const T a = (active && m < p.nx) ? src[m] : T(0);
        const T c = (active && m + 1 < p.nx) ? src[m + 1] : T(0);
        v[s * R0 + r] = mk<V>(a, c);
      }
  }
  auto addr = [b](int i) { return b * LP + row_swz<N>(i); };
  F::run(v, lds, q, tw, 2, addr);   // its first LDS store follows a barrier
  __syncthreads();
  F::store_last(lds, v, q, addr);
  __syncthreads();
  if (!active) return;
  // twiddles of this thread's output bins k = q + Q j (k <= N), all loads issued at once
  constexpr int NK = N / Q + 1;
  V twk[NK];
#pragma unroll
  for (int j = 0; j < NK; ++j) twk[j] = q + Q * j <= N ? tw[q + Q * j] : mk<V>(T(0), T(0));
  V* dst = out + line * (int64_t)p.pitch;
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    const int k = q + Q * j;
    if (k > N) break;
    const V zk = lds[addr(row_wrap<N>(k))];
    const V zc = cconj(lds[addr(row_wrap<N>(N - k))]);
    const V ev = cscale(cadd(zk, zc), T(0.5));
    const V od = cscale(mul_mi(csub(zk, zc)), T(0.5));
    dst[k] = cadd(ev, cmul(twk[j], od));
  }
}

// ---------------------------------------------------------------------------
// Column pass (C2C along a strided axis), tiles of NB consecutive kx bins
// ---------------------------------------------------------------------------
template <typename T, int N, int NB, int NT, int DIR>
__global__ void __launch_bounds__(NT) k_col_c2c(const Cx<T>* __restrict__ in, Cx<T>* __restrict__ out,
                                                ColParams p) {
  using V = Cx<T>;
  constexpr int E = N * NB / NT;
  constexpr int R0 = fft_radix(N, 0);
  constexpr int S = fft_stages(N);
  constexpr int RL = fft_radix(N, S - 1);
  using F = Stockham<T, N, E, DIR>;
  static_assert(F::Q * NB == NT, "block shape");
  __shared__ V lds[N * NB];
  const int tid = threadIdx.x;
  const int b = tid % NB, q = tid / NB;
  const int kx = blockIdx.x * NB + b;
  const bool active = kx < p.inner;
  const V* src = in + blockIdx.z * p.in_ch + blockIdx.y * p.in_outer + (active ? kx : 0);
  V v[E];
#pragma unroll
  for (int s = 0; s < E / R0; ++s)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int i = F::template in_index<0>(q, s, r);
      v[s * R0 + r] = (active && i < p.n_in) ? src[(int64_t)i * p.in_line] : mk<V>(T(0), T(0));
    }
  auto addr = [b](int i) { return i * NB + b; };
  F::run(v, lds, q, (const V*)p.tw, p.tw_stride, addr);
  if (!active) return;
  V* dst = out + blockIdx.z * p.out_ch + blockIdx.y * p.out_outer + kx;
#pragma unroll
  for (int s = 0; s < E / RL; ++s)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int i = F::template in_index<S - 1>(q, s, r);
      if (i < p.n_out) dst[(int64_t)i * p.out_line] = v[s * RL + r];
    }
}

// ---------------------------------------------------------------------------
// Fused last-axis pass: forward, multiply by kernel spectra, inverse
// ---------------------------------------------------------------------------
template <typename T, int N, int NB, int NT>
__global__ void __launch_bounds__(NT) k_col_fused(const Cx<T>* __restrict__ in, Cx<T>* __restrict__ out,
                                                  ColParams p, FusedSpec fs) {
  using V = Cx<T>;
  constexpr int E = N * NB / NT;
  constexpr int S = fft_stages(N);
  constexpr int R0 = fft_radix(N, 0);
  constexpr int RL = fft_radix(N, S - 1);
  static_assert(R0 == RL, "forward output slots must be the inverse input slots");
  using Fw = Stockham<T, N, E, +1>;
  using Bw = Stockham<T, N, E, -1>;
  __shared__ V lds[N * NB];
  const int tid = threadIdx.x;
  const int b = tid % NB, q = tid / NB;
  const int kx = blockIdx.x * NB + b;
  const bool active = kx < p.inner;
  const int kxs = active ? kx : 0;
  const int o = blockIdx.y;
  const bool o_neg = 2 * o > p.outer_len;
  const int of = o_neg ? p.outer_len - o : o;
  const FusedItem& IT = fs.items[blockIdx.z];
  const FusedGroup& G = fs.g[IT.group];
  const V* tw = (const V*)p.tw;
  auto addr = [b](int i) { return i * NB + b; };

  auto load_fwd = [&](int ch, V* v) {
    const V* src = in + (int64_t)ch * p.in_ch + (int64_t)o * p.in_outer + kxs;
#pragma unroll
    for (int s = 0; s < E / R0; ++s)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int i = Fw::template in_index<0>(q, s, r);
        v[s * R0 + r] = (active && i < p.n_in) ? src[(int64_t)i * p.in_line] : mk<V>(T(0), T(0));
      }
    Fw::run(v, lds, q, tw, p.tw_stride, addr);
  };
  // v *= kernel spectrum of table t at this block's (kx, outer, line) slots
  auto times_table = [&](const TabRef& t, const V* v, V* res, bool accumulate) {
    const T* tab = (const T*)t.ptr + (int64_t)of * fs.tab_outer_stride + (int64_t)blockIdx.x * fs.tab_tile_stride + b;
    const bool flip_o = t.odd_outer && o_neg;
#pragma unroll
    for (int s = 0; s < E / RL; ++s)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int l = Fw::template in_index<S - 1>(q, s, r);
        const bool l_neg = 2 * l > N;
        const int lf = l_neg ? N - l : l;
        T tv = tab[(int64_t)lf * fs.tab_line_stride];
        if (flip_o != (t.odd_line && l_neg)) tv = -tv;
        const V prod = mul_mi_pow(cscale(v[s * RL + r], tv), t.phase);
        res[s * RL + r] = accumulate ? cadd(res[s * RL + r], prod) : prod;
      }
  };
  auto inv_store = [&](V* v, int ch) {
    Bw::run(v, lds, q, tw, p.tw_stride, addr);
    if (!active) return;
    V* dst = out + (int64_t)ch * p.out_ch + (int64_t)o * p.out_outer + kx;
#pragma unroll
    for (int s = 0; s < E / RL; ++s)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int i = Bw::template in_index<S - 1>(q, s, r);
        if (i < p.n_out) dst[(int64_t)i * p.out_line] = v[s * RL + r];
      }
  };

  if (G.mode == 0) {
    V spec[E];
    load_fwd(G.in_ch[0], spec);
    for (int c = IT.c0; c < IT.c1; ++c) {
      V v[E];
      times_table(fs.tabs[G.tab[c]], spec, v, false);
      inv_store(v, G.out_ch[c]);
    }
  } else {
    V acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = mk<V>(T(0), T(0));
    for (int i = 0; i < G.n_in; ++i) {
      V v[E];
      load_fwd(G.in_ch[i], v);
      times_table(fs.tabs[G.tab[i]], v, acc, true);
    }
    inv_store(acc, G.out_ch[0]);
  }
}

// ---------------------------------------------------------------------------
// Row pass: half spectrum -> real, fused with the epilogue
// ---------------------------------------------------------------------------
// The float32 S/grad instantiation is held to eight waves per SIMD: left to
// itself the compiler keeps about 106 scalar registers (seven waves), and the
// pass is VALU-bound, so the eighth wave pays for the few scalar spills.
template <typename T, int N, bool CURV>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && !CURV) ? 8 : 1)))
k_row_c2r_epi(const Cx<T>* __restrict__ in, RowParams p, EpiParams e) {
  using V = Cx<T>;
  constexpr int E = row_E(N);
  constexpr int Q = N / E;
  constexpr int LP = N + 1;
  constexpr int R0 = fft_radix(N, 0);
  constexpr int S = fft_stages(N);
  constexpr int RL = fft_radix(N, S - 1);
  using B = Stockham<T, N, E, -1>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const int C = e.C;
  const int lines = blockDim.x / Q;
  const int RPB = lines / C;
  const int tid = threadIdx.x;
  const int q = tid % Q, b = tid / Q;
  const int rl = b / C;
  const int64_t row = (int64_t)blockIdx.x * RPB + rl;
  const bool active = row < e.n_rows;
  const V* tw = (const V*)p.tw;  // exp(-2 pi i m / M), M = 2N
  const EpiConst<T> kc = epi_const<T>(e);
  V v[E];
  // Copy the block's half-spectrum lines into LDS with direct global-to-LDS
  // loads (16-byte words, one contiguous run per line, no registers), then
  // read each bin k and its mirror N - k from there.  A line of N + 1 bins
  // is rounded up to whole words; the row pitch (>= N + 2 complex values)
  // keeps the rounded read inside the row.
  constexpr int W16 = ((N + 1) * (int)sizeof(V) + 15) / 16;   // words per line
  constexpr int LW = W16 * 16 / (int)sizeof(V);               // complex values per staged line
  V twk[E];
#pragma unroll
  for (int s = 0; s < E / R0; ++s)
#pragma unroll
    for (int r = 0; r < R0; ++r) twk[s * R0 + r] = tw[B::template in_index<0>(q, s, r)];
  {
    // Only whole waves copy: a wave's copy writes 64 consecutive words, one
    // per hardware lane, and a partial last wave lacks some of those lanes.
    // The launch has at least one whole wave.
    const int words = lines * W16;
    const int lane = tid & 63, w = tid >> 6, nfw = blockDim.x >> 6;
    for (int r = w; w < nfw && r * 64 < words; r += nfw) {
      const int u = r * 64 + lane;
      const int line = u / W16, wd = u - line * W16;
      const int64_t row_u = (int64_t)blockIdx.x * RPB + line / C;
      if (u < words && row_u < e.n_rows) {
        const uint4* g = reinterpret_cast<const uint4*>(in + (int64_t)(line % C) * e.ch_stride +
                                                        row_u * (int64_t)p.pitch) + wd;
        __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)g,
                                         (__attribute__((address_space(3))) void*)((uint4*)smem_raw + r * 64), 16,
                                         0, 0);
      }
    }
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
  }
  const V* raw = lds + b * LW;
#pragma unroll
  for (int s = 0; s < E / R0; ++s)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int k = B::template in_index<0>(q, s, r);
      V z = mk<V>(T(0), T(0));
      if (active) {
        const V xk = raw[k];
        const V xc = cconj(raw[N - k]);
        const V ev = cadd(xk, xc);
        const V od = cmul(csub(xk, xc), cconj(twk[s * R0 + r]));
        z = mk<V>(ev.x - od.y, ev.y + od.x);  // ev + i * od
      }
      v[s * R0 + r] = z;
    }
  // the staged lines alias the exchange buffer: B::run passes a barrier
  // before its first LDS store
  auto addr = [b](int i) { return b * LP + row_swz<N>(i); };
  B::run(v, lds, q, tw, 2, addr);
  __syncthreads();
  T* ldr = reinterpret_cast<T*>(lds);
#pragma unroll
  for (int s = 0; s < E / RL; ++s)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int j = B::template in_index<S - 1>(q, s, r);
      ldr[(int64_t)b * 2 * LP + 2 * j] = v[s * RL + r].x;
      ldr[(int64_t)b * 2 * LP + 2 * j + 1] = v[s * RL + r].y;
    }
  __syncthreads();
  // channel c of a node sits 2 LP values after channel c - 1
  const int nx = p.nx;
  if (RPB == 1) {
    if (active)
      for (int x = tid; x < nx; x += blockDim.x)
        epilogue_node<T, CURV>(e, kc, [&](int cc) { return ldr[cc * 2 * LP + x]; }, row * nx + x);
  } else {
    for (int t = tid; t < RPB * nx; t += blockDim.x) {
      const int r2 = t / nx, x = t % nx;
      const int64_t row2 = (int64_t)blockIdx.x * RPB + r2;
      if (row2 >= e.n_rows) continue;
      const T* base = ldr + (int64_t)r2 * C * 2 * LP + x;
      epilogue_node<T, CURV>(e, kc, [&](int cc) { return base[cc * 2 * LP]; }, row2 * nx + x);
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Column tile shapes: NB consecutive kx bins per block (NB * sizeof(complex)
// >= 128 bytes per row segment where the LDS budget allows), NT threads,
// E = N * NB / NT elements per thread.  Separate shapes for the plain and the
// fused column passes.
constexpr int cmin(int a, int b) { return a < b ? a : b; }
template <typename T, bool FUSED> struct ColShape {
  static constexpr bool F64 = sizeof(T) == 8;
  static constexpr int NBP = F64 ? 8 : 16;
  static constexpr int NTP = 512;
  static constexpr int nb(int N) { return cmin(NBP, 65536 / (N * (int)sizeof(Cx<T>))); }
  static constexpr int nt(int N) { return cmin(NTP, N * nb(N) / 8); }
};

int col2_tile_width(int N, bool fp64, bool fused);
template <typename T> bool launch_col2_c2c(const void* in, void* out, const ColParams& p, int N, int dir, int tiles,
                                           int outer, int chans, hipStream_t st);
template <typename T> bool launch_col2_fused(const void* in, void* out, const ColParams& p, const FusedSpec& fs,
                                             int N, int tiles, int outer, hipStream_t st);

// Row engine of an N-point line, for the plan log: points per thread and
// the radix of each stage (returns the stage count).
int row_points_per_thread(int N) { return row_E(N); }
int row_radices(int N, int* radix, int cap) {
  const int S = fft_stages(N);
  for (int s = 0; s < S && s < cap; ++s) radix[s] = fft_radix(N, s);
  return S;
}

int col_tile_width(int N, bool fp64, bool fused) {
  const int nb2 = col2_tile_width(N, fp64, fused);
  if (nb2 > 0) return nb2;
  if (fp64) return fused ? ColShape<double, true>::nb(N) : ColShape<double, false>::nb(N);
  return fused ? ColShape<float, true>::nb(N) : ColShape<float, false>::nb(N);
}

// Row passes transform M_x/2 complex points, column passes M points; M >= 64.
#define DT_FOR_EACH_N(X) X(32) X(64) X(128) X(144) X(196) X(256) X(512) X(1024)
#define DT_FOR_EACH_COL_N(X) X(64) X(128) X(256) X(512) X(1024) X(2048)

template <typename T> bool launch_row_r2c(const T* in, void* out, const RowParams& p, int N, hipStream_t st) {
  const int Q = N / row_E(N);
  const int lpb = Q >= 256 ? 1 : 256 / Q;
  const int64_t blocks = (p.n_lines + lpb - 1) / lpb;
  if (blocks <= 0) return true;
  switch (N) {
#define CASE(NN)                                                                                  \
  case NN:                                                                                        \
    hipLaunchKernelGGL((k_row_r2c<T, NN>), dim3((unsigned)blocks), dim3(lpb * Q), 0, st, in, (Cx<T>*)out, p); \
    return true;
    DT_FOR_EACH_N(CASE)
#undef CASE
    default: return false;
  }
}

template <typename T> bool launch_col_c2c(const void* in, void* out, const ColParams& p, int N, int dir, int tiles,
                                          int outer, int chans, hipStream_t st) {
  if (launch_col2_c2c<T>(in, out, p, N, dir, tiles, outer, chans, st)) return true;
  const dim3 grid(tiles, outer, chans);
  switch (N) {
#define CASE(NN)                                                                                         \
  case NN: {                                                                                             \
    constexpr int NB = ColShape<T, false>::nb(NN), NT = ColShape<T, false>::nt(NN);                      \
    if (dir > 0)                                                                                         \
      hipLaunchKernelGGL((k_col_c2c<T, NN, NB, NT, 1>), grid, dim3(NT), 0, st, (const Cx<T>*)in, (Cx<T>*)out, p); \
    else                                                                                                 \
      hipLaunchKernelGGL((k_col_c2c<T, NN, NB, NT, -1>), grid, dim3(NT), 0, st, (const Cx<T>*)in, (Cx<T>*)out, p); \
    return true;                                                                                         \
  }
    DT_FOR_EACH_COL_N(CASE)
#undef CASE
    default: return false;
  }
}

template <typename T> bool launch_col_fused(const void* in, void* out, const ColParams& p, const FusedSpec& fs,
                                            int N, int tiles, int outer, hipStream_t st) {
  if (launch_col2_fused<T>(in, out, p, fs, N, tiles, outer, st)) return true;
  const dim3 grid(tiles, outer, fs.n_items);
  switch (N) {
#define CASE(NN)                                                                                         \
  case NN: {                                                                                             \
    constexpr int NB = ColShape<T, true>::nb(NN), NT = ColShape<T, true>::nt(NN);                        \
    hipLaunchKernelGGL((k_col_fused<T, NN, NB, NT>), grid, dim3(NT), 0, st, (const Cx<T>*)in, (Cx<T>*)out, p, fs); \
    return true;                                                                                         \
  }
    DT_FOR_EACH_COL_N(CASE)
#undef CASE
    default: return false;
  }
}

template <typename T, int N, bool CURV>
static bool launch_epi_kernel(const void* in, const RowParams& p, const EpiParams& e, int64_t blocks, int threads,
                              size_t shmem, hipStream_t st) {
  if (shmem > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_row_c2r_epi<T, N, CURV>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem) != hipSuccess)
    return false;
  hipLaunchKernelGGL((k_row_c2r_epi<T, N, CURV>), dim3((unsigned)blocks), dim3(threads), shmem, st,
                     (const Cx<T>*)in, p, e);
  return true;
}

constexpr int kEpiThreads = 128;   // threads per block of the final row pass (whole rows per block)
template <typename T> bool launch_row_c2r_epi(const void* in, const RowParams& p, const EpiParams& e, int N,
                                              hipStream_t st) {
  const int Q = N / row_E(N);
  int rpb = kEpiThreads / (e.C * Q);
  if (rpb < 1) rpb = 1;
  // lines of 12 or 14 threads (N = 144, 196): more rows per block, up to
  // 256 threads, for whole wavefronts where that is possible
  if ((Q & (Q - 1)) != 0)
    while ((rpb * e.C * Q) % 64 != 0 && (rpb + 1) * e.C * Q <= 256) ++rpb;
  const int threads = rpb * e.C * Q;
  if (threads > 1024 || threads < 64) return false;
  const int64_t blocks = (e.n_rows + rpb - 1) / rpb;
  // exchange lines of N + 1 values; the staged input lines are rounded up to
  // whole 16-byte words (and need that much row pitch)
  const size_t stage_line = ((size_t)(N + 1) * sizeof(Cx<T>) + 15) / 16 * 16;
  if ((size_t)p.pitch * sizeof(Cx<T>) < stage_line) return false;
  const size_t shmem = std::max((size_t)rpb * e.C * (N + 1) * sizeof(Cx<T>),
                                (size_t)rpb * e.C * stage_line);
  // Beyond 64 KiB (long float64 rows with many channels) the kernel needs the
  // larger per-workgroup LDS of gfx950, granted per kernel.
  int dev = 0, lds_max = 65536;
  if (shmem > 65536) {
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return false;
    if (shmem > (size_t)lds_max) return false;
  }
  if (blocks <= 0) return true;
  switch (N) {
#define CASE(NN)                                                                                         \
  case NN:                                                                                               \
    return e.curv ? launch_epi_kernel<T, NN, true>(in, p, e, blocks, threads, shmem, st)                 \
                  : launch_epi_kernel<T, NN, false>(in, p, e, blocks, threads, shmem, st);
    DT_FOR_EACH_N(CASE)
#undef CASE
    default: return false;
  }
}

template bool launch_row_r2c<float>(const float*, void*, const RowParams&, int, hipStream_t);
template bool launch_row_r2c<double>(const double*, void*, const RowParams&, int, hipStream_t);
template bool launch_col_c2c<float>(const void*, void*, const ColParams&, int, int, int, int, int, hipStream_t);
template bool launch_col_c2c<double>(const void*, void*, const ColParams&, int, int, int, int, int, hipStream_t);
template bool launch_col_fused<float>(const void*, void*, const ColParams&, const FusedSpec&, int, int, int,
                                      hipStream_t);
template bool launch_col_fused<double>(const void*, void*, const ColParams&, const FusedSpec&, int, int, int,
                                       hipStream_t);
template bool launch_row_c2r_epi<float>(const void*, const RowParams&, const EpiParams&, int, hipStream_t);
template bool launch_row_c2r_epi<double>(const void*, const RowParams&, const EpiParams&, int, hipStream_t);

}  // namespace dt
