// Runtime mixed-radix FFT in LDS for the batched path (gfx950).
//
// Batched instances have padded lengths that are 7-smooth (2^a 3^b 5^c 7^d)
// rather than powers of two, and their lengths differ inside one launch, so
// the radix schedule is a runtime list: the prime-power radices 8, 4, 2, 7,
// 5, 3, and fused radices up to 16 (16, 6, 10, 12, 14, 9, 15) whose register
// DFT takes two of those stages at once and saves an LDS round trip and its
// barriers.  A block
// holds L independent lines of length N in LDS; element i of line l sits at
// lds[i * istride + l * lstride].  Each stage is a self-sorting (Stockham,
// decimation in time) pass: butterfly j (k = j mod Ns, Ns = product of the
// earlier radices) reads x[j + r N/R], multiplies input r by W_(Ns R)^(k r),
// does a size-R DFT and writes X[(j / Ns) Ns R + k + r Ns].  All butterflies
// of a stage are read into registers before any result is written back, so
// one LDS buffer suffices (two barriers per stage).
#pragma once

#include "fft_engine.hpp"
#include "fft_twostep.hpp"

namespace dt {

constexpr int kMixedMaxStages = 12;

// Multiply-high constant of FastDiv for divisor d (0 for d <= 1); computed on
// the host where the divisor is known at plan time.
__host__ __device__ constexpr uint32_t fastdiv_magic(uint32_t d) { return d > 1 ? 0xFFFFFFFFu / d + 1u : 0u; }

struct MixedPlan {
  int n_st;
  int radix[kMixedMaxStages];
  uint32_t m_ns[kMixedMaxStages];    // fastdiv_magic(N_s): product of the earlier radices
  uint32_t m_nbf[kMixedMaxStages];   // fastdiv_magic(N / R_s): butterflies per line
};

// Size-3/5/7 DFTs: pair inputs j and R-j, X_k = x0 + sum_j a_j cos(2 pi j k/R)
// - i DIR sum_j b_j sin(2 pi j k/R) with a_j = x_j + x_(R-j), b_j = x_j - x_(R-j);
// X_(R-k) takes the opposite sign of the sine part.
template <int R, int DIR, typename V> __device__ __forceinline__ void dft_odd(V* x) {
  using T = decltype(V::x);
  constexpr int H = (R - 1) / 2;
  V a[H], b[H];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    a[j - 1] = cadd(x[j], x[R - j]);
    b[j - 1] = csub(x[j], x[R - j]);
  }
  V x0 = x[0];
  V s0 = x0;
#pragma unroll
  for (int j = 0; j < H; ++j) s0 = cadd(s0, a[j]);
  V out[R];
  out[0] = s0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    V A = x0, B = mk<V>(T(0), T(0));
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const T c = (T)ct_cos2pi((long)j * k, R);
      const T s = (T)ct_sin2pi((long)j * k, R);
      A = mk<V>(A.x + c * a[j - 1].x, A.y + c * a[j - 1].y);
      B = mk<V>(B.x + s * b[j - 1].x, B.y + s * b[j - 1].y);
    }
    // -i * DIR * B = DIR * (B.y, -B.x)
    const V mb = DIR > 0 ? mk<V>(B.y, -B.x) : mk<V>(-B.y, B.x);
    out[k] = cadd(A, mb);
    out[R - k] = csub(A, mb);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = out[r];
}

template <int R, int DIR, typename V> __device__ __forceinline__ void dft_small(V* x) {
  if constexpr (R == 2 || R == 4 || R == 8) Bfly<R, DIR, V>::run(x);
  else if constexpr (R == 3 || R == 5 || R == 7) dft_odd<R, DIR, V>(x);
  else RegDFT<R, DIR, V>::run(x);
}

// The radices a schedule may use (mixed_plan_for builds schedules from these).
__host__ __device__ constexpr bool mixed_radix_supported(int R) {
  return R == 2 || R == 3 || R == 4 || R == 5 || R == 7 || R == 8 || R == 16 || R == 6 || R == 10 || R == 12 ||
         R == 14 || R == 9 || R == 15;
}

// Division by a block-uniform divisor d in [1, 4096] through a multiply-high:
// q = floor(u * (floor((2^32 - 1) / d) + 1) / 2^32) equals u / d for every
// u < 2^16 (checked exhaustively), which covers every index of a stage.
struct FastDiv {
  uint32_t d, m;
  __device__ __forceinline__ explicit FastDiv(uint32_t d_) : d(d_), m(fastdiv_magic(d_)) {}
  // with the constant precomputed (no division on the device)
  __device__ __forceinline__ FastDiv(uint32_t d_, uint32_t m_) : d(d_), m(m_) {}
  __device__ __forceinline__ uint32_t div(uint32_t u) const { return d > 1 ? __umulhi(u, m) : u; }
};

// One Stockham stage of radix R over all L lines.  ECAP bounds the elements a
// thread holds: the caller guarantees N * L <= ECAP * nthr (< 2^16).
template <typename T, int DIR, int R, int ECAP, bool LINE_FAST>
__device__ __forceinline__ void mixed_stage(Cx<T>* lds, int N, int L, int istride, int lstride, int Ns,
                                            const Cx<T>* __restrict__ tw, int twstride, int tid, int nthr,
                                            const FastDiv& fL, const FastDiv& fNs, const FastDiv& fnbf) {
  using V = Cx<T>;
  constexpr int BM = (ECAP + R - 1) / R;
  const int nbf = (int)fnbf.d;
  const int total = nbf * L;
  const int tstep = (N / (Ns * R)) * twstride;   // twiddle index step per unit of k * r
  V v[BM][R];
#pragma unroll
  for (int b = 0; b < BM; ++b) {
    const int u = tid + b * nthr;
    if (u < total) {
      int l, j;
      if (LINE_FAST) {
        j = (int)fL.div((uint32_t)u);
        l = u - j * L;
      } else {
        l = (int)fnbf.div((uint32_t)u);
        j = u - l * nbf;
      }
      const int g = (int)fNs.div((uint32_t)j);
      const int k = j - g * Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = lds[(j + r * nbf) * istride + l * lstride];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], twiddle<DIR>(tw, k * r * tstep));
      }
      dft_small<R, DIR>(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BM; ++b) {
    const int u = tid + b * nthr;
    if (u < total) {
      int l, j;
      if (LINE_FAST) {
        j = (int)fL.div((uint32_t)u);
        l = u - j * L;
      } else {
        l = (int)fnbf.div((uint32_t)u);
        j = u - l * nbf;
      }
      const int g = (int)fNs.div((uint32_t)j);
      const int k = j - g * Ns;
      const int base = g * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[(base + r * Ns) * istride + l * lstride] = v[b][r];
    }
  }
  __syncthreads();
}

// Full transform of L lines held in LDS (natural order in and out).  The
// caller must have synchronised after filling LDS; on return the results are
// visible to the whole block.  tw holds exp(-2 pi i m / (N * twstride)).
// fL: the line count L with its precomputed constant; every divisor of the
// stages comes with its constant from the plan, so no integer division runs
// on the device.
template <typename T, int DIR, int ECAP, bool LINE_FAST>
__device__ __forceinline__ void mixed_fft(Cx<T>* lds, int N, const FastDiv& fL, int istride, int lstride, const MixedPlan& mp,
                          const Cx<T>* __restrict__ tw, int twstride, int tid, int nthr) {
  const int L = (int)fL.d;
  int Ns = 1;
  for (int s = 0; s < mp.n_st; ++s) {
    const int R = mp.radix[s];
    const FastDiv fNs((uint32_t)Ns, mp.m_ns[s]), fnbf((uint32_t)(N / R), mp.m_nbf[s]);
    switch (R) {
#define DT_MIXED_STAGE(RR)                                                                                     \
      mixed_stage<T, DIR, RR, ECAP, LINE_FAST>(lds, N, L, istride, lstride, Ns, tw, twstride, tid, nthr, fL, fNs, \
                                               fnbf)
      case 8: DT_MIXED_STAGE(8); break;
      case 4: DT_MIXED_STAGE(4); break;
      case 2: DT_MIXED_STAGE(2); break;
      case 7: DT_MIXED_STAGE(7); break;
      case 5: DT_MIXED_STAGE(5); break;
      case 16: DT_MIXED_STAGE(16); break;
      case 6: DT_MIXED_STAGE(6); break;
      case 10: DT_MIXED_STAGE(10); break;
      case 12: DT_MIXED_STAGE(12); break;
      case 14: DT_MIXED_STAGE(14); break;
      case 9: DT_MIXED_STAGE(9); break;
      case 15: DT_MIXED_STAGE(15); break;
      default: DT_MIXED_STAGE(3); break;
#undef DT_MIXED_STAGE
    }
    Ns *= R;
  }
}

}  // namespace dt
