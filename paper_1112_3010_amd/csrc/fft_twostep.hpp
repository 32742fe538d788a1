// Two-step register FFT for column tiles (gfx950).
//
// A length-N transform with N = E * P is split the classic four-step way:
// each of the P threads that share a column holds the E samples
// x[p + P e] (e < E) and transforms them in registers (size-E DFT with
// compile-time twiddles), multiplies by the thread twiddles W_N^(p k1),
// exchanges through LDS once, and finishes with E/P register DFTs of size P.
// Output slot (t, k2) of thread p holds X[(p + P t) + E k2].  The inverse
// runs the same steps backwards from those slots and ends with the natural
// sample order x[p + P n2] in registers, so a forward transform's outputs are
// exactly the inverse's inputs (used by the fused multiply pass).
//
// Compared with a radix-8 Stockham sequence this needs one LDS exchange per
// transform instead of N's stage count minus one, all LDS offsets are
// compile-time immediates, and only E/8 + 7 thread twiddles are loaded per
// kernel.
#pragma once

#include <type_traits>

#include "fft_engine.hpp"

namespace dt {

// ---------------------------------------------------------------------------
// Compile-time cos/sin of 2 pi m / R (octant reduction in exact integer
// arithmetic, then a Taylor series on [0, pi/4] in double precision).
// ---------------------------------------------------------------------------
constexpr double kPiCT = 3.14159265358979323846264338327950288;

constexpr double ct_taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
constexpr double ct_taylor_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi m / R for integers m, R > 0
constexpr double ct_cos2pi(long m, long R) {
  m = ((m % R) + R) % R;
  const long e8 = m * 8;
  const long oct = e8 / R;
  const long rem = e8 % R;
  const double a = (kPiCT / 4.0) * (double)rem / (double)R;
  const double b = (kPiCT / 4.0) * (double)(R - rem) / (double)R;
  switch (oct) {
    case 0: return ct_taylor_cos(a);
    case 1: return ct_taylor_sin(b);
    case 2: return -ct_taylor_sin(a);
    case 3: return -ct_taylor_cos(b);
    case 4: return -ct_taylor_cos(a);
    case 5: return -ct_taylor_sin(b);
    case 6: return ct_taylor_sin(a);
    default: return ct_taylor_cos(b);
  }
}
constexpr double ct_sin2pi(long m, long R) {
  m = ((m % R) + R) % R;
  const long e8 = m * 8;
  const long oct = e8 / R;
  const long rem = e8 % R;
  const double a = (kPiCT / 4.0) * (double)rem / (double)R;
  const double b = (kPiCT / 4.0) * (double)(R - rem) / (double)R;
  switch (oct) {
    case 0: return ct_taylor_sin(a);
    case 1: return ct_taylor_cos(b);
    case 2: return ct_taylor_cos(a);
    case 3: return ct_taylor_sin(b);
    case 4: return -ct_taylor_sin(a);
    case 5: return -ct_taylor_cos(b);
    case 6: return -ct_taylor_cos(a);
    default: return -ct_taylor_sin(b);
  }
}

// a * exp(-2 pi i DIR m / R) with m, R compile-time; trivial angles are
// rotations and cost no multiplications.
template <int DIR, int M, int R, typename V> __device__ __forceinline__ V cmul_w(V a) {
  using T = decltype(V::x);
  constexpr int m = ((M % R) + R) % R;
  if constexpr (m == 0) {
    return a;
  } else if constexpr ((4 * m) % R == 0) {
    constexpr int q = (4 * m) / R;  // multiple of a quarter turn
    return mul_mi_pow(a, DIR > 0 ? q : (4 - q) & 3);
  } else if constexpr ((8 * m) % R == 0 && ((8 * m) / R) % 2 == 1) {
    constexpr int o = (8 * m) / R;  // odd multiple of an eighth turn
    const V r = (o == 1 || o == 5) ? rot8_1<DIR>(a) : rot8_3<DIR>(a);
    return (o >= 4) ? mk<V>(-r.x, -r.y) : r;
  } else {
    constexpr T c = (T)ct_cos2pi(m, R);
    constexpr T s = (T)(DIR > 0 ? -ct_sin2pi(m, R) : ct_sin2pi(m, R));
    return mk<V>(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// Odd prime-length DFT (5, 7) from the pairs (a_j, a_(R-j)): with
// t_j = a_j + a_(R-j), d_j = a_j - a_(R-j) and theta = 2 pi j k / R,
//   y_k, y_(R-k) = a_0 + sum_j t_j cos(theta) -+ i DIR sum_j d_j sin(theta).
template <int R, int DIR, typename V> __device__ __forceinline__ void odd_prime_dft(V* a) {
  using T = decltype(V::x);
  constexpr int H = (R - 1) / 2;
  V t[H + 1], d[H + 1];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    t[j] = cadd(a[j], a[R - j]);
    d[j] = csub(a[j], a[R - j]);
  }
  const V a0 = a[0];
  V s0 = a0;
#pragma unroll
  for (int j = 1; j <= H; ++j) s0 = cadd(s0, t[j]);
  a[0] = s0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    V re = a0, im = mk<V>(T(0), T(0));
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const T c = (T)ct_cos2pi((long)j * k, R), sn = (T)ct_sin2pi((long)j * k, R);
      re = mk<V>(fma(c, t[j].x, re.x), fma(c, t[j].y, re.y));
      im = mk<V>(fma(sn, d[j].x, im.x), fma(sn, d[j].y, im.y));
    }
    // -i DIR im
    const V r = DIR > 0 ? mk<V>(im.y, -im.x) : mk<V>(-im.y, im.x);
    a[k] = cadd(re, r);
    a[R - k] = csub(re, r);
  }
}
template <int DIR, typename V> struct Bfly<5, DIR, V> {
  static __device__ __forceinline__ void run(V* a) { odd_prime_dft<5, DIR, V>(a); }
};
template <int DIR, typename V> struct Bfly<7, DIR, V> {
  static __device__ __forceinline__ void run(V* a) { odd_prime_dft<7, DIR, V>(a); }
};

// In-register DFT of size R, natural order in and out, R a 7-smooth number
// up to 64: R = R1 x R2 Cooley-Tukey with compile-time twiddles W_R^(n1 k2),
// down to the butterflies of size 2, 3, 4, 5, 7 and 8.
template <int R, int DIR, typename V> struct RegDFT {
  // 12 = 4 x 3, 14 = 2 x 7, 15 = 3 x 5, 16 = 4 x 4, 25 = 5 x 5, 32 = 8 x 4, 64 = 8 x 8
  static constexpr int R1 = (R >= 32 && R % 8 == 0) ? 8
                          : R % 4 == 0 ? 4 : R % 2 == 0 ? 2 : R % 3 == 0 ? 3 : R % 5 == 0 ? 5 : 7;
  static constexpr bool LEAF = R == 2 || R == 3 || R == 4 || R == 5 || R == 7 || R == 8;
  static constexpr int R2 = R / R1;

  template <int N1, int K2> static __device__ __forceinline__ void twiddle(const V* t, V* b) {
    if constexpr (K2 < R2) {
      b[N1 * R2 + K2] = cmul_w<DIR, N1 * K2, R>(t[K2]);
      twiddle<N1, K2 + 1>(t, b);
    }
  }
  template <int N1> static __device__ __forceinline__ void step1(const V* a, V* b) {
    if constexpr (N1 < R1) {
      V t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = a[N1 + R1 * n2];
      RegDFT<R2, DIR, V>::run(t);
      twiddle<N1, 0>(t, b);
      step1<N1 + 1>(a, b);
    }
  }
  static __device__ __forceinline__ void run(V* a) {
    if constexpr (LEAF) {
      Bfly<R, DIR, V>::run(a);
    } else {
      V b[R];
      step1<0>(a, b);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        V t[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) t[n1] = b[n1 * R2 + k2];
        RegDFT<R1, DIR, V>::run(t);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) a[k2 + R2 * k1] = t[k1];
      }
    }
  }
};

// The 12- and 14-point DFTs as butterflies of the Stockham engine (rows of
// length 144 and 196).
template <int DIR, typename V> struct Bfly<12, DIR, V> {
  static __device__ __forceinline__ void run(V* a) { RegDFT<12, DIR, V>::run(a); }
};
template <int DIR, typename V> struct Bfly<14, DIR, V> {
  static __device__ __forceinline__ void run(V* a) { RegDFT<14, DIR, V>::run(a); }
};

// Thread twiddles W_N^(DIR p k) for k < E from two small sets:
// k = a + 8 b, W^(p k) = W^(p a) W^(8 p b).
template <typename T, int N, int E> struct ThreadTwiddles {
  using V = Cx<T>;
  static constexpr bool NEEDS_BARRIER = false;
  static constexpr int NB8 = (E + 7) / 8;
  V A[8];
  V B[NB8 > 0 ? NB8 : 1];
  __device__ __forceinline__ void load(const V* tw, int p) {
    A[0] = mk<V>(T(1), T(0));
#pragma unroll
    for (int a = 1; a < 8; ++a) A[a] = tw[(p * a) % N];
    B[0] = mk<V>(T(1), T(0));
#pragma unroll
    for (int b = 1; b < NB8; ++b) B[b] = tw[(p * 8 * b) % N];
  }
  // W_N^(p k) (forward sign); the inverse uses the conjugate
  __device__ __forceinline__ V get(int k) const {
    const int a = k & 7, b = k >> 3;
    if (b == 0) return A[a];
    if (a == 0) return B[b];
    return cmul(A[a], B[b]);
  }
};

template <typename T, int N, int E_, int NB> struct TwoStep {
  using V = Cx<T>;
  static constexpr int E = E_;
  static constexpr int P = N / E;
  using Tw = ThreadTwiddles<T, N, E>;
  static_assert(E >= P && E % P == 0, "each thread must own whole second-step DFTs");
  static constexpr int PAD = 16;                           // LDS padding (complex) per row group
  static constexpr int LDS_F = E * (P * NB + PAD);         // forward exchange footprint
  static constexpr int LDS_I = P * (E * NB + PAD);         // inverse exchange footprint
  static constexpr int LDS = LDS_F > LDS_I ? LDS_F : LDS_I;

  // Forward: v[e] = x[p + P e] on entry; on exit v[t * P + k2] = X[(p + P t) + E k2].
  static __device__ __forceinline__ void forward(V* v, V* lds, int p, int b, const ThreadTwiddles<T, N, E>& tw) {
    RegDFT<E, +1, V>::run(v);
#pragma unroll
    for (int k = 1; k < E; ++k) v[k] = cmul(v[k], tw.get(k));
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) lds[k * (P * NB + PAD) + p * NB + b] = v[k];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < E / P; ++t)
#pragma unroll
      for (int pp = 0; pp < P; ++pp) v[t * P + pp] = lds[(p + P * t) * (P * NB + PAD) + pp * NB + b];
#pragma unroll
    for (int t = 0; t < E / P; ++t) RegDFT<P, +1, V>::run(&v[t * P]);
  }

  // Inverse (unnormalised): v[t * P + k2] = X[(p + P t) + E k2] on entry;
  // on exit v[n2] = x[p + P n2].
  static __device__ __forceinline__ void inverse(V* v, V* lds, int p, int b, const ThreadTwiddles<T, N, E>& tw) {
#pragma unroll
    for (int t = 0; t < E / P; ++t) RegDFT<P, -1, V>::run(&v[t * P]);
    // twiddle W_N^(-n1 (p + P t)) = conj(W_N^(n1 p)) * W_E^(-n1 t)
#pragma unroll
    for (int t = 0; t < E / P; ++t)
#pragma unroll
      for (int n1 = 1; n1 < P; ++n1) v[t * P + n1] = cmul(v[t * P + n1], cconj(tw.get(n1)));
    apply_const_tw<1>(v);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < E / P; ++t)
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) lds[n1 * (E * NB + PAD) + (p + P * t) * NB + b] = v[t * P + n1];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = lds[p * (E * NB + PAD) + k * NB + b];
    RegDFT<E, -1, V>::run(v);
  }

  // Same transforms with the LDS exchange done in two rounds (real parts,
  // then imaginary parts) through a real buffer of LDS elements: half the
  // LDS footprint for two more barriers.
  static __device__ __forceinline__ void exchange_f(V* v, T* ldsr, int p, int b) {
    constexpr int RS = P * NB + PAD;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) ldsr[k * RS + p * NB + b] = v[k].x;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < E / P; ++t)
#pragma unroll
      for (int pp = 0; pp < P; ++pp) v[t * P + pp].x = ldsr[(p + P * t) * RS + pp * NB + b];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) ldsr[k * RS + p * NB + b] = v[k].y;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < E / P; ++t)
#pragma unroll
      for (int pp = 0; pp < P; ++pp) v[t * P + pp].y = ldsr[(p + P * t) * RS + pp * NB + b];
  }
  static __device__ __forceinline__ void forward_split(V* v, T* ldsr, int p, int b,
                                                       const ThreadTwiddles<T, N, E>& tw) {
    RegDFT<E, +1, V>::run(v);
#pragma unroll
    for (int k = 1; k < E; ++k) v[k] = cmul(v[k], tw.get(k));
    exchange_f(v, ldsr, p, b);
#pragma unroll
    for (int t = 0; t < E / P; ++t) RegDFT<P, +1, V>::run(&v[t * P]);
  }
  static __device__ __forceinline__ void inverse_split(V* v, T* ldsr, int p, int b,
                                                       const ThreadTwiddles<T, N, E>& tw) {
    constexpr int RS = E * NB + PAD;
#pragma unroll
    for (int t = 0; t < E / P; ++t) RegDFT<P, -1, V>::run(&v[t * P]);
#pragma unroll
    for (int t = 0; t < E / P; ++t)
#pragma unroll
      for (int n1 = 1; n1 < P; ++n1) v[t * P + n1] = cmul(v[t * P + n1], cconj(tw.get(n1)));
    apply_const_tw<1>(v);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < E / P; ++t)
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) ldsr[n1 * RS + (p + P * t) * NB + b] = v[t * P + n1].x;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k].x = ldsr[p * RS + k * NB + b];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < E / P; ++t)
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) ldsr[n1 * RS + (p + P * t) * NB + b] = v[t * P + n1].y;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k].y = ldsr[p * RS + k * NB + b];
    RegDFT<E, -1, V>::run(v);
  }

  // multiply slot (t, n1) by W_E^(-n1 t) for t >= 1 (compile-time)
  template <int TT> static __device__ __forceinline__ void apply_const_tw(V* v) {
    if constexpr (TT < E / P) {
      apply_const_tw_n1<TT, 1>(v);
      apply_const_tw<TT + 1>(v);
    }
  }
  template <int TT, int N1> static __device__ __forceinline__ void apply_const_tw_n1(V* v) {
    if constexpr (N1 < P) {
      v[TT * P + N1] = cmul_w<-1, N1 * TT, E>(v[TT * P + N1]);
      apply_const_tw_n1<TT, N1 + 1>(v);
    }
  }

  // Spectral index held in forward-output slot (t, k2) of thread p.
  static __device__ __forceinline__ int slot_index(int p, int t, int k2) { return (p + P * t) + E * k2; }
  static __device__ __forceinline__ int slot(int p, int i) { return slot_index(p, i / P, i % P); }
  static constexpr bool LINEAR_FOLD = false;
  static constexpr bool PAIR_PRODUCT = false;
};

// ---------------------------------------------------------------------------
// Pair-split four-step FFT for N = E * P with P = 2E (32, 128, 288, 392,
// 512, 2048).
//
// Thread p < P of a column holds x[p + P e] (e < E).  Step 1: size-E DFT in
// registers and the thread twiddles W_N^(p k1).  One LDS exchange gives
// thread q = 2 k1 + h the values of k1 at p = 2m + h (m < E); a size-E DFT
// over m is half of the size-P DFT over p, and the two halves are joined by
// one radix-2 step between the lane pair (q, q ^ 1) through cross-lane
// shuffles:  X[k1 + E j + (N/2) h] = Z_0[j] + (-1)^h W_2E^j Z_1[j].
// With E = N/P = sqrt(N/2) elements per thread instead of the two-step
// engine's E >= sqrt(N), the per-thread register footprint halves at
// N = 512.  The inverse runs the adjoint steps in reverse order and ends
// with x[p + P e] in registers, so forward outputs are inverse inputs.
// The exchange is done in two rounds (real, then imaginary parts) through a
// real LDS buffer of LDS elements.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int pair_E(int N) {
  return N == 32 ? 4 : N == 128 ? 8 : N == 288 ? 12 : N == 392 ? 14 : N == 512 ? 16 : N == 2048 ? 32 : 0;
}

template <typename T, int N, int NB, int SPLIT = 0, bool TWL = false> struct PairFFT {
  using V = Cx<T>;
  static constexpr int E = pair_E(N);
  static constexpr int P = 2 * E;
  static_assert(E > 0 && E * P == N, "pair split needs N = 2 E^2");
  static_assert(NB <= 32 && (NB & (NB - 1)) == 0, "lane pairs (q, q ^ 1) must share a wavefront");
  // row stride of the exchange buffer (elements of the exchanged type): the
  // padding puts the two rows that a half-wave reads on disjoint banks
  static constexpr int PAD = SPLIT ? 32 : 16;
  static constexpr int RS = P * NB + PAD;
  static constexpr int LDS = E * RS * (SPLIT ? 1 : 2);   // reals
  // all E - 1 thread twiddles W_N^(p k), k = 1 .. E-1, formed once per block
  struct TwReg {
    static constexpr bool NEEDS_BARRIER = false;
    V w[E];
    __device__ __forceinline__ void load(const V* tw, int p) {
      ThreadTwiddles<T, N, E> ab;
      ab.load(tw, p);
#pragma unroll
      for (int k = 0; k < E; ++k) w[k] = ab.get(k);
    }
    __device__ __forceinline__ V get(int k) const { return w[k]; }
  };
  // The same twiddles in an LDS table (row p, odd row stride), read at each
  // use: frees 2E registers per thread.  The block fills the table together,
  // so a barrier must pass before the first get.
  struct TwLds {
    static constexpr bool NEEDS_BARRIER = true;
    const V* row;
    __device__ __forceinline__ void load(const V* tw, int p) {
      __shared__ V tab[P * (E + 1)];
      for (int i = threadIdx.x; i < P * E; i += blockDim.x) {
        const int r = i / E, k = i % E;
        tab[r * (E + 1) + k] = tw[(r * k) % N];
      }
      row = tab + p * (E + 1);
    }
    __device__ __forceinline__ V get(int k) const { return row[k]; }
  };
  using Tw = typename std::conditional<TWL, TwLds, TwReg>::type;

  template <int DIR, int J> static __device__ __forceinline__ void pair_twiddle(V* v, bool h) {
    if constexpr (J < E) {
      const V w = cmul_w<DIR, J, 2 * E>(v[J]);
      v[J].x = h ? w.x : v[J].x;    // component-wise: a select of whole structs goes through memory
      v[J].y = h ? w.y : v[J].y;
      pair_twiddle<DIR, J + 1>(v, h);
    }
  }
  // value of lane ^ NB.  For NB = 8 the partner sits in the other half of the
  // same 16-lane row: a DPP row rotate by 8 (a plain VALU move); otherwise a
  // cross-lane permute.
  static __device__ __forceinline__ int lane_xor_i(int x) {
    if constexpr (NB == 8) return __builtin_amdgcn_mov_dpp(x, 0x128 /* row_ror:8 */, 0xF, 0xF, false);
    else return __shfl_xor(x, NB);
  }
  static __device__ __forceinline__ float lane_xor(float x) { return __int_as_float(lane_xor_i(__float_as_int(x))); }
  static __device__ __forceinline__ double lane_xor(double x) {
    const int hi = lane_xor_i(__double2hiint(x));
    const int lo = lane_xor_i(__double2loint(x));
    return __hiloint2double(hi, lo);
  }
  // v[j] <- Z0 + (-1)^h Z1 where this lane holds Z_h and its partner Z_(1-h):
  // lane 0 adds the partner's value, lane 1 subtracts its own from it, i.e.
  // v <- sgn v + partner with sgn = (-1)^h (one FMA per component, no select)
  static __device__ __forceinline__ void pair_join(V* v, bool h) {
    const T sgn = h ? T(-1) : T(1);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const T ox = lane_xor(v[j].x);
      const T oy = lane_xor(v[j].y);
      v[j].x = fma(sgn, v[j].x, ox);
      v[j].y = fma(sgn, v[j].y, oy);
    }
  }
  // (k1, p) -> (p >> 1, 2 m + (p & 1)) for the forward direction; reversed for the inverse
  template <bool FWD> static __device__ __forceinline__ void exchange(V* v, T* ldsr, int p, int b) {
    const int rq = (p >> 1) * RS + (p & 1) * NB + b;   // read base of the forward direction
    const int wp = p * NB + b;
    if constexpr (SPLIT == 0) {
      // whole complex values in one round (needs LDS complex elements)
      V* lds = reinterpret_cast<V*>(ldsr);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; ++k) {
        if (FWD) lds[k * RS + wp] = v[k];
        else lds[rq + 2 * k * NB] = v[k];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = FWD ? lds[rq + 2 * k * NB] : lds[k * RS + wp];
      return;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) {
      if (FWD) ldsr[k * RS + wp] = v[k].x;
      else ldsr[rq + 2 * k * NB] = v[k].x;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k].x = FWD ? ldsr[rq + 2 * k * NB] : ldsr[k * RS + wp];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) {
      if (FWD) ldsr[k * RS + wp] = v[k].y;
      else ldsr[rq + 2 * k * NB] = v[k].y;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k].y = FWD ? ldsr[rq + 2 * k * NB] : ldsr[k * RS + wp];
  }

  // Forward: v[e] = x[p + P e] on entry; on exit v[j] = X[slot(p, j)].
  static __device__ __forceinline__ void forward_split(V* v, T* ldsr, int p, int b, const Tw& tw) {
    RegDFT<E, +1, V>::run(v);
#pragma unroll
    for (int k = 1; k < E; ++k) v[k] = cmul(v[k], tw.get(k));
    exchange<true>(v, ldsr, p, b);
    RegDFT<E, +1, V>::run(v);
    const bool h = (p & 1) != 0;
    pair_twiddle<+1, 0>(v, h);
    pair_join(v, h);
  }
  // Inverse (unnormalised): v[j] = X[slot(p, j)] on entry; on exit v[e] = x[p + P e].
  static __device__ __forceinline__ void inverse_split(V* v, T* ldsr, int p, int b, const Tw& tw) {
    const bool h = (p & 1) != 0;
    pair_join(v, h);
    pair_twiddle<-1, 0>(v, h);
    RegDFT<E, -1, V>::run(v);
    exchange<false>(v, ldsr, p, b);
#pragma unroll
    for (int k = 1; k < E; ++k) v[k] = cmul(v[k], cconj(tw.get(k)));
    RegDFT<E, -1, V>::run(v);
  }
  // --- The kernel-spectrum product taken in the pair basis -----------------
  // After the second size-E DFT, lane h of the pair (2 k1, 2 k1 + 1) holds
  // Z_h[j]; the forward transform then forms X_h = Z_0 + (-1)^h W^j Z_1
  // (W = W_2E), the product is Y_h = K_h X_h with K_h the kernel spectrum at
  // the lane's slot, and the inverse starts with the same butterfly and the
  // conjugate twiddle on lane 1.  Composed, those steps are
  //   Z'_h = (K_0 + K_1) Z_h + (K_0 - K_1) U_h,
  //   U_0 = W^j Z_1,  U_1 = W^-j Z_0,
  // so the partner's half is fetched and twiddled once per column (cross)
  // and each kernel costs two real-by-complex products per slot.
  // float64 keeps the plain product: the 16 extra complex registers of the
  // partner's half would spill at N = 512
  static constexpr bool PAIR_PRODUCT = sizeof(T) == 4;
  // Forward up to the lane butterfly: on exit v[j] = Z_h[j].
  static __device__ __forceinline__ void forward_half(V* v, T* ldsr, int p, int b, const Tw& tw) {
    RegDFT<E, +1, V>::run(v);
#pragma unroll
    for (int k = 1; k < E; ++k) v[k] = cmul(v[k], tw.get(k));
    exchange<true>(v, ldsr, p, b);
    RegDFT<E, +1, V>::run(v);
  }
  template <int J> static __device__ __forceinline__ void cross_j(const V* z, V* u, T sg) {
    if constexpr (J < E) {
      const T zx = lane_xor(z[J].x);
      const T zy = lane_xor(z[J].y);
      if constexpr (J == 0) {
        u[J] = mk<V>(zx, zy);
      } else if constexpr (2 * J == E) {
        // W^(+-E/2) = -+i
        u[J] = mk<V>(sg * zy, -sg * zx);
      } else {
        // lane 0: W^J = (c, -s); lane 1: W^-J = (c, s)
        constexpr T c = (T)ct_cos2pi(J, 2 * E);
        constexpr T s = (T)ct_sin2pi(J, 2 * E);
        const T ss = sg * s;
        u[J] = mk<V>(fma(c, zx, ss * zy), fma(c, zy, -ss * zx));
      }
      cross_j<J + 1>(z, u, sg);
    }
  }
  // u[j] = U_h[j] from the pair's halves z
  static __device__ __forceinline__ void cross(const V* z, V* u, int p) {
    cross_j<0>(z, u, (p & 1) ? T(-1) : T(1));
  }
  // Inverse (unnormalised) from v[j] = Z'_h[j]; on exit v[e] = x[p + P e].
  static __device__ __forceinline__ void inverse_half(V* v, T* ldsr, int p, int b, const Tw& tw) {
    RegDFT<E, -1, V>::run(v);
    exchange<false>(v, ldsr, p, b);
#pragma unroll
    for (int k = 1; k < E; ++k) v[k] = cmul(v[k], cconj(tw.get(k)));
    RegDFT<E, -1, V>::run(v);
  }

  static __device__ __forceinline__ int slot(int p, int j) { return (p >> 1) + E * j + (N / 2) * (p & 1); }
  // Folded index |k| of slot j is linear in j: lanes with h = 0 hold k < N/2,
  // lanes with h = 1 hold k >= N/2 (negative frequencies; k = N/2 is the
  // Nyquist index, where every odd kernel spectrum vanishes).
  static constexpr bool LINEAR_FOLD = true;
  static __device__ __forceinline__ int fold_base(int p) { return (p & 1) ? N / 2 - (p >> 1) : (p >> 1); }
  static __device__ __forceinline__ int fold_step(int p) { return (p & 1) ? -E : E; }
  static __device__ __forceinline__ bool fold_neg(int p) { return (p & 1) != 0; }
};

}  // namespace dt
