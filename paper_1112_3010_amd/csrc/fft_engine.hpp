// Register + LDS Stockham FFT engine for gfx950 (64-wide wavefronts).
//
// A block transforms several independent lines of length N (a power of two)
// at once.  Each thread owns E consecutive-butterfly slots of one line:
// at a stage of radix R it computes E/R butterflies j = q + Q*s (s < E/R),
// Q = N/E threads per line.  Stages follow the self-sorting (Stockham)
// decimation-in-time ordering: butterfly j of a stage with stride Ns reads
// elements j + r*N/R and writes (j/Ns)*Ns*R + j%Ns + r*Ns, so the output
// needs no bit reversal.  Consecutive stages exchange data through LDS; the
// first stage reads straight from global memory and the last stage leaves its
// outputs in registers at indices j + r*N/R_last.  The radix schedules below
// start and end with radix 8, so a forward transform's output slots are
// exactly the next inverse transform's input slots (used by the fused
// forward-multiply-inverse column pass).
#pragma once

#include <hip/hip_runtime.h>

namespace dt {

template <typename T> struct CxOf;
template <> struct CxOf<float> { using type = float2; };
template <> struct CxOf<double> { using type = double2; };
template <typename T> using Cx = typename CxOf<T>::type;

template <typename V> __device__ __forceinline__ V mk(decltype(V::x) a, decltype(V::x) b) {
  V r; r.x = a; r.y = b; return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return mk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return mk<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return mk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return mk<V>(a.x, -a.y); }
template <typename V> __device__ __forceinline__ V cscale(V a, decltype(V::x) s) { return mk<V>(a.x * s, a.y * s); }
// a * (-i) and a * (+i)
template <typename V> __device__ __forceinline__ V mul_mi(V a) { return mk<V>(a.y, -a.x); }
template <typename V> __device__ __forceinline__ V mul_pi(V a) { return mk<V>(-a.y, a.x); }

// Multiply by (-i)^p, p in [0, 4).
template <typename V> __device__ __forceinline__ V mul_mi_pow(V a, int p) {
  switch (p & 3) {
    case 0: return a;
    case 1: return mul_mi(a);
    case 2: return mk<V>(-a.x, -a.y);
    default: return mul_pi(a);
  }
}

// DIR = +1: forward (kernel exp(-2 pi i/R)); DIR = -1: inverse (unnormalised).
template <int DIR, typename V> __device__ __forceinline__ V rot4(V a) {
  return DIR > 0 ? mul_mi(a) : mul_pi(a);
}
template <int DIR, typename V> __device__ __forceinline__ V rot8_1(V a) {
  using T = decltype(V::x);
  const T c = T(0.70710678118654752440084436210484903928);
  return DIR > 0 ? mk<V>(c * (a.x + a.y), c * (a.y - a.x)) : mk<V>(c * (a.x - a.y), c * (a.x + a.y));
}
template <int DIR, typename V> __device__ __forceinline__ V rot8_3(V a) {
  using T = decltype(V::x);
  const T c = T(0.70710678118654752440084436210484903928);
  return DIR > 0 ? mk<V>(c * (a.y - a.x), -c * (a.x + a.y)) : mk<V>(-c * (a.x + a.y), c * (a.x - a.y));
}

// In-register DFTs, natural order in and out.
template <int R, int DIR, typename V> struct Bfly;

template <int DIR, typename V> struct Bfly<2, DIR, V> {
  static __device__ __forceinline__ void run(V* a) {
    V t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

// 3-point DFT: y0 = a0 + t, y1,2 = a0 - t/2 -+ i DIR (sqrt(3)/2) d with
// t = a1 + a2, d = a1 - a2 (the roots of unity exp(-+2 pi i DIR / 3)).
template <int DIR, typename V> struct Bfly<3, DIR, V> {
  static __device__ __forceinline__ void run(V* a) {
    using T = decltype(V::x);
    const T h = T(0.86602540378443864676372317075293618347);   // sqrt(3) / 2
    const V t = cadd(a[1], a[2]), d = csub(a[1], a[2]);
    const V m = mk<V>(a[0].x - T(0.5) * t.x, a[0].y - T(0.5) * t.y);
    const V s = DIR > 0 ? mk<V>(h * d.y, -h * d.x) : mk<V>(-h * d.y, h * d.x);
    a[0] = cadd(a[0], t);
    a[1] = cadd(m, s);
    a[2] = csub(m, s);
  }
};

template <int DIR, typename V> struct Bfly<4, DIR, V> {
  static __device__ __forceinline__ void run(V* a) {
    V s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    V s13 = cadd(a[1], a[3]), d13 = rot4<DIR>(csub(a[1], a[3]));
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, d13);
    a[3] = csub(d02, d13);
  }
};

template <int DIR, typename V> struct Bfly<8, DIR, V> {
  static __device__ __forceinline__ void run(V* a) {
    // split into even / odd outputs (decimation in frequency), then 4-point DFTs
    V e[4], o[4];
    e[0] = cadd(a[0], a[4]); o[0] = csub(a[0], a[4]);
    e[1] = cadd(a[1], a[5]); o[1] = rot8_1<DIR>(csub(a[1], a[5]));
    e[2] = cadd(a[2], a[6]); o[2] = rot4<DIR>(csub(a[2], a[6]));
    e[3] = cadd(a[3], a[7]); o[3] = rot8_3<DIR>(csub(a[3], a[7]));
    Bfly<4, DIR, V>::run(e);
    Bfly<4, DIR, V>::run(o);
    a[0] = e[0]; a[2] = e[1]; a[4] = e[2]; a[6] = e[3];
    a[1] = o[0]; a[3] = o[1]; a[5] = o[2]; a[7] = o[3];
  }
};

// Radix schedules (first and last stage radix 8 for power-of-two N >= 64;
// 144 = 12 x 12 and 196 = 14 x 14 for the rows of 288- and 392-point padded
// axes).
__host__ __device__ constexpr int fft_stages(int N) {
  return N == 144 || N == 196 ? 2 : N <= 64 ? 2 : (N <= 512 ? 3 : 4);
}
__host__ __device__ constexpr int fft_radix(int N, int s) {
  return N == 144 ? 12
       : N == 196 ? 14
       : N == 16 ? 4
       : N == 32 ? (s == 0 ? 8 : 4)
       : N == 64 ? 8
       : N == 128 ? (s == 1 ? 2 : 8)
       : N == 256 ? (s == 1 ? 4 : 8)
       : N == 512 ? 8
       : N == 1024 ? ((s == 1 || s == 2) ? 4 : 8)
       : N == 2048 ? (s == 1 ? 4 : 8)
       : 8;
}
__host__ __device__ constexpr int fft_stride(int N, int s) {  // product of earlier radices
  return s == 0 ? 1 : fft_stride(N, s - 1) * fft_radix(N, s - 1);
}

// Twiddle exp(-2 pi i DIR m / L) from a table of exp(-2 pi i m / L).
template <int DIR, typename V> __device__ __forceinline__ V twiddle(const V* tw, int m) {
  V w = tw[m];
  return DIR > 0 ? w : cconj(w);
}

// Elements per thread of the row passes: whole butterflies of every stage.
__host__ __device__ constexpr int row_E(int N) { return N == 144 ? 12 : N == 196 ? 14 : 8; }

// Per-thread view of one line.  Addr maps a within-line index to an LDS slot.
template <typename T, int N, int E, int DIR> struct Stockham {
  using V = Cx<T>;
  static constexpr int Q = N / E;
  static constexpr int S = fft_stages(N);
  static_assert(E % 8 == 0 || (N == 16 && E % 4 == 0) || (N == 144 && E == 12) || (N == 196 && E == 14),
                "elements per thread must hold whole butterflies");

  // Index of slot (s, r) for the input of stage `st` (or the output of the last stage).
  template <int st> static __device__ __forceinline__ int in_index(int q, int s, int r) {
    constexpr int R = fft_radix(N, st);
    return (q + Q * s) + r * (N / R);
  }
  template <int st> static __device__ __forceinline__ int out_index(int q, int s, int r) {
    constexpr int R = fft_radix(N, st);
    constexpr int Ns = fft_stride(N, st);
    const int j = q + Q * s;
    return (j / Ns) * Ns * R + (j % Ns) + r * Ns;
  }

  template <int st> static __device__ __forceinline__ void compute(V* v, int q, const V* tw, int tws) {
    constexpr int R = fft_radix(N, st);
    constexpr int Ns = fft_stride(N, st);
#pragma unroll
    for (int s = 0; s < E / R; ++s) {
      if constexpr (Ns > 1) {
        const int j = q + Q * s;
        const int step = (j % Ns) * (N / (Ns * R)) * tws;
#pragma unroll
        for (int r = 1; r < R; ++r) v[s * R + r] = cmul(v[s * R + r], twiddle<DIR>(tw, r * step));
      }
      Bfly<R, DIR, V>::run(&v[s * R]);
    }
  }

  template <int st, class Addr> static __device__ __forceinline__ void store(V* lds, const V* v, int q, Addr addr) {
    constexpr int R = fft_radix(N, st);
#pragma unroll
    for (int s = 0; s < E / R; ++s)
#pragma unroll
      for (int r = 0; r < R; ++r) lds[addr(out_index<st>(q, s, r))] = v[s * R + r];
  }

  template <int st, class Addr> static __device__ __forceinline__ void load(const V* lds, V* v, int q, Addr addr) {
    constexpr int R = fft_radix(N, st);
#pragma unroll
    for (int s = 0; s < E / R; ++s)
#pragma unroll
      for (int r = 0; r < R; ++r) v[s * R + r] = lds[addr(in_index<st>(q, s, r))];
  }

  // Stages 1..S-1 after stage 0's inputs are in registers; leaves the last
  // stage's outputs in registers.  All threads of the block must call this.
  template <int st, class Addr>
  static __device__ __forceinline__ void run_from(V* v, V* lds, int q, const V* tw, int tws, Addr addr) {
    compute<st>(v, q, tw, tws);
    if constexpr (st + 1 < S) {
      __syncthreads();
      store<st>(lds, v, q, addr);
      __syncthreads();
      load<st + 1>(lds, v, q, addr);
      run_from<st + 1>(v, lds, q, tw, tws, addr);
    }
  }

  template <class Addr>
  static __device__ __forceinline__ void run(V* v, V* lds, int q, const V* tw, int tws, Addr addr) {
    run_from<0>(v, lds, q, tw, tws, addr);
  }

  // Write the last stage's outputs (natural order) to LDS.
  template <class Addr> static __device__ __forceinline__ void store_last(V* lds, const V* v, int q, Addr addr) {
    store<S - 1>(lds, v, q, addr);
  }
};

}  // namespace dt
