// Quad-double arithmetic for the widest extended-precision pipeline.
//
// A value is the unevaluated sum x0 + x1 + x2 + x3 of four float64 numbers,
// each at most half an ulp of the one before (about 212 significand bits).
// The operations follow the quad-double algorithms of Hida, Li and Bailey
// (2000/2001: "Algorithms for quad-double precision floating point
// arithmetic", and the QD library report): the four parts are combined term
// by term with TwoSum / TwoProd, the error terms of each order are gathered
// with three-term sums, and a final renormalisation restores the
// non-overlapping form.  Addition is the variant whose error is bounded
// relative to |a| + |b| (the bound the FFT's normwise analysis uses);
// products drop the terms below order four.  Division takes five quotient
// digits; sqrt, exp and sin/cos use argument reduction, Taylor series by
// Horner's rule and Newton steps in this arithmetic.
//
// The functions are usable on the host as well, so that the arithmetic can be
// checked against exact rational arithmetic on the CPU.  As for the
// double-double header, every rounding must happen as written: files that
// include it are compiled with -ffp-contract=off.
#pragma once
#include <hip/hip_runtime.h>

#include "dd.hpp"

#pragma clang fp contract(off)

namespace dt {
namespace ddm {

struct qd {
  double x0, x1, x2, x3;
};

// 2 pi and ln 2 to four float64 parts (each part the float64 nearest the
// remainder of the constant after the parts before it; from exact rational
// series: Machin's formula for pi, sum 1/(k 2^k) for ln 2).
constexpr double kTwoPi2 = -0x1.f1976b7ed8fbcp-108, kTwoPi3 = 0x1.4cf98e804177dp-162;
constexpr double kLn2_2 = 0x1.7b57a079a1934p-111, kLn2_3 = -0x1.ace93a4ebe5d1p-165;

__host__ __device__ __forceinline__ void q_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
// requires |a| >= |b| (or a == 0)
__host__ __device__ __forceinline__ void q_fast_sum(double a, double b, double& s, double& e) {
  s = a + b;
  e = b - (s - a);
}
__host__ __device__ __forceinline__ void q_two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = __builtin_fma(a, b, -p);
}
// (a, b, c) <- (a + b + c, and two error terms): a becomes the rounded sum
__host__ __device__ __forceinline__ void q_three_sum(double& a, double& b, double& c) {
  double t1, t2, t3;
  q_two_sum(a, b, t1, t2);
  q_two_sum(c, t1, a, t3);
  q_two_sum(t2, t3, b, c);
}
// the same with the two error terms folded into b
__host__ __device__ __forceinline__ void q_three_sum2(double& a, double& b, double c) {
  double t1, t2, t3;
  q_two_sum(a, b, t1, t2);
  q_two_sum(c, t1, a, t3);
  b = t2 + t3;
}

// Five roughly ordered terms (|c_i| decreasing, possibly overlapping) to four
// non-overlapping parts.  A bottom-up pass of fast sums makes c0 the rounded
// total with c1 its error; the top-down pass then gathers the lower terms
// into the next parts, starting a new part only where a sum leaves a nonzero
// error, so that exact zeros never sit between two parts.
__host__ __device__ inline qd renorm(double c0, double c1, double c2, double c3, double c4) {
  double s;
  q_fast_sum(c3, c4, s, c4);
  q_fast_sum(c2, s, s, c3);
  q_fast_sum(c1, s, s, c2);
  q_fast_sum(c0, s, c0, c1);
  double s0 = c0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (c1 != 0.0) {
    q_fast_sum(c1, c2, s1, s2);
    if (s2 != 0.0) {
      q_fast_sum(s2, c3, s2, s3);
      if (s3 != 0.0) s3 += c4;
      else q_fast_sum(s2, c4, s2, s3);
    } else {
      q_fast_sum(s1, c3, s1, s2);
      if (s2 != 0.0) q_fast_sum(s2, c4, s2, s3);
      else q_fast_sum(s1, c4, s1, s2);
    }
  } else {
    q_fast_sum(s0, c2, s0, s1);
    if (s1 != 0.0) {
      q_fast_sum(s1, c3, s1, s2);
      if (s2 != 0.0) q_fast_sum(s2, c4, s2, s3);
      else q_fast_sum(s1, c4, s1, s2);
    } else {
      q_fast_sum(s0, c3, s0, s1);
      if (s1 != 0.0) q_fast_sum(s1, c4, s1, s2);
      else q_fast_sum(s0, c4, s0, s1);
    }
  }
  return {s0, s1, s2, s3};
}

__host__ __device__ __forceinline__ qd neg(qd a) { return {-a.x0, -a.x1, -a.x2, -a.x3}; }

__host__ __device__ inline qd add(qd a, qd b) {
  double s0, s1, s2, s3, t0, t1, t2, t3;
  q_two_sum(a.x0, b.x0, s0, t0);
  q_two_sum(a.x1, b.x1, s1, t1);
  q_two_sum(a.x2, b.x2, s2, t2);
  q_two_sum(a.x3, b.x3, s3, t3);
  // order 1: s1 + t0; order 2: s2 + t0' + t1; order 3: s3 + the rest
  q_two_sum(s1, t0, s1, t0);
  q_three_sum(s2, t0, t1);
  q_three_sum2(s3, t0, t2);
  t0 = t0 + t1 + t3;
  return renorm(s0, s1, s2, s3, t0);
}

__host__ __device__ __forceinline__ qd sub(qd a, qd b) { return add(a, neg(b)); }

__host__ __device__ inline qd mul(qd a, qd b) {
  double p0, p1, p2, p3, p4, p5, q0, q1, q2, q3, q4, q5;
  q_two_prod(a.x0, b.x0, p0, q0);   // order 0 (and its error, order 1)
  q_two_prod(a.x0, b.x1, p1, q1);   // order 1
  q_two_prod(a.x1, b.x0, p2, q2);
  q_two_prod(a.x0, b.x2, p3, q3);   // order 2
  q_two_prod(a.x1, b.x1, p4, q4);
  q_two_prod(a.x2, b.x0, p5, q5);
  // order 1: p1 + p2 + q0 -> p1 (p2, q0 move to order 2)
  q_three_sum(p1, p2, q0);
  // order 2: p2 + q1 + q2 + p3 + p4 + p5 -> s0 (s1, s2 lower)
  q_three_sum(p2, q1, q2);
  q_three_sum(p3, p4, p5);
  double s0, s1, s2, t0, t1;
  q_two_sum(p2, p3, s0, t0);
  q_two_sum(q1, p4, s1, t1);
  s2 = q2 + p5;
  q_two_sum(s1, t0, s1, t0);
  s2 += t0 + t1;
  // order 3 terms in plain float64
  s1 += a.x0 * b.x3 + a.x1 * b.x2 + a.x2 * b.x1 + a.x3 * b.x0 + q0 + q3 + q4 + q5;
  return renorm(p0, p1, s0, s1, s2);
}

__host__ __device__ inline qd mul_d(qd a, double b) {
  double p0, p1, p2, q0, q1, q2;
  q_two_prod(a.x0, b, p0, q0);
  q_two_prod(a.x1, b, p1, q1);
  q_two_prod(a.x2, b, p2, q2);
  const double p3 = a.x3 * b;
  double s1, s2;
  q_two_sum(q0, p1, s1, s2);        // order 1
  q_three_sum(s2, q1, p2);          // order 2
  q_three_sum2(q1, q2, p3);         // order 3
  return renorm(p0, s1, s2, q1, q2 + p2);
}

// a * 2^e, exact while no part leaves the normal range
__host__ __device__ __forceinline__ qd scale2(qd a, int e) {
  return {__builtin_ldexp(a.x0, e), __builtin_ldexp(a.x1, e), __builtin_ldexp(a.x2, e), __builtin_ldexp(a.x3, e)};
}

// a / b: five quotient digits, each the float64 quotient of the current
// remainder's leading part.
__host__ __device__ inline qd div(qd a, qd b) {
  const double q0 = a.x0 / b.x0;
  qd r = sub(a, mul_d(b, q0));
  const double q1 = r.x0 / b.x0;
  r = sub(r, mul_d(b, q1));
  const double q2 = r.x0 / b.x0;
  r = sub(r, mul_d(b, q2));
  const double q3 = r.x0 / b.x0;
  r = sub(r, mul_d(b, q3));
  const double q4 = r.x0 / b.x0;
  return renorm(q0, q1, q2, q3, q4);
}
__host__ __device__ inline qd div_d(qd a, double b) { return div(a, qd{b, 0.0, 0.0, 0.0}); }

// sqrt(a) for a >= 0: the float64 root and two Newton steps x <- (x + a / x) / 2.
__host__ __device__ inline qd sqrt(qd a) {
  if (!(a.x0 > 0.0)) return {0.0, 0.0, 0.0, 0.0};
  qd x = {__builtin_sqrt(a.x0), 0.0, 0.0, 0.0};
  for (int i = 0; i < 2; ++i) x = scale2(add(x, div(a, x)), -1);
  return x;
}

// exp(x) for x <= 0.  x = k ln 2 + r with |r| <= ln 2 / 2, r scaled by 2^-8;
// expm1 of the scaled argument by its Taylor series to the 18th power (the
// first omitted term is below 2^-220 relative), then (1 + t)^2 - 1 = 2t + t^2
// applied eight times undoes the scaling.
__host__ __device__ inline qd exp_nonpos(qd x) {
  if (x.x0 < -745.0) return {0.0, 0.0, 0.0, 0.0};
  const qd ln2 = {kLn2Hi, kLn2Lo, kLn2_2, kLn2_3};
  const double k = __builtin_rint(x.x0 / kLn2Hi);
  qd r = sub(x, mul_d(ln2, k));
  r = scale2(r, -8);
  const qd one = {1.0, 0.0, 0.0, 0.0};
  qd p = one;
  for (int n = 18; n >= 2; --n) p = add(one, div_d(mul(r, p), (double)n));
  qd t = mul(r, p);
  for (int i = 0; i < 8; ++i) t = add(scale2(t, 1), mul(t, t));
  return scale2(add(one, t), (int)k);
}

// sin and cos of |a| <= pi/4 by their Taylor series (26 terms each: the first
// omitted term is below 2^-250).
__host__ __device__ inline void sincos_reduced(qd a, qd& s, qd& c) {
  const qd a2 = mul(a, a);
  const qd one = {1.0, 0.0, 0.0, 0.0};
  qd ps = one, pc = one;
  for (int k = 26; k >= 1; --k) {
    ps = sub(one, div_d(mul(a2, ps), (double)((2 * k) * (2 * k + 1))));
    pc = sub(one, div_d(mul(a2, pc), (double)((2 * k - 1) * (2 * k))));
  }
  s = mul(a, ps);
  c = pc;
}

template <> struct xp<qd> {
  __device__ static qd zero() { return {0.0, 0.0, 0.0, 0.0}; }
  __device__ static qd from(double a) { return {a, 0.0, 0.0, 0.0}; }
  __device__ static qd prod(double a, double b) {
    double p, e;
    q_two_prod(a, b, p, e);
    return {p, e, 0.0, 0.0};
  }
  __device__ static qd two_pi() { return {kTwoPiHi, kTwoPiLo, kTwoPi2, kTwoPi3}; }
  __device__ static double lead(qd a) { return a.x0; }
  __device__ static double next(qd a) { return a.x1; }
};
using qdc = cplx<qd>;

}  // namespace ddm
}  // namespace dt
