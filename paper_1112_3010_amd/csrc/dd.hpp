// Double-double arithmetic for the extended-precision pipeline.
//
// A value is the unevaluated sum hi + lo of two float64 numbers with
// |lo| <= ulp(hi) / 2, which carries about 106 significand bits.  The
// error-free transformations are Knuth's TwoSum, Dekker's Fast2Sum and the
// FMA form of Dekker's product; the compound operations follow the
// "accurate" variants of Hida, Li and Bailey (2001), QD library report.
// The elementary functions (exp, sqrt, sin/cos on a reduced argument) use
// argument reduction, Taylor series evaluated by Horner's rule and one
// Newton step, all in this arithmetic.
//
// Every rounding the transformations rely on must happen as written: a file
// that includes this header is compiled with -ffp-contract=off (the pragma
// below covers the front end only; a global fast-contraction flag still lets
// the backend fuse a product into a later sum).
#pragma once
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace dt {
namespace ddm {

struct dd {
  double hi, lo;
};

// 2 pi and ln 2 to 106 bits (hi = the float64 nearest the constant, lo = the
// float64 nearest the remainder).
constexpr double kTwoPiHi = 0x1.921fb54442d18p+2, kTwoPiLo = 0x1.1a62633145c07p-52;
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1, kLn2Lo = 0x1.abc9e3b39803fp-56;

__device__ __forceinline__ dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

// requires |a| >= |b| (or a == 0)
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
  const double p = a * b;
  return {p, __builtin_fma(a, b, -p)};
}

__device__ __forceinline__ dd neg(dd a) { return {-a.hi, -a.lo}; }

__device__ __forceinline__ dd add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  const dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd sub(dd a, dd b) { return add(a, neg(b)); }

__device__ __forceinline__ dd mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ dd mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return fast_two_sum(p.hi, p.lo);
}

// a * 2^e, exact while neither part leaves the normal range
__device__ __forceinline__ dd scale2(dd a, int e) { return {__builtin_ldexp(a.hi, e), __builtin_ldexp(a.lo, e)}; }

__device__ __forceinline__ dd div_d(dd a, double b) {
  const double q1 = a.hi / b;
  const dd p = two_prod(q1, b);
  dd s = two_sum(a.hi, -p.hi);
  s.lo -= p.lo;
  s.lo += a.lo;
  const double q2 = (s.hi + s.lo) / b;
  return fast_two_sum(q1, q2);
}

// a / b: three quotient digits, each from the float64 quotient of the
// current remainder's leading part.
__device__ __forceinline__ dd div(dd a, dd b) {
  const double q1 = a.hi / b.hi;
  dd r = sub(a, mul_d(b, q1));
  const double q2 = r.hi / b.hi;
  r = sub(r, mul_d(b, q2));
  const double q3 = r.hi / b.hi;
  return add(fast_two_sum(q1, q2), {q3, 0.0});
}

// sqrt(a) for a >= 0: the float64 root refined by one Newton step whose
// residual a - x^2 is formed in double-double.
__device__ __forceinline__ dd sqrt(dd a) {
  if (!(a.hi > 0.0)) return {0.0, 0.0};
  const double x = __builtin_sqrt(a.hi);
  const dd r = sub(a, two_prod(x, x));
  return fast_two_sum(x, r.hi / (2.0 * x));
}

// exp(x) for x <= 0 (the only sign the kernels need).  x = k ln 2 + r with
// |r| <= ln 2 / 2, r scaled by 2^-10; expm1 of the scaled argument by its
// Taylor series (terms beyond the 10th are below 2^-140 relative), then
// (1 + t)^2 - 1 = 2t + t^2 applied ten times undoes the scaling.
__device__ inline dd exp_nonpos(dd x) {
  if (x.hi < -745.0) return {0.0, 0.0};
  const dd ln2 = {kLn2Hi, kLn2Lo};
  const double k = __builtin_rint(x.hi / kLn2Hi);
  dd r = sub(x, mul_d(ln2, k));
  r = scale2(r, -10);
  dd p = {1.0, 0.0};
  for (int n = 10; n >= 2; --n) p = add({1.0, 0.0}, div_d(mul(r, p), (double)n));
  dd t = mul(r, p);
  for (int i = 0; i < 10; ++i) t = add(scale2(t, 1), mul(t, t));
  const dd e = add({1.0, 0.0}, t);
  return scale2(e, (int)k);
}

// sin and cos of |a| <= pi/4 by their Taylor series (15 terms each: the
// first omitted term is below 3e-36).
__device__ inline void sincos_reduced(dd a, dd& s, dd& c) {
  const dd a2 = mul(a, a);
  dd ps = {1.0, 0.0}, pc = {1.0, 0.0};
  for (int k = 15; k >= 1; --k) {
    ps = sub({1.0, 0.0}, div_d(mul(a2, ps), (double)((2 * k) * (2 * k + 1))));
    pc = sub({1.0, 0.0}, div_d(mul(a2, pc), (double)((2 * k - 1) * (2 * k))));
  }
  s = mul(a, ps);
  c = pc;
}

// Complex values over an extended real type R (dd here, qd in qd.hpp); the
// operations resolve to R's add, sub and mul.
template <class R> struct cplx {
  R re, im;
};
using ddc = cplx<dd>;

template <class R> __device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) {
  return {add(a.re, b.re), add(a.im, b.im)};
}
template <class R> __device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) {
  return {sub(a.re, b.re), sub(a.im, b.im)};
}
template <class R> __device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {sub(mul(a.re, b.re), mul(a.im, b.im)), add(mul(a.re, b.im), mul(a.im, b.re))};
}
template <class R> __device__ __forceinline__ cplx<R> cmul_real(cplx<R> a, R b) { return {mul(a.re, b), mul(a.im, b)}; }

// What the pipeline needs of an extended real type beyond its arithmetic:
// constants, the exact product of two float64 numbers, its leading float64
// part and the part after it.
template <class R> struct xp;
template <> struct xp<dd> {
  __device__ static dd zero() { return {0.0, 0.0}; }
  __device__ static dd from(double a) { return {a, 0.0}; }
  __device__ static dd prod(double a, double b) { return two_prod(a, b); }
  __device__ static dd two_pi() { return {kTwoPiHi, kTwoPiLo}; }
  __device__ static double lead(dd a) { return a.hi; }
  __device__ static double next(dd a) { return a.lo; }
};

}  // namespace ddm
}  // namespace dt
