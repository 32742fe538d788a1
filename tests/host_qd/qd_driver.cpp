// Runs quad-double operations of the extended-precision pipeline on the host
// for the arithmetic checks in tests/test_qd_arith.py.
//
// stdin: one operation per line, "<op> a0 a1 a2 a3 b0 b1 b2 b3" with the
// parts as C99 hexadecimal floats (b is ignored by the unary operations;
// mul_d and div_d use b0 only).  stdout: the result parts, four per line
// (eight for sincos: sin, then cos).
#include <cstdio>
#include <cstring>

#include "qd.hpp"

using dt::ddm::qd;

static void put(const qd& r) { std::printf("%a %a %a %a", r.x0, r.x1, r.x2, r.x3); }

int main() {
  char op[32];
  qd a, b;
  while (std::scanf("%31s %la %la %la %la %la %la %la %la", op, &a.x0, &a.x1, &a.x2, &a.x3, &b.x0, &b.x1, &b.x2,
                    &b.x3) == 9) {
    if (!std::strcmp(op, "add")) put(dt::ddm::add(a, b));
    else if (!std::strcmp(op, "sub")) put(dt::ddm::sub(a, b));
    else if (!std::strcmp(op, "mul")) put(dt::ddm::mul(a, b));
    else if (!std::strcmp(op, "mul_d")) put(dt::ddm::mul_d(a, b.x0));
    else if (!std::strcmp(op, "div")) put(dt::ddm::div(a, b));
    else if (!std::strcmp(op, "div_d")) put(dt::ddm::div_d(a, b.x0));
    else if (!std::strcmp(op, "sqrt")) put(dt::ddm::sqrt(a));
    else if (!std::strcmp(op, "exp")) put(dt::ddm::exp_nonpos(a));
    else if (!std::strcmp(op, "sincos")) {
      qd s, c;
      dt::ddm::sincos_reduced(a, s, c);
      put(s);
      std::printf(" ");
      put(c);
    } else {
      std::fprintf(stderr, "unknown op %s\n", op);
      return 2;
    }
    std::printf("\n");
  }
  return 0;
}
