"""Quad-double arithmetic of the widest extended-precision pipeline, checked
on the CPU against exact rational arithmetic.

The header's functions are host-callable; tests/host_qd/qd_driver.cpp runs
them on seeded inputs, and every result is compared with the exact value
(fractions.Fraction; exp, sin and cos from decimal arithmetic at 100
digits).  The bounds are the quad-double ones of Hida, Li and Bailey with a
few bits of slack: sums within 2^-204 of |a| + |b| (the bound the FFT's
normwise error analysis needs), products, quotients and roots within 2^-204
relative, exp within 2^-198 relative (eight squarings of the reduced
argument's expm1), sin and cos within 2^-203.  Every result must also be
non-overlapping: each part at most 2^-52 of the one before."""

import decimal
import os
import shutil
import subprocess
from fractions import Fraction as F

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1112_3010_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "host_qd", "qd_driver.cpp")

DEC = decimal.Context(prec=100)   # a local context: other modules may change the global one


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("qd") / "qd_driver")
    res = subprocess.run([hipcc, "--offload-host-only", "-O2", "-std=c++17", "-ffp-contract=off",
                          f"-I{CSRC}", DRIVER, "-o", exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    return exe


def split4(v):
    """The exact rational v as four non-overlapping float64 parts (each the
    nearest float64 to what the earlier parts leave), and their exact sum."""
    parts, r = [], F(v)
    for _ in range(4):
        d = float(r)
        parts.append(d)
        r -= F(d)
    return parts, sum(F(p) for p in parts)


def rand_qd(rng, lo=-20, hi=20, sign=True):
    m = F(int(rng.integers(1, 2**62)) * 2**180 + int(rng.integers(0, 2**62)) * 2**118
          + int(rng.integers(0, 2**62)) * 2**56 + int(rng.integers(0, 2**56)), 2**242)
    v = m * F(2) ** int(rng.integers(lo, hi))
    if sign and rng.random() < 0.5:
        v = -v
    return split4(v)


def run(exe, lines):
    inp = "\n".join(lines) + "\n"
    res = subprocess.run([exe], input=inp, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    out = []
    for ln in res.stdout.strip().splitlines():
        vals = [float.fromhex(t) for t in ln.split()]
        out.append(vals)
    assert len(out) == len(lines)
    return out


def line(op, a, b=(0.0, 0.0, 0.0, 0.0)):
    return " ".join([op] + [float(x).hex() for x in list(a) + list(b)])


def exact(parts):
    return sum(F(p) for p in parts)


def nonoverlap(parts):
    for i in range(3):
        if parts[i + 1] != 0.0 and abs(parts[i + 1]) > abs(parts[i]) * 2.0**-52:
            return False
    return True


def D(fr):
    return decimal.Decimal(fr.numerator) / decimal.Decimal(fr.denominator)


def dec_sin_cos(x):
    x = D(x)
    s, c, term = decimal.Decimal(0), decimal.Decimal(0), decimal.Decimal(1)
    for n in range(0, 120):
        if n > 0:
            term = term * x / n
        if n % 4 == 0:
            c += term
        elif n % 4 == 1:
            s += term
        elif n % 4 == 2:
            c -= term
        else:
            s -= term
    return s, c


N = 400


def test_add_sub_mul_div(driver):
    rng = np.random.default_rng(20240611)
    cases = []
    for i in range(N):
        a, A = rand_qd(rng)
        if i % 4 == 0:
            # near cancellation: b = -a plus a perturbation at a random depth
            b, B = split4(-A + A * F(2) ** -int(rng.integers(10, 200)) * F(int(rng.integers(1, 1000)), 997))
        elif i % 4 == 1:
            b, B = rand_qd(rng, -250, -150)   # far below a
        else:
            b, B = rand_qd(rng)
        cases.append((a, A, b, B))
    cases.append(([1.0, 0, 0, 0], F(1), [-1.0, 0, 0, 0], F(-1)))       # exact zero
    cases.append(([0.0, 0, 0, 0], F(0), [3.0, 0, 0, 0], F(3)))
    ops = ["add", "sub", "mul", "div"]
    lines = [line(op, a, b) for (a, A, b, B) in cases for op in ops]
    out = iter(run(driver, lines))
    worst = {op: 0.0 for op in ops}
    for (a, A, b, B) in cases:
        for op in ops:
            r = next(out)
            R = exact(r)
            assert nonoverlap(r), (op, a, b, r)
            if op in ("add", "sub"):
                want = A + B if op == "add" else A - B
                scale = abs(A) + abs(B)
            elif op == "mul":
                want, scale = A * B, abs(A * B)
            else:
                if B == 0:
                    continue
                want, scale = A / B, abs(A / B)
            err = abs(R - want)
            if scale == 0:
                assert err == 0
                continue
            rel = float(err / scale)
            worst[op] = max(worst[op], rel)
            assert rel <= 2.0**-204, (op, a, b, r, rel)
    print({k: (np.log2(v) if v > 0 else -np.inf) for k, v in worst.items()})


def test_mul_d_div_d_sqrt(driver):
    rng = np.random.default_rng(99)
    lines, ref = [], []
    for _ in range(N):
        a, A = rand_qd(rng)
        d = float(rng.uniform(-1e3, 1e3))
        lines.append(line("mul_d", a, (d, 0, 0, 0)))
        ref.append(("mul_d", A * F(d), abs(A * F(d))))
        lines.append(line("div_d", a, (d, 0, 0, 0)))
        ref.append(("div_d", A / F(d), abs(A / F(d))))
        p, P = rand_qd(rng, sign=False)
        lines.append(line("sqrt", p))
        ref.append(("sqrt", P, None))
    for (op, want, scale), r in zip(ref, run(driver, lines)):
        R = exact(r)
        assert nonoverlap(r), (op, r)
        if op == "sqrt":
            # |r^2 - p| <= 2^-203 p  <=>  relative error of the root about 2^-204
            assert abs(R * R - want) <= want * F(2) ** -203, (r, float(want))
        else:
            assert abs(R - want) <= scale * F(2) ** -204, (op, r, float(want))


def test_exp(driver):
    with decimal.localcontext(DEC):
        _check_exp(driver)


def _check_exp(driver):
    rng = np.random.default_rng(7)
    xs = [split4(-F(int(rng.integers(0, 2**60)), 2**60) * F(int(rng.integers(1, 300)))) for _ in range(150)]
    xs += [split4(F(0)), split4(-F(1, 2**40)), split4(-F(700))]
    lines = [line("exp", x) for x, _ in xs]
    worst = 0.0
    for (x, X), r in zip(xs, run(driver, lines)):
        assert nonoverlap(r)
        want = D(X).exp()
        got = sum(decimal.Decimal(p) for p in r)
        if X < -600:
            # the lower parts of e^-700 (about 1e-304) are subnormal: only
            # the absolute error is bounded, by the subnormal spacing
            assert abs(got - want) <= decimal.Decimal(2) ** -1070
            continue
        rel = abs(got - want) / want
        worst = max(worst, float(rel))
        assert rel <= decimal.Decimal(2) ** -198, (x, float(rel))
    print("exp worst log2 rel", np.log2(worst) if worst > 0 else "-inf")


def test_sin_cos(driver):
    with decimal.localcontext(DEC):
        _check_sin_cos(driver)


def _check_sin_cos(driver):
    rng = np.random.default_rng(11)
    quarter = F(7853981633974483096156608458198757, 10**34)   # below pi/4
    args = [split4(quarter * F(int(rng.integers(-2**50, 2**50)), 2**50)) for _ in range(150)]
    args += [split4(F(0)), split4(quarter)]
    lines = [line("sincos", a) for a, _ in args]
    for (a, A), r in zip(args, run(driver, lines)):
        s_ref, c_ref = dec_sin_cos(A)
        s = sum(decimal.Decimal(p) for p in r[:4])
        c = sum(decimal.Decimal(p) for p in r[4:])
        assert nonoverlap(r[:4]) and nonoverlap(r[4:])
        tol = decimal.Decimal(2) ** -203
        assert abs(s - s_ref) <= tol and abs(c - c_ref) <= tol, (a, float(s - s_ref), float(c - c_ref))


def test_constants():
    """The four-part 2 pi and ln 2 of the header against exact series."""
    import re
    src = open(os.path.join(CSRC, "qd.hpp")).read() + open(os.path.join(CSRC, "dd.hpp")).read()

    def const(name):
        return float.fromhex(re.search(name + r"\s*=\s*(-?0x[0-9a-fp.+-]+)", src).group(1))

    def atan_inv(n, terms):
        s, x = F(0), F(1, n)
        p = x
        for k in range(terms):
            s += p / (2 * k + 1) * (1 if k % 2 == 0 else -1)
            p *= x * x
        return s

    two_pi = 8 * (4 * atan_inv(5, 200) - atan_inv(239, 80))
    ln2 = sum(F(1, k * 2**k) for k in range(1, 800))
    tp = exact([const("kTwoPiHi"), const("kTwoPiLo"), const("kTwoPi2"), const("kTwoPi3")])
    l2 = exact([const("kLn2Hi"), const("kLn2Lo"), const("kLn2_2"), const("kLn2_3")])
    assert abs(tp - two_pi) <= two_pi * F(2) ** -212
    assert abs(l2 - ln2) <= ln2 * F(2) ** -212
