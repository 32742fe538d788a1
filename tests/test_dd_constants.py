"""The double-double constants of the extended-precision kernels (2 pi and
ln 2 as hi + lo pairs) against 50-digit decimal arithmetic: pi from Machin's
formula, ln 2 from the decimal module's correctly rounded logarithm."""

import os
import re
from decimal import Decimal, getcontext

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1112_3010_amd", "csrc", "dd.hpp")


def _consts():
    text = open(HEADER).read()
    found = dict(re.findall(r"(k\w+(?:Hi|Lo)) = (0x[0-9a-fp.+-]+)", text))
    return {k: float.fromhex(v) for k, v in found.items()}


def _arctan_inv(x):
    x = Decimal(x)
    t = 1 / x
    total, n, sign, x2 = t, 1, -1, x * x
    while True:
        t /= x2
        n += 2
        term = t / n
        if term < Decimal(10) ** -58:
            return total
        total += sign * term
        sign = -sign


def test_two_pi_and_ln2_pairs():
    getcontext().prec = 60
    c = _consts()
    pi = 16 * _arctan_inv(5) - 4 * _arctan_inv(239)
    for name, exact in (("kTwoPi", 2 * pi), ("kLn2", Decimal(2).ln())):
        hi, lo = c[name + "Hi"], c[name + "Lo"]
        assert hi == float(exact)                       # hi is the nearest float64
        assert abs(lo) <= abs(hi) * 2.0 ** -53           # normalised pair
        rel = abs((exact - Decimal(hi) - Decimal(lo)) / exact)
        assert rel < Decimal(2) ** -105, (name, rel)
