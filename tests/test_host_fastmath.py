"""The FP64 e^x and sin / cos of the kernel evaluations (csrc/fastmath_dev.h): Cody-Waite
reduction plus Taylor polynomials.

Pins: every constant of the header equals the nearest double to its exact value, recomputed
here in 80-digit decimal arithmetic (pi by Machin's formula, ln 2 by the decimal module,
1/k! as exact fractions); the functions, compiled for the host, agree with the C library's
exp, sin and cos within 1 unit in the last place over 2e6 seeded arguments (e^x on
[-745, 709], sin and cos on |x| in [1e-3, 1e6], both signs), and the special cases
(e^x = 0 below -745.2, +inf above 709.8, sin/cos beyond 2^20 and NaN through the library)."""
import math
import os
import re
import subprocess
import tempfile
from decimal import Decimal, getcontext
from fractions import Fraction

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2312_11219_amd", "csrc")
HEADER = os.path.join(CSRC, "fastmath_dev.h")


def _exact():
    getcontext().prec = 80

    def atan_inv(x):
        x = Decimal(x)
        s, t, k, x2 = Decimal(0), 1 / x, 0, x * x
        while True:
            term = t / (2 * k + 1)
            if term < Decimal(10) ** -78:
                return s
            s += term if k % 2 == 0 else -term
            t /= x2
            k += 1

    pi = 16 * atan_inv(5) - 4 * atan_inv(239)
    ln2 = Decimal(2).ln()
    hp = pi / 2
    a = float(hp)
    b = float(hp - Decimal(a))
    c = float(hp - Decimal(a) - Decimal(b))
    hi = float(ln2)
    lo = float(ln2 - Decimal(hi))
    return {"kLog2e": float(1 / ln2), "kLn2Hi": hi, "kLn2Lo": lo, "kTwoOverPi": float(2 / pi),
            "kPio2A": a, "kPio2B": b, "kPio2C": c}


def _header_constants():
    src = open(HEADER).read()
    out = {}
    for name, val in re.findall(r"constexpr double (k\w+) = (-?0x[0-9a-fp.+-]+);", src):
        out[name] = float.fromhex(val)
    table = re.search(r"kInvFact\[18\] = \{(.*?)\};", src, re.S).group(1)
    out["kInvFact"] = [float.fromhex(v) for v in re.findall(r"0x[0-9a-fp.+-]+", table)]
    return out


def test_constants_are_nearest_doubles():
    h = _header_constants()
    for name, v in _exact().items():
        assert h[name] == v, name
    assert h["kInvFact"] == [float(Fraction(1, math.factorial(k))) for k in range(18)]
    # the pi / 2 split really sums to pi / 2 beyond double precision
    getcontext().prec = 80
    assert abs(Decimal(h["kPio2A"]) + Decimal(h["kPio2B"]) + Decimal(h["kPio2C"])
               - Decimal("1.5707963267948966192313216916397514420985846996875529104874722961")) \
        < Decimal(10) ** -48


HARNESS = r"""
#include "fastmath_dev.h"
#include <cmath>
#include <cstdio>
#include <random>
static double ulp(double v) { return std::nextafter(std::fabs(v), INFINITY) - std::fabs(v); }
int main() {
    std::mt19937_64 g(1);
    std::uniform_real_distribution<double> U(0, 1);
    double we = 0, ws = 0, wc = 0;
    for (int i = 0; i < 2000000; ++i) {
        double x = (i % 3 == 0) ? -200.0 * U(g) : -745.0 + 1454.0 * U(g);
        double r = std::exp(x), a = gaca::fm::exp(x);
        if (r > 1e-300 && std::isfinite(r)) we = std::fmax(we, std::fabs(a - r) / ulp(r));
        double t = std::pow(10.0, -3 + 9 * U(g)) * (U(g) < 0.5 ? -1 : 1);
        double s, c;
        gaca::fm::sincos(t, &s, &c);
        double rs = std::sin(t), rc = std::cos(t);
        if (std::fabs(rs) > 1e-3) ws = std::fmax(ws, std::fabs(s - rs) / ulp(rs));
        if (std::fabs(rc) > 1e-3) wc = std::fmax(wc, std::fabs(c - rc) / ulp(rc));
        if (std::fabs(s - rs) > 2.3e-16 || std::fabs(c - rc) > 2.3e-16) { printf("abs %g\n", t); return 1; }
    }
    double s, c;
    gaca::fm::sincos(3.0e7, &s, &c);
    int special = gaca::fm::exp(-746.0) == 0.0 && std::isinf(gaca::fm::exp(710.0)) &&
                  gaca::fm::exp(0.0) == 1.0 && s == std::sin(3.0e7) && c == std::cos(3.0e7) &&
                  std::isnan(gaca::fm::exp(NAN));
    gaca::fm::sincos(NAN, &s, &c);
    special = special && std::isnan(s) && std::isnan(c);
    printf("%.3f %.3f %.3f %d\n", we, ws, wc, special);
    return 0;
}
"""


def test_functions_within_one_ulp():
    if not shutil_which("g++"):
        pytest.skip("g++ not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        exe = os.path.join(d, "t")
        with open(src, "w") as fh:
            fh.write(HARNESS)
        subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC, "-o", exe, src],
                       check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    we, ws, wc, special = float(out[0]), float(out[1]), float(out[2]), int(out[3])
    assert we <= 1.0 and ws <= 1.0 and wc <= 1.0, (we, ws, wc)
    assert special == 1


def shutil_which(name):
    import shutil
    return shutil.which(name)
