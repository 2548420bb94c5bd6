"""Host: the multi-component scalar arithmetic of csrc/mc.h and csrc/dd.h (the
TD and DD LU, the simple in-format products of TD, QD and TS), compiled with
the host compiler from the same headers (a stub stands in for the HIP runtime
header), checked against exact rational arithmetic:

* TD division: relative error below 2^-155 (three quotient digits leave a
  remainder near 2^-156 |a|; TD's own rounding is near 2^-159), and clearly
  worse with two digits, so the third digit is needed;
* TD addition, multiplication and fused multiply-add: below 2^-155;
* DD division below 2^-102, DD multiply and add below 2^-103;
* TS (three binary32 components) fused multiply-add below 2^-68.
"""
import math
import pathlib
import random
import shutil
import subprocess
from fractions import Fraction

import pytest

CSRC = pathlib.Path(__file__).resolve().parents[1] / "paper_2301_09960_amd" / "csrc"

STUB = r'''
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#define __device__
#define __host__
#define __forceinline__ inline
using std::fma; using std::fabs; using std::ldexp; using std::frexp;
inline long long __double_as_longlong(double x) { long long b; std::memcpy(&b, &x, 8); return b; }
inline double __longlong_as_double(long long b) { double x; std::memcpy(&x, &b, 8); return x; }
inline unsigned int __float_as_uint(float x) { unsigned int b; std::memcpy(&b, &x, 4); return b; }
inline float __uint_as_float(unsigned int b) { float x; std::memcpy(&x, &b, 4); return x; }
'''

PROG = r'''
#include <cstdio>
#include <cstdlib>
#include "mc.h"
#include "dd.h"
using namespace mp;
int main() {
  char op[16];
  while (std::scanf("%15s", op) == 1) {
    if (op[0] == 'T') {  // TD: op a0 a1 a2 b0 b1 b2 c0 c1 c2
      mc<3> a, b, c, r;
      for (int i = 0; i < 3; ++i) std::scanf("%la", &a.x[i]);
      for (int i = 0; i < 3; ++i) std::scanf("%la", &b.x[i]);
      for (int i = 0; i < 3; ++i) std::scanf("%la", &c.x[i]);
      switch (op[1]) {
        case 'a': r = mc_add<3>(a, b); break;
        case 'm': r = mc_mul<3>(a, b); break;
        case 'd': r = mc_div<3>(a, b); break;
        default: r = mc_fma<3>(c, a, b); break;
      }
      std::printf("%a %a %a\n", r.x[0], r.x[1], r.x[2]);
    } else if (op[0] == 'Q') {  // TD division with two digits only: q1, q2 and the rest dropped
      mc<3> a, b;
      for (int i = 0; i < 3; ++i) std::scanf("%la", &a.x[i]);
      for (int i = 0; i < 3; ++i) std::scanf("%la", &b.x[i]);
      double q[2];
      mc<3> r = a;
      q[0] = r.x[0] / b.x[0];
      r = mc_sub_scaled<3>(r, q[0], b);
      q[1] = r.x[0] / b.x[0];
      std::printf("%a %a\n", q[0], q[1]);
    } else if (op[0] == 'D') {  // DD: op a0 a1 b0 b1
      dd a, b, r;
      std::scanf("%la %la %la %la", &a.hi, &a.lo, &b.hi, &b.lo);
      r = op[1] == 'a' ? dd_add(a, b) : op[1] == 'm' ? dd_mul(a, b) : dd_div(a, b);
      std::printf("%a %a\n", r.hi, r.lo);
    } else {  // S: TS fused multiply-add c + a b, 9 floats
      float x[9];
      for (int i = 0; i < 9; ++i) { double v; std::scanf("%la", &v); x[i] = (float)v; }
      mc<3, float> a{{x[0], x[1], x[2]}}, b{{x[3], x[4], x[5]}}, c{{x[6], x[7], x[8]}};
      mc<3, float> r = mc_fma<3>(c, a, b);
      std::printf("%a %a %a\n", (double)r.x[0], (double)r.x[1], (double)r.x[2]);
    }
  }
  return 0;
}
'''


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("mc")
    (d / "hip").mkdir()
    (d / "hip" / "hip_runtime.h").write_text(STUB)
    (d / "prog.cpp").write_text(PROG)
    exe = d / "prog"
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wno-unused-result", f"-I{d}", f"-I{CSRC}", "-o",
                    str(exe), str(d / "prog.cpp")], check=True)

    def run(lines):
        out = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
        return [[float.fromhex(v) for v in line.split()] for line in out.stdout.strip().split("\n")]
    return run


def expansion(rng, c, scale, bits=53):
    """A normalized c-term expansion: each term below half an ulp of the one above."""
    x0 = rng.uniform(1.0, 2.0) * 2.0 ** scale * rng.choice((-1, 1))
    out = [x0]
    for _ in range(c - 1):
        prev = out[-1]
        out.append(prev * 2.0 ** -(bits + 1) * rng.uniform(-1, 1))
    if bits == 24:
        import numpy as np
        out = [float(np.float32(v)) for v in out]
        # re-normalize after rounding to binary32
        for i in range(1, c):
            if abs(out[i]) > abs(out[i - 1]) * 2.0 ** -24:
                out[i] = float(np.float32(out[i - 1] * 2.0 ** -25))
    return out


def val(terms):
    return sum(Fraction(t) for t in terms)


def rel(got, want):
    return abs(val(got) - want) / abs(want)


def hexs(v):
    return " ".join(float(x).hex() for x in v)


def test_td_division_needs_three_digits(prog):
    rng = random.Random(1)
    cases = [(expansion(rng, 3, rng.randint(-30, 30)), expansion(rng, 3, rng.randint(-30, 30))) for _ in range(400)]
    cases += [([1.0, 0.0, 0.0], [3.0, 0.0, 0.0]), ([1.0, 2.0 ** -60, 0.0], [7.0, -2.0 ** -55, 2.0 ** -110])]
    three = prog([f"Td {hexs(a)} {hexs(b)} 0x0p+0 0x0p+0 0x0p+0" for a, b in cases])
    two = prog([f"Q {hexs(a)} {hexs(b)}" for a, b in cases])
    worst3 = max(rel(q, val(a) / val(b)) for q, (a, b) in zip(three, cases))
    worst2 = max(rel(q, val(a) / val(b)) for q, (a, b) in zip(two, cases))
    print(f"TD division: log2 of the worst relative error {math.log2(worst3):.1f} with three digits, "
          f"{math.log2(worst2):.1f} with two")
    assert worst3 < Fraction(2) ** -155
    assert worst2 > Fraction(2) ** -110  # the third digit is what brings it to TD precision


@pytest.mark.parametrize("op", ["Ta", "Tm", "Tf"])
def test_td_add_mul_fma(prog, op):
    rng = random.Random(2)
    cases = [[expansion(rng, 3, rng.randint(-20, 20)) for _ in range(3)] for _ in range(300)]
    out = prog([f"{op} {hexs(a)} {hexs(b)} {hexs(c)}" for a, b, c in cases])
    worst = 0
    for r, (a, b, c) in zip(out, cases):
        want = {"Ta": val(a) + val(b), "Tm": val(a) * val(b), "Tf": val(c) + val(a) * val(b)}[op]
        scale = {"Ta": abs(val(a)) + abs(val(b)), "Tm": abs(want),
                 "Tf": abs(val(c)) + abs(val(a) * val(b))}[op]
        worst = max(worst, abs(val(r) - want) / scale)
        assert abs(r[1]) <= abs(r[0]) * 2.0 ** -52 and abs(r[2]) <= abs(r[1]) * 2.0 ** -52
    assert worst < Fraction(2) ** -155, float(worst)


@pytest.mark.parametrize("op,bound", [("Da", 103), ("Dm", 103), ("Dd", 102)])
def test_dd_operations(prog, op, bound):
    rng = random.Random(3)
    cases = [(expansion(rng, 2, rng.randint(-20, 20)), expansion(rng, 2, rng.randint(-20, 20))) for _ in range(300)]
    out = prog([f"{op} {hexs(a)} {hexs(b)}" for a, b in cases])
    for r, (a, b) in zip(out, cases):
        want = {"Da": val(a) + val(b), "Dm": val(a) * val(b), "Dd": val(a) / val(b)}[op]
        scale = abs(val(a)) + abs(val(b)) if op == "Da" else abs(want)
        assert abs(val(r) - want) <= Fraction(2) ** -bound * scale, (op, a, b)


def test_ts_fused_multiply_add(prog):
    rng = random.Random(4)
    cases = [[expansion(rng, 3, rng.randint(-10, 10), bits=24) for _ in range(3)] for _ in range(300)]
    out = prog([f"S {hexs(a)} {hexs(b)} {hexs(c)}" for a, b, c in cases])
    for r, (a, b, c) in zip(out, cases):
        want = val(c) + val(a) * val(b)
        scale = abs(val(c)) + abs(val(a) * val(b))
        assert abs(val(r) - want) <= Fraction(2) ** -68 * scale, (a, b, c)
