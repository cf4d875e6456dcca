"""The table behind the bounds kernels' exp (paper_2407_20966_amd/csrc/
exp2_table.h): the committed header is what its generator writes, and its
values are 2^(j/256), 2^(j/256)/24 and a two-part ln(2)/256, checked against
the host libm.  The kernels' exp itself is covered by the GPU parity tests
(bounds within 1e-12 of the oracle's numpy exp)."""

import math
import os
from fractions import Fraction
import re
import subprocess
import sys

import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2407_20966_amd", "csrc")
HEADER = os.path.join(CSRC, "exp2_table.h")


def ulp(x: float) -> float:
    return math.nextafter(abs(x), math.inf) - abs(x)


def parse(text):
    hexf = r"(-?0x[0-9a-fA-F.]+p[-+]?\d+)"
    hi = float.fromhex(re.search(r"kLn2By256Hi = " + hexf, text).group(1))
    lo = float.fromhex(re.search(r"kLn2By256Lo = " + hexf, text).group(1))
    pairs = [(float.fromhex(a), float.fromhex(b))
             for a, b in re.findall(r"\{" + hexf + r", " + hexf + r"\}", text)]
    return hi, lo, pairs


def test_header_is_what_the_generator_writes(tmp_path):
    out = tmp_path / "t.h"
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_exp2_table.py"), str(out)], check=True)
    assert out.read_text() == open(HEADER).read()


def test_table_values():
    hi, lo, pairs = parse(open(HEADER).read())
    assert len(pairs) == 256
    for j, (t, t24) in enumerate(pairs):
        ref = math.pow(2.0, j / 256.0)          # j/256 is exact in binary
        assert abs(t - ref) <= ulp(ref), j
        assert 1.0 <= t < 2.0
        assert abs(t24 * 24.0 - t) <= 2 * ulp(t), j
    assert pairs[0] == (1.0, float.fromhex("0x1.5555555555555p-5"))


def test_ln2_split():
    hi, lo, _ = parse(open(HEADER).read())
    assert hi == pytest.approx(math.log(2.0) / 256, rel=2.3e-16)
    # the tail is below half an ulp of the head and carries ln 2 to ~1e-32
    assert 0 < abs(lo) <= ulp(hi) / 2
    assert abs((hi + lo) - math.log(2.0) / 256) <= ulp(hi)


def fma(a: float, b: float, c: float) -> float:
    """a * b + c rounded once, as the GPU's fused multiply-add."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_reduction_reproduces_exp_on_the_host():
    """The kernels' steps (n = round(x 256/ln2) by the 1.5 2^52 shift, r = x -
    n ln2/256 in two fused parts, r (24 + r (12 + r (4 + r))) / 24 with the
    1/24 from the table, 2^m) evaluated with exactly rounded fused
    multiply-adds stay within 2 ulp of the host exp over the range the bounds
    use, and -inf or very negative arguments give 0."""
    hi, lo, pairs = parse(open(HEADER).read())
    inv = float.fromhex("0x1.71547652b82fep+8")
    shift = float.fromhex("0x1.8p52")

    def exp_tab(x):
        x = max(x, -1100.0)
        t = fma(x, inv, shift)
        n = t - shift
        ni = int(n)
        r = fma(-n, hi, x)
        r = fma(-n, lo, r)
        q = r + 4.0
        q = fma(r, q, 12.0)
        q = fma(r, q, 24.0)
        q = r * q
        tt, t24 = pairs[ni & 255]
        return math.ldexp(fma(t24, q, tt), ni >> 8)

    worst = 0.0
    for i in range(3001):
        x = -700.0 + i * 0.2369
        y, ref = exp_tab(x), math.exp(x)
        worst = max(worst, abs(y - ref) / ulp(ref))
    assert worst <= 2.0, worst
    assert exp_tab(-math.inf) == 0.0
    assert exp_tab(-1.0e6) == 0.0
    assert exp_tab(0.0) == 1.0
