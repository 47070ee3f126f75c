"""Pins of the oracle's 32-bit integer element types (I32, U32; the paper's
integer matrices and their fused conversions, Section 7 conv_to, Section 2
element types) against Python's exact integers and fractions: exact widening
of the range ends, the conversion rule (fraction dropped toward zero, then
clamped to the range, NaN to 0), integer arithmetic through FP64 trees (sums,
products and truncated quotients equal exact integer results) and exact
integer sums."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth import conv, leaf, leaves

X = leaf(0)


def M(a, dt):
    a = np.asarray(a)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return synth.Mat(np.asfortranarray(a), dt)


def test_widening_is_exact_at_the_range_ends():
    v = np.array([-2 ** 31, -1, 0, 1, 2 ** 31 - 1], np.int32)
    assert list(oracle.evaluate(X.postfix(), [M(v, "i32")])[:, 0]) == [float(int(t)) for t in v]
    u = np.array([0, 1, 2 ** 31, 2 ** 32 - 1], np.uint32)
    assert list(oracle.evaluate(X.postfix(), [M(u, "u32")])[:, 0]) == [float(int(t)) for t in u]


SPECIAL = [2.5, -2.5, -0.7, 0.7, -0.0, 1e10, -1e10, 2147483647.4, 2147483647.6, -2147483648.9, 4294967295.9,
           4294967296.0, -1.5, math.inf, -math.inf, math.nan]


def expected_int(x, lo, hi):
    if math.isnan(x):
        return 0
    if math.isinf(x):
        return hi if x > 0 else lo
    t = int(Fraction(x))            # toward zero, exact
    return min(max(t, lo), hi)


@pytest.mark.parametrize("dt,lo,hi", [("i32", -2 ** 31, 2 ** 31 - 1), ("u32", 0, 2 ** 32 - 1)])
def test_conversion_rule(dt, lo, hi):
    got = oracle.round_to(dt, np.array(SPECIAL))
    assert [int(v) for v in got] == [expected_int(x, lo, hi) for x in SPECIAL]
    # the same rule as a conversion node of a tree
    v = oracle.evaluate(conv(X, dt).postfix(), [M(np.array(SPECIAL), "f64")])[:, 0]
    assert [int(t) for t in v] == [expected_int(x, lo, hi) for x in SPECIAL]


def test_integer_arithmetic_through_fp64_is_exact():
    g = np.random.default_rng(31)
    a = g.integers(-2 ** 31, 2 ** 31, 5000).astype(np.int64)
    b = g.integers(-2 ** 31, 2 ** 31, 5000).astype(np.int64)
    b[b == 0] = 7
    A, B = M(a.astype(np.int32), "i32"), M(b.astype(np.int32), "i32")
    x, y = leaves(2)
    s = oracle.evaluate((x + y).postfix(), [A, B], "emu")[:, 0]
    assert all(int(s[i]) == int(a[i]) + int(b[i]) for i in range(a.size))
    d = oracle.evaluate((x - y).postfix(), [A, B], "emu")[:, 0]
    assert all(int(d[i]) == int(a[i]) - int(b[i]) for i in range(a.size))
    # a quotient converted to I32: the integer division that truncates toward zero
    q = oracle.evaluate(conv(x / y, "i32").postfix(), [A, B], "emu")[:, 0]
    assert all(int(q[i]) == int(Fraction(int(a[i]), int(b[i]))) for i in range(a.size))
    # products of 16-bit-sized values are exact
    sa, sb = a % 40000, b % 40000
    p = oracle.evaluate((x % y).postfix(), [M(sa.astype(np.int32), "i32"), M(sb.astype(np.int32), "i32")], "emu")
    assert all(int(p[i, 0]) == int(sa[i]) * int(sb[i]) for i in range(a.size))


def test_integer_sums_and_conversion_to_float():
    g = np.random.default_rng(32)
    a = g.integers(-2 ** 31, 2 ** 31, 100000).astype(np.int32)
    s, _, _ = oracle.reduce("accu", X.postfix(), [M(a, "i32")])
    assert s[0] == float(sum(int(v) for v in a))
    # conversion of an integer to F32 rounds to nearest even
    v = np.array([2 ** 24 + 1, 2 ** 24 + 3, -(2 ** 31), 16777217], np.int32)
    got = oracle.evaluate(conv(X, "f32").postfix(), [M(v, "i32")])[:, 0]
    assert list(got) == [float(np.float32(int(t))) for t in v]
    assert got[0] == 2 ** 24 and got[1] == 2 ** 24 + 4
