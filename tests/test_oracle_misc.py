"""Pins of the oracle's misc and trig element-wise functions (Table 7: pow,
log10, square, cos, sin, tan, acos, asin, atan, ...): closed forms, exact
results of the rounding functions checked with exact rationals, identities
between different functions (a swapped or mistyped function breaks one), and
the rounding of the scalar exponent to the compute type."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth import (acos, asin, atan, ceil, cos, cosh, exp2, floor, leaf, log2, log10, pow_, round_, sign, sin,
                   sinh, square, tan, tanh, trunc)

X = leaf(0)


def M(a, dt="f64"):
    a = np.asarray(a, np.float64 if dt == "f64" else np.float32).reshape(-1, 1)
    return synth.Mat(np.asfortranarray(a), dt)


def ev(tree, a, mode="exact", dt="f64"):
    return oracle.evaluate(tree.postfix(), [M(a, dt)], mode)[:, 0]


def test_closed_forms():
    assert np.array_equal(ev(log10(X), [1.0, 10.0, 1000.0, 1e-3]), [0.0, 1.0, 3.0, -3.0])
    assert np.array_equal(ev(log2(X), [1.0, 8.0, 0.5, 2.0 ** 40]), [0.0, 3.0, -1.0, 40.0])
    assert np.array_equal(ev(exp2(X), [0.0, 10.0, -2.0]), [1.0, 1024.0, 0.25])
    assert np.array_equal(ev(pow_(X, 10.0), [2.0, 1.0, 0.5]), [1024.0, 1.0, 2.0 ** -10])
    assert np.array_equal(ev(pow_(X, 0.5), [9.0, 16.0, 0.25]), [3.0, 4.0, 0.5])
    assert np.array_equal(ev(square(X), [3.0, -1.5, 0.0]), [9.0, 2.25, 0.0])
    assert np.array_equal(ev(cos(X), [0.0]), [1.0])
    assert np.array_equal(ev(sin(X), [0.0, -0.0]), [0.0, -0.0])
    assert np.array_equal(ev(tanh(X), [0.0, np.inf, -np.inf]), [0.0, 1.0, -1.0])
    assert np.array_equal(ev(atan(X), [0.0, np.inf]), [0.0, math.pi / 2])
    assert np.array_equal(ev(acos(X), [1.0]), [0.0])
    assert np.array_equal(ev(cosh(X), [0.0]), [1.0])


def test_rounding_functions_exact():
    vals = [-2.5, -1.5, -0.5, -0.49999999999999994, 0.5, 1.5, 2.5, -2.7, 2.7, 1e15 + 0.5, -0.0, 3.0]
    fr = [Fraction(v) for v in vals]
    fl = [math.floor(v) for v in fr]                      # exact on rationals
    ce = [math.ceil(v) for v in fr]
    tr = [int(v) for v in fr]                             # toward zero
    ro = [int(v + Fraction(1, 2)) if v >= 0 else -int(-v + Fraction(1, 2)) for v in fr]  # half away from zero
    assert np.array_equal(ev(floor(X), vals), np.array(fl, np.float64))
    assert np.array_equal(ev(ceil(X), vals), np.array(ce, np.float64))
    assert np.array_equal(ev(trunc(X), vals), np.array(tr, np.float64))
    assert np.array_equal(ev(round_(X), vals), np.array(ro, np.float64))


def test_sign():
    got = ev(sign(X), [-3.0, -0.0, 0.0, 2.0, np.inf, -np.inf, np.nan])
    assert np.array_equal(got[:6], [-1.0, -0.0, 0.0, 1.0, 1.0, -1.0])
    assert np.signbit(got[1]) and not np.signbit(got[2])
    assert np.isnan(got[6])


def test_trig_and_hyperbolic_identities():
    g = np.random.default_rng(3131)
    x = g.uniform(-3, 3, 5000)
    s, c, t = ev(sin(X), x), ev(cos(X), x), ev(tan(X), x)
    assert np.max(np.abs(s * s + c * c - 1.0)) <= 4e-16
    ok = np.abs(c) > 1e-3
    assert np.max(np.abs(t[ok] - s[ok] / c[ok]) / np.abs(t[ok])) <= 1e-14
    h = g.uniform(-1.5, 1.5, 5000)                      # inside (-pi/2, pi/2)
    assert np.max(np.abs(ev(asin(sin(X)), h) - h)) <= 4e-15
    assert np.max(np.abs(ev(atan(tan(X)), h) - h)) <= 4e-15
    p = g.uniform(0.3, 2.8, 5000)                       # inside [0, pi], away from acos's infinite slope
    assert np.max(np.abs(ev(acos(cos(X)), p) - p)) <= 4e-15
    y = g.uniform(-5, 5, 5000)
    ch, sh, th = ev(cosh(X), y), ev(sinh(X), y), ev(tanh(X), y)
    assert np.max(np.abs(ch * ch - sh * sh - 1.0) / (ch * ch)) <= 1e-15
    assert np.max(np.abs(th - sh / ch)) <= 1e-15
    assert np.max(np.abs(ev(log2(exp2(X)), y) - y)) <= 1e-14
    z = g.uniform(0.1, 100, 5000)
    assert np.max(np.abs(ev(log10(X), z) - ev(log2(X), z) * math.log10(2.0))) <= 1e-14


def test_emu_rounds_to_float32_and_scalar_exponent_is_float32():
    x = np.array([0.7, 1.3, 2.9], np.float32)
    em = ev(sin(X), x, "emu", "f32")
    assert np.array_equal(em, np.array([np.float32(math.sin(float(v))) for v in x], np.float64))
    # an FP32 tree uses float32(0.1) as the exponent
    em = ev(pow_(X, 0.1), x, "emu", "f32")
    k = float(np.float32(0.1))
    assert np.array_equal(em, np.array([np.float32(float(v) ** k) for v in x], np.float64))
    assert not np.array_equal(em, np.array([np.float32(float(v) ** 0.1) for v in x], np.float64))


def test_error_scale_of_functions_is_finite_on_their_domains():
    g = np.random.default_rng(77)
    x = g.uniform(0.1, 0.9, 100)
    for f in (acos, asin, atan, cos, sin, tan, cosh, sinh, tanh, log10, log2, exp2, square, floor, sign):
        _, S = oracle.evaluate(f(X).postfix(), [M(x)], "exact", scale=True)
        assert np.all(np.isfinite(S)) and np.all(S > 0), f.__name__
