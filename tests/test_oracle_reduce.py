"""Pins of the oracle's reductions (Tables 5 and 6) against independent references:
closed forms, Python's correctly rounded ``math.fsum``, exact rational
arithmetic (``fractions``) on tiny inputs, numpy's first-occurrence argmax /
argmin on the column-major flatten, and hand-computed golden values."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth import abs_, leaf, leaves

HERE = os.path.dirname(os.path.abspath(__file__))


def M(a, dt=None):
    a = np.asarray(a)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    dt = dt or {np.dtype(np.float32): "f32", np.dtype(np.float64): "f64"}[a.dtype]
    return synth.Mat(np.asfortranarray(a), dt)


X = [synth.Node("leaf", 0)]
XY = (leaf(0) % leaf(1)).postfix()


@pytest.fixture(scope="module")
def g():
    return np.random.default_rng(777)


@pytest.mark.parametrize("dt", ["f32", "f64", "f16", "bf16"])
def test_accu_of_ones_is_n(dt):
    n = 1 << 20
    ones = synth.store(np.ones(n), dt)
    v, _, _ = oracle.reduce("accu", X, [(ones.reshape(-1, 1), dt)])
    assert v[0] == float(n)


def test_sum_of_0_to_n_minus_1():
    n = 1 << 20
    v, _, _ = oracle.reduce("accu", X, [M(np.arange(n, dtype=np.float64))])
    assert v[0] == n * (n - 1) / 2
    v32, _, _ = oracle.reduce("accu", X, [M(np.arange(1 << 16, dtype=np.float32))])
    assert v32[0] == (1 << 16) * ((1 << 16) - 1) / 2


def test_sum_matches_fsum(g):
    for dt, scale in (("f64", 1.0), ("f32", 1.0), ("f64", 1e10)):
        x = (g.standard_normal(300_000) * scale)
        x = x.astype(np.float32) if dt == "f32" else x
        x[:10] = [1e16, -1e16, 1.0, 3e-5, -2.0, 1e15, -1e15, 0.5, 7.0, -7.0]
        x = x.astype(np.float32) if dt == "f32" else x
        v, _, asum = oracle.reduce("accu", X, [M(x)])
        exact = math.fsum(x.astype(np.float64))
        assert abs(v[0] - exact) <= 2 * np.spacing(abs(exact))
        assert abs(asum[0] - math.fsum(np.abs(x.astype(np.float64)))) <= 1e-15 * asum[0]


def test_sum_and_dot_against_exact_rationals(g):
    for trial in range(40):
        n = int(g.integers(1, 17))
        x = g.standard_normal(n) * 10.0 ** g.integers(-8, 8, n)
        y = g.standard_normal(n) * 10.0 ** g.integers(-8, 8, n)
        s_exact = sum(Fraction(v) for v in x)
        d_exact = sum(Fraction(a) * Fraction(b) for a, b in zip(x, y))
        s, _, _ = oracle.reduce("accu", X, [M(x)])
        d, _, _ = oracle.reduce("dot", XY, [M(x), M(y)])
        for got, ex in ((s[0], s_exact), (d[0], d_exact)):
            exf = float(ex)
            assert abs(Fraction(got) - ex) <= Fraction(np.spacing(abs(exf))), (trial, got, exf)


def test_dot_of_single_products_is_exact_sum(g):
    x = g.standard_normal(100_000).astype(np.float32)
    y = g.standard_normal(100_000).astype(np.float32)
    d, _, asum = oracle.reduce("dot", XY, [M(x), M(y)])
    prods = x.astype(np.float64) * y.astype(np.float64)  # exact: 24+24 bits <= 53
    exact = math.fsum(prods)
    assert abs(d[0] - exact) <= np.spacing(abs(exact))
    assert asum[0] == pytest.approx(math.fsum(np.abs(prods)), rel=1e-15)


def test_accu_of_product_equals_dot(g):
    x, y = g.standard_normal(5000), g.standard_normal(5000)
    a, _, _ = oracle.reduce("accu", XY, [M(x), M(y)])
    d, _, _ = oracle.reduce("dot", XY, [M(x), M(y)])
    assert a[0] == d[0]


def test_dot_xx_equals_norm_squared(g):
    x = g.standard_normal(200_000)
    d, _, _ = oracle.reduce("dot", (leaf(0) % leaf(0)).postfix(), [M(x)])
    n2, _, _ = oracle.reduce("norm2", X, [M(x)])
    assert n2[0] ** 2 == pytest.approx(d[0], rel=4e-16)
    assert n2[0] == pytest.approx(math.sqrt(math.fsum(x * x)), rel=2e-16)


def test_norms_against_numpy(g):
    x = g.standard_normal(10_000)
    x[17] = -9.0
    x[18] = 1e-9
    assert oracle.reduce("norm1", X, [M(x)])[0][0] == pytest.approx(math.fsum(np.abs(x)), rel=1e-16)
    assert oracle.reduce("norminf", X, [M(x)])[0][0] == 9.0
    assert oracle.reduce("normneginf", X, [M(x)])[0][0] == np.min(np.abs(x))
    A = g.standard_normal((40, 25))
    assert oracle.reduce("norm2", X, [M(A)])[0][0] == pytest.approx(np.linalg.norm(A, "fro"), rel=1e-15)


def test_index_extrema_first_occurrence(g):
    A = np.asfortranarray(g.integers(-5, 6, (31, 17)).astype(np.float32))  # many ties
    flat = A.reshape(-1, order="F")
    for op, ref in (("index_max", np.argmax), ("index_min", np.argmin)):
        _, i, _ = oracle.reduce(op, X, [M(A)])
        assert i[0] == ref(flat)
    v, i, _ = oracle.reduce("max", X, [M(A)])
    assert v[0] == flat.max()


def test_index_max_injected_ties():
    d = synth.cfg2_inputs("f32", n=1 << 16, n_ties=64)
    _, i, _ = oracle.reduce("index_max", X, [M(d["x"])])
    assert i[0] == d["ties"].min()
    _, i, _ = oracle.reduce("index_max", abs_(leaf(0)).postfix(), [M(-d["x"])])
    assert i[0] == d["ties"].min()


def test_dim_reductions_against_numpy(g):
    A = np.asfortranarray(g.standard_normal((23, 41)))
    A[3, 5] = A[7, 5] = 50.0  # tie within column 5
    s0, _, _ = oracle.reduce("sum", X, [M(A)], dim=0)
    s1, _, _ = oracle.reduce("sum", X, [M(A)], dim=1)
    assert s0.shape == (41,) and s1.shape == (23,)
    assert np.allclose(s0, [math.fsum(A[:, j]) for j in range(41)], rtol=0, atol=1e-15)
    assert np.allclose(s1, [math.fsum(A[i, :]) for i in range(23)], rtol=0, atol=1e-15)
    mx, ix, _ = oracle.reduce("max", X, [M(A)], dim=0)
    assert np.array_equal(mx, A.max(axis=0)) and np.array_equal(ix, A.argmax(axis=0))
    assert ix[5] == 3
    mn, im, _ = oracle.reduce("min", X, [M(A)], dim=1)
    assert np.array_equal(mn, A.min(axis=1)) and np.array_equal(im, A.argmin(axis=1))


def test_nan_skipped_and_all_nan():
    x = np.array([np.nan, 1.0, np.nan, 3.0, 3.0, np.nan])
    v, i, _ = oracle.reduce("index_max", X, [M(x)])
    assert v[0] == 3.0 and i[0] == 3
    v, i, _ = oracle.reduce("min", X, [M(x)])
    assert v[0] == 1.0 and i[0] == 1
    v, i, _ = oracle.reduce("max", X, [M(np.full(4, np.nan))])
    assert np.isnan(v[0]) and i[0] == 0


def test_empty_inputs():
    e = np.zeros((0, 3))
    assert oracle.reduce("accu", X, [M(e)])[0][0] == 0.0
    with pytest.raises(oracle.OracleError) as err:
        oracle.reduce("max", X, [M(e)])
    assert err.value.code == -5


def test_golden_hand_values():
    with open(os.path.join(HERE, "golden", "reductions_small.json")) as f:
        gold = json.load(f)
    A = M(np.array(gold["A"]["flat"], np.float64).reshape(gold["A"]["shape"], order="F"))
    B = M(np.array(gold["B"]["flat"], np.float64).reshape(gold["B"]["shape"], order="F"))
    e = gold["expect"]
    assert oracle.reduce("accu", X, [A])[0][0] == e["accu_A"]
    assert list(oracle.reduce("sum", X, [A], 0)[0]) == e["sum_A_dim0"]
    assert list(oracle.reduce("sum", X, [A], 1)[0]) == e["sum_A_dim1"]
    assert oracle.reduce("dot", (leaf(0) % leaf(0)).postfix(), [A])[0][0] == e["dot_A_A"]
    assert oracle.reduce("norm1", X, [A])[0][0] == e["norm1_A"]
    assert oracle.reduce("norm2", X, [A])[0][0] ** 2 == pytest.approx(e["norm2_A_squared"], rel=1e-15)
    assert oracle.reduce("norminf", X, [A])[0][0] == e["norminf_A"]
    assert oracle.reduce("max", X, [A])[0][0] == e["max_A"]
    assert oracle.reduce("index_max", X, [A])[1][0] == e["index_max_A"]
    assert oracle.reduce("index_min", X, [A])[1][0] == e["index_min_A"]
    assert list(oracle.reduce("min", X, [A], 1)[0]) == e["min_A_dim1"]
    assert oracle.reduce("index_max", X, [B])[1][0] == e["index_max_B"]
    v, i, _ = oracle.reduce("max", X, [B], 0)
    assert list(v) == e["max_B_dim0"] and list(i) == e["index_max_B_dim0"]
    assert oracle.reduce("index_min", X, [B])[1][0] == e["index_min_B"]


def test_sum2_dot2_alone(g):
    x = g.standard_normal(50_000) * 1e6
    s, a = oracle.sum2(x)
    assert abs(s - math.fsum(x)) <= np.spacing(abs(math.fsum(x)))
    y = g.standard_normal(50_000)
    d = oracle.dot2(x, y)
    exact = sum(Fraction(p) * Fraction(q) for p, q in zip(x[:2000], y[:2000]))
    assert abs(Fraction(oracle.dot2(x[:2000], y[:2000])) - exact) <= Fraction(np.spacing(abs(float(exact))))
    assert np.isfinite(d)


def test_emu_sum_is_exact_sum_of_single_precision_tree_values(g):
    a = g.uniform(-1, 1, 20_000).astype(np.float32)
    b = g.uniform(-1, 1, 20_000).astype(np.float32)
    vals = (a * a - np.float32(0.25)).astype(np.float64)   # IEEE single per node (numpy)
    s, _, asum = oracle.reduce("accu", (leaf(0) % leaf(0) - 0.25).postfix(), [M(a)], mode="emu")
    assert abs(s[0] - math.fsum(vals)) <= np.spacing(abs(math.fsum(vals)))
    # product root in EMU mode: exact sum of products of the single-precision children
    ch = (a + np.float32(1.0)).astype(np.float64) * b.astype(np.float64)
    d, _, _ = oracle.reduce("dot", ((leaf(0) + 1.0) % leaf(1)).postfix(), [M(a), M(b)], mode="emu")
    assert abs(d[0] - math.fsum(ch)) <= np.spacing(abs(math.fsum(ch)))
