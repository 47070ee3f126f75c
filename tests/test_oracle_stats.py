"""Pins of the oracle's relational nodes (Table 5's all(A < x) / any(A < x),
Section 3's counting example A > 0.3) and statistics (Table 6: mean, var,
stddev) against references other than itself: numpy's comparison operators
and count_nonzero / all / any, closed forms (mean and variance of 0..n-1),
exact rational arithmetic on tiny inputs, and invariants a wrong formula
breaks (shift invariance of the variance, n - 1 normalisation)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth import eq, leaf, leaves, ne


def M(a, dt=None):
    a = np.asarray(a)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    dt = dt or {np.dtype(np.float32): "f32", np.dtype(np.float64): "f64"}[a.dtype]
    return synth.Mat(np.asfortranarray(a), dt)


X = leaf(0)


@pytest.fixture(scope="module")
def g():
    return np.random.default_rng(9090)


SPECIAL = np.array([-np.inf, -2.0, -0.0, 0.0, 0.3, 1.0, np.inf, np.nan], np.float64)


@pytest.mark.parametrize("mode", ["exact", "emu"])
def test_relational_nodes_match_numpy(mode):
    a = np.repeat(SPECIAL, SPECIAL.size)
    b = np.tile(SPECIAL, SPECIAL.size)
    A, B = M(a.reshape(8, 8)), M(b.reshape(8, 8))
    x, y = leaves(2)
    for tree, ref in ((x > y, a > b), (x < y, a < b), (x >= y, a >= b), (x <= y, a <= b), (eq(x, y), a == b),
                      (ne(x, y), a != b)):
        got = oracle.evaluate(tree.postfix(), [A, B], mode).reshape(-1, order="F")
        assert np.array_equal(got, ref.reshape(8, 8).reshape(-1, order="F").astype(np.float64))
    for tree, ref in ((x > 0.3, a > 0.3), (0.3 > x, a < 0.3), (x >= 0.0, a >= 0.0), (x <= 1.0, a <= 1.0),
                      (eq(x, 0.0), a == 0.0), (ne(x, 0.0), a != 0.0)):
        got = oracle.evaluate(tree.postfix(), [A], mode).reshape(-1, order="F")
        assert np.array_equal(got, ref.reshape(8, 8).reshape(-1, order="F").astype(np.float64))


def test_relational_scalar_rounds_to_the_compute_type():
    # 0.1 is not a float32: in an FP32 tree it compares as float32(0.1)
    v = np.array([np.float32(0.1), np.nextafter(np.float32(0.1), np.float32(1))], np.float32)
    got = oracle.evaluate((X > 0.1).postfix(), [M(v)], "emu")[:, 0]
    assert np.array_equal(got, [0.0, 1.0])
    got = oracle.evaluate(eq(X, 0.1).postfix(), [M(v)], "emu")[:, 0]
    assert np.array_equal(got, [1.0, 0.0])


def test_count_all_any_match_numpy(g):
    A = g.uniform(-1, 1, (37, 53))
    A[3, 4] = np.nan
    m = M(A)
    for dim, axis in ((-1, None), (0, 0), (1, 1)):
        for tree, pred in ((X > 0.3, A > 0.3), (X, A), (0.3 > X, A < 0.3)):
            c, ci, _ = oracle.reduce("count", tree.postfix(), [m], dim=dim)
            assert np.array_equal(c, np.atleast_1d(np.count_nonzero(pred, axis=axis)).astype(np.float64))
            assert np.array_equal(ci, np.atleast_1d(np.count_nonzero(pred, axis=axis)))
            al, _, _ = oracle.reduce("all", tree.postfix(), [m], dim=dim)
            an, _, _ = oracle.reduce("any", tree.postfix(), [m], dim=dim)
            # NaN is nonzero for numpy's all/any too
            assert np.array_equal(al, np.atleast_1d(np.all(pred, axis=axis)).astype(np.float64))
            assert np.array_equal(an, np.atleast_1d(np.any(pred, axis=axis)).astype(np.float64))


def test_count_all_any_of_empty_input():
    e = M(np.zeros((0, 3)))
    assert oracle.reduce("count", X.postfix(), [e])[0][0] == 0.0
    assert oracle.reduce("all", X.postfix(), [e])[0][0] == 1.0
    assert oracle.reduce("any", X.postfix(), [e])[0][0] == 0.0
    assert np.array_equal(oracle.reduce("all", X.postfix(), [e], dim=0)[0], [1.0, 1.0, 1.0])


@pytest.mark.parametrize("n", [1 << 10, (1 << 20) + 3])
def test_mean_and_variance_of_an_arithmetic_progression(n):
    x = np.arange(n, dtype=np.float64)
    m = M(x)
    mu, _, _ = oracle.reduce("mean", X.postfix(), [m])
    var, _, _ = oracle.reduce("var", X.postfix(), [m])
    sd, _, _ = oracle.reduce("stddev", X.postfix(), [m])
    # sum of (i - (n-1)/2)^2 over i < n is n (n^2 - 1) / 12; divided by n - 1
    assert mu[0] == (n - 1) / 2
    assert var[0] == n * (n + 1) / 12
    assert sd[0] == np.sqrt(n * (n + 1) / 12)


def test_variance_exact_on_tiny_inputs(g):
    for _ in range(20):
        k = int(g.integers(2, 9))
        x = g.uniform(-3, 3, k)
        fx = [Fraction(v) for v in x]
        mean = sum(fx) / k
        var = sum((v - mean) ** 2 for v in fx) / (k - 1)
        got, _, _ = oracle.reduce("var", X.postfix(), [M(x)])
        assert abs(Fraction(got[0]) - var) <= Fraction(1, 2 ** 50) * abs(var)
        gm, _, _ = oracle.reduce("mean", X.postfix(), [M(x)])
        assert abs(Fraction(gm[0]) - mean) <= Fraction(1, 2 ** 52) * max(abs(mean), Fraction(1, 2 ** 60))


def test_variance_is_shift_invariant_and_unbiased(g):
    x = g.standard_normal(4097)
    v0 = oracle.reduce("var", X.postfix(), [M(x)])[0][0]
    # a large offset breaks the one-pass E[x^2] - E[x]^2 formula, not two passes
    v1 = oracle.reduce("var", X.postfix(), [M(x + 1e8)])[0][0]
    assert abs(v1 - v0) <= 1e-7 * v0
    assert abs(v0 - np.var(x, ddof=1)) <= 1e-13 * v0
    assert abs(v0 - np.var(x, ddof=0)) > 1e-5 * v0      # n - 1, not n


def test_statistics_along_dims_match_numpy(g):
    A = g.uniform(-2, 2, (61, 29))
    m = M(A)
    for dim, axis in ((0, 0), (1, 1)):
        mu = oracle.reduce("mean", X.postfix(), [m], dim=dim)[0]
        var = oracle.reduce("var", X.postfix(), [m], dim=dim)[0]
        sd = oracle.reduce("stddev", X.postfix(), [m], dim=dim)[0]
        assert np.allclose(mu, A.mean(axis=axis), rtol=1e-14, atol=1e-15)
        assert np.allclose(var, A.var(axis=axis, ddof=1), rtol=1e-13)
        assert np.allclose(sd, A.std(axis=axis, ddof=1), rtol=1e-13)


def test_statistics_special_cases():
    one = M(np.array([3.5]))
    assert oracle.reduce("var", X.postfix(), [one])[0][0] == 0.0
    assert oracle.reduce("mean", X.postfix(), [one])[0][0] == 3.5
    const = M(np.full(1000, 0.1))
    assert oracle.reduce("var", X.postfix(), [const])[0][0] == 0.0
    empty = M(np.zeros((0, 1)))
    assert np.isnan(oracle.reduce("mean", X.postfix(), [empty])[0][0])
    assert np.isnan(oracle.reduce("var", X.postfix(), [empty])[0][0])
    withnan = M(np.array([1.0, np.nan, 2.0]))
    assert np.isnan(oracle.reduce("var", X.postfix(), [withnan])[0][0])
    assert np.isnan(oracle.reduce("mean", X.postfix(), [withnan])[0][0])


def test_mean_of_a_predicate_is_the_fraction_true(g):
    A = g.uniform(0, 1, 10000)
    mu = oracle.reduce("mean", (X > 0.3).postfix(), [M(A)], mode="emu")[0][0]
    assert mu == np.count_nonzero(A > 0.3) / A.size
