"""Pins of the oracle's generator operands (Table 1 fill / ones / zeros / eye,
Table 4 eye / ones / zeros / linspace) and of the view definitions the GPU
tests use (Table 1 submatrix views; Table 5 trace; Table 6 diagvec), against
references other than the oracle: numpy's eye / full / diagonal / trace,
textbook 16-bit encodings of 0.1 and 1, exact rational arithmetic for
linspace, and the end-point and spacing properties the definition fixes."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth import leaf, trans

X = leaf(0)


def values(op):
    data, dt = op
    if dt in ("f16", "bf16"):
        return oracle.widen16(dt, data)
    return np.asarray(data, np.float64)


@pytest.mark.parametrize("dt", ["f32", "f64", "f16", "bf16"])
@pytest.mark.parametrize("shape", [(5, 5), (3, 7), (7, 3), (1, 4), (0, 3)])
def test_eye_matches_numpy(dt, shape):
    r, c = shape
    assert np.array_equal(values(oracle.eye(r, c, dt)), np.eye(r, c))


def test_fill_ones_zeros_and_16_bit_encodings():
    for dt in ("f32", "f64", "f16", "bf16"):
        assert np.array_equal(values(oracle.fill(4, 3, 1.0, dt)), np.ones((4, 3)))
        assert np.array_equal(values(oracle.fill(4, 3, 0.0, dt)), np.zeros((4, 3)))
        assert np.array_equal(values(oracle.fill(2, 2, -2.5, dt)), np.full((2, 2), -2.5))
    # 0.1 stored in each type: the nearest value of that type
    assert values(oracle.fill(1, 1, 0.1, "f64"))[0, 0] == 0.1
    assert values(oracle.fill(1, 1, 0.1, "f32"))[0, 0] == float(np.float32(0.1))
    assert oracle.fill(1, 1, 0.1, "f16")[0][0, 0] == 0x2E66     # 0.0999755859375
    assert oracle.fill(1, 1, 0.1, "bf16")[0][0, 0] == 0x3DCD    # 0.10009765625
    assert oracle.fill(1, 1, 1.0, "bf16")[0][0, 0] == 0x3F80
    assert oracle.fill(1, 1, 1.0, "f16")[0][0, 0] == 0x3C00


def test_linspace_exact_cases():
    assert np.array_equal(oracle.linspace_values(0.0, 1.0, 5), [0.0, 0.25, 0.5, 0.75, 1.0])
    assert np.array_equal(oracle.linspace_values(-1.0, 1.0, 3), [-1.0, 0.0, 1.0])
    assert np.array_equal(oracle.linspace_values(10.0, 0.0, 11), np.arange(10.0, -1.0, -1.0))
    assert np.array_equal(oracle.linspace_values(2.0, 3.0, 2), [2.0, 3.0])
    assert np.array_equal(oracle.linspace_values(2.0, 3.0, 1), [3.0])       # one element: the end
    assert oracle.linspace_values(2.0, 3.0, 0).size == 0


def test_linspace_against_exact_rationals():
    g = np.random.default_rng(4242)
    for _ in range(50):
        a, b = g.uniform(-100, 100, 2)
        n = int(g.integers(2, 300))
        x = oracle.linspace_values(a, b, n)
        assert x[0] == a and x[-1] == b
        fa, fb = Fraction(a), Fraction(b)
        for i in range(n):
            exact = fa + (fb - fa) * i / (n - 1)
            # two roundings (the step, then start + i * step) away from the line
            err = abs(Fraction(x[i]) - exact)
            assert err <= Fraction(4 * (abs(a) + abs(b))) * Fraction(1, 2 ** 52) * max(1, i), (i, n)
        d = np.diff(x)
        assert np.all(d > 0) if b > a else np.all(d < 0)


def test_linspace_agrees_with_numpy_within_rounding():
    for a, b, n in ((0.0, 1.0, 1001), (-3.5, 7.25, 17), (1e-3, 1e3, 50)):
        x = oracle.linspace_values(a, b, n)
        assert np.allclose(x, np.linspace(a, b, n), rtol=1e-14, atol=1e-15 * max(abs(a), abs(b)))


def test_linspace_storage_rounds_once():
    # the FP64 value is rounded once to the storage type
    x = oracle.linspace_values(0.0, 1.0, 11)
    assert np.array_equal(values(oracle.linspace(0.0, 1.0, 11, "f32")).ravel(),
                          x.astype(np.float32).astype(np.float64))
    assert np.array_equal(values(oracle.linspace(0.0, 1.0, 11, "f16")).ravel(),
                          x.astype(np.float16).astype(np.float64))
    assert values(oracle.linspace(0.0, 1.0, 11, "f64", row=True)).shape == (1, 11)


def test_generators_as_leaves_of_trees():
    g = np.random.default_rng(5)
    A = g.uniform(-1, 1, (6, 6))
    E = oracle.eye(6, 6, "f64")
    got = oracle.evaluate((X + leaf(1)).postfix(), [synth.Mat(np.asfortranarray(A), "f64"), E])
    assert np.array_equal(got, A + np.eye(6))
    # trans(eye(r, c)) is eye(c, r)
    got = oracle.evaluate(trans(X).postfix(), [oracle.eye(3, 5, "f64")])
    assert np.array_equal(got, np.eye(5, 3))
    # accu(linspace(0, 1, 5)) = 2.5; the sum of linspace(1, n, n) is n (n + 1) / 2
    assert oracle.reduce("accu", X.postfix(), [oracle.linspace(0.0, 1.0, 5)])[0][0] == 2.5
    assert oracle.reduce("accu", X.postfix(), [oracle.linspace(1.0, 1000.0, 1000)])[0][0] == 500500.0


def test_view_definitions():
    """The views are slices of the stored matrix: trace = sum of the diagonal,
    diagvec(A, k) = the k-th diagonal as a column."""
    g = np.random.default_rng(11)
    A = g.uniform(-1, 1, (7, 9))
    for k in (-3, 0, 2):
        d = np.diagonal(A, k).copy()
        assert np.array_equal(d, [A[i - min(k, 0), i + max(k, 0)] for i in range(d.size)])
        col = oracle.evaluate(trans(X).postfix(), [synth.Mat(np.asfortranarray(d.reshape(1, -1)), "f64")])
        assert np.array_equal(col[:, 0], d)
    S = g.uniform(-1, 1, (50, 50))
    t = oracle.reduce("accu", X.postfix(), [synth.Mat(np.asfortranarray(np.diagonal(S).reshape(1, -1)), "f64")])[0][0]
    assert abs(t - np.trace(S)) <= 1e-14 * np.sum(np.abs(np.diagonal(S)))
