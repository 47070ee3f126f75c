"""Pins of the oracle's element-wise evaluation against things other than itself.

* IEEE single/double arithmetic through numpy (+, -, *, /, sqrt are correctly
  rounded by IEEE 754, so numpy float32 results are the textbook values);
* numpy's transpose and Fortran-order slicing for the column-major layout
  (Section 2, Table 1) and trans (Table 7);
* library conversions (numpy float16, torch bfloat16) for the storage rounding;
* hand-computed values (tests/golden/elementwise_small.json);
* the running-error scale S as a bound on |EMU - EXACT|.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from synth import E, abs_, exp, leaf, leaves, log, sqrt, trans, conv

HERE = os.path.dirname(os.path.abspath(__file__))


def f32mat(g, r, c, lo=-2.0, hi=2.0):
    return synth.Mat(np.asfortranarray(g.uniform(lo, hi, (r, c)).astype(np.float32)), "f32")


def f64mat(g, r, c, lo=-2.0, hi=2.0):
    return synth.Mat(np.asfortranarray(g.uniform(lo, hi, (r, c))), "f64")


@pytest.fixture(scope="module")
def g():
    return np.random.default_rng(12345)


BIN_NUMPY = {
    "plus": lambda a, b: a + b,
    "minus": lambda a, b: a - b,
    "schur": lambda a, b: a * b,
    "div": lambda a, b: a / b,
}

SCAL_NUMPY = {
    "scal_plus": lambda a, k: a + k,
    "scal_minus_post": lambda a, k: a - k,
    "scal_minus_pre": lambda a, k: k - a,
    "scal_times": lambda a, k: a * k,
    "scal_div_post": lambda a, k: a / k,
    "scal_div_pre": lambda a, k: k / a,
}


@pytest.mark.parametrize("op", list(BIN_NUMPY))
def test_binary_emu_equals_ieee_single(g, op):
    A, B = f32mat(g, 37, 11), f32mat(g, 37, 11)
    tree = [synth.Node("leaf", 0), synth.Node("leaf", 1), synth.Node(op, 0, 1)]
    got = oracle.evaluate(tree, [A, B], "emu")
    with np.errstate(all="ignore"):
        want = BIN_NUMPY[op](A.data, B.data).astype(np.float64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("op", list(BIN_NUMPY))
def test_binary_exact_equals_ieee_double(g, op):
    A, B = f64mat(g, 13, 29), f64mat(g, 13, 29)
    tree = [synth.Node("leaf", 0), synth.Node("leaf", 1), synth.Node(op, 0, 1)]
    got = oracle.evaluate(tree, [A, B], "exact")
    assert np.array_equal(got, BIN_NUMPY[op](A.data, B.data))


@pytest.mark.parametrize("op", list(SCAL_NUMPY))
@pytest.mark.parametrize("k", [0.75, 2.5, -3.0, 0.1])
def test_scalar_emu_equals_ieee_single(g, op, k):
    A = f32mat(g, 64, 3)
    tree = [synth.Node("leaf", 0), synth.Node(op, 0, -1, k)]
    got = oracle.evaluate(tree, [A], "emu")
    # the scalar is the literal converted to the element type (float)
    want = SCAL_NUMPY[op](A.data, np.float32(k)).astype(np.float64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("fn,npf", [("sqrt", np.sqrt), ("abs", np.abs)])
def test_sqrt_abs_emu_equals_ieee_single(g, fn, npf):
    A = f32mat(g, 100, 7, 0.0, 1e4)
    A.data[0, 0] = 0.0
    A.data[1, 0] = np.float32(4.0)
    A.data[2, 0] = np.float32(1e-40)  # subnormal single
    tree = [synth.Node("leaf", 0), synth.Node(fn, 0)]
    got = oracle.evaluate(tree, [A], "emu")
    assert np.array_equal(got, npf(A.data).astype(np.float64))
    if fn == "sqrt":
        assert got[1, 0] == 2.0


def test_abs_of_negative_zero_is_positive_zero():
    A = synth.Mat(np.asfortranarray(np.array([[-0.0]], np.float32)), "f32")
    v = oracle.evaluate([synth.Node("leaf", 0), synth.Node("abs", 0)], [A], "emu")
    assert v[0, 0] == 0.0 and math.copysign(1.0, v[0, 0]) == 1.0


def test_x_minus_x_and_power_of_two_scaling(g):
    A = f32mat(g, 50, 4)
    x = leaf(0)
    assert np.all(oracle.evaluate((x - x).postfix(), [A], "emu") == 0.0)
    half = oracle.evaluate((0.5 * x).postfix(), [A], "emu")
    assert np.array_equal(half, A.data.astype(np.float64) / 2)


def test_exp_log_closed_forms():
    A = synth.Mat(np.asfortranarray(np.array([[0.0], [1.0]], np.float64)), "f64")
    e = oracle.evaluate((exp(leaf(0))).postfix(), [A], "exact")
    lg = oracle.evaluate((log(leaf(0))).postfix(), [A], "exact")
    assert e[0, 0] == 1.0 and lg[1, 0] == 0.0 and lg[0, 0] == -math.inf


def test_exp_log_round_trip_and_library(g):
    x = f64mat(g, 200, 5, 1e-3, 50.0)
    rt = oracle.evaluate(exp(log(leaf(0))).postfix(), [x], "exact")
    assert np.max(np.abs(rt - x.data) / x.data) < 1e-14
    e = oracle.evaluate(exp(leaf(0)).postfix(), [x], "exact")
    assert np.max(np.abs(e - np.exp(x.data)) / np.exp(x.data)) < 4e-16
    xs = f32mat(g, 300, 2, -20.0, 20.0)
    es = oracle.evaluate(exp(leaf(0)).postfix(), [xs], "emu")
    # single precision exp = the double-precision library exp rounded once to float
    want = np.exp(xs.data.astype(np.float64)).astype(np.float32).astype(np.float64)
    assert np.array_equal(es, want)


def test_column_major_and_trans(g):
    A = f32mat(g, 5, 3)
    t = oracle.evaluate(trans(leaf(0)).postfix(), [A], "exact")
    assert t.shape == (3, 5)
    assert np.array_equal(t, A.data.T.astype(np.float64))
    # trans(trans(X)) is X; trans of a product is the product of transposes
    tt = oracle.evaluate(trans(trans(leaf(0))).postfix(), [A], "exact")
    assert np.array_equal(tt, A.data.astype(np.float64))
    B = f32mat(g, 3, 5)
    v = oracle.evaluate((trans(leaf(0)) % leaf(1)).postfix(), [A, B], "emu")
    assert np.array_equal(v, (A.data.T * B.data).astype(np.float64))


def test_evaluate_at_agrees_with_unfused(g):
    mats = [f32mat(g, 17, 9), f32mat(g, 17, 9), f32mat(g, 9, 17)]
    a, b, c = leaves(3)
    t = sqrt(abs_(a)) % b - a / (1.0 + abs_(b)) + trans(c) * 0.75
    full = oracle.evaluate(t.postfix(), mats, "emu")
    lin = np.arange(17 * 9)
    pts = oracle.evaluate_at(t.postfix(), mats, lin, "emu")
    assert np.array_equal(pts, full.reshape(-1, order="F"))
    # the pointwise running-error scale is the unfused one, element for element
    for mode in ("emu", "exact"):
        v, S = oracle.evaluate(t.postfix(), mats, mode, scale=True)
        pv, pS = oracle.evaluate_at(t.postfix(), mats, lin[::-1], mode, scale=True)
        assert np.array_equal(pv, v.reshape(-1, order="F")[::-1])
        assert np.array_equal(pS, S.reshape(-1, order="F")[::-1])


def test_pointwise_scale_of_z_by_hand(g):
    """S of z = sqrt|x| % y - x / (1 + |y|), derived by hand from the
    first-order rules: S(sqrt|x|) = sqrt|x| + |x| / (2 sqrt|x|) = 1.5 sqrt|x|,
    times S(y) = |y|; S(1 + |y|) = 1 + |y|, so S(x / (1 + |y|)) =
    (|x| + |x| (1 + |y|) / (1 + |y|)) / (1 + |y|) = 2|x| / (1 + |y|); the
    difference adds the two."""
    x = g.standard_normal(4000)
    y = g.standard_normal(4000)
    tree = synth.cfg2_trees()["z"]
    lin = np.arange(4000)[::7]
    v, S = oracle.evaluate_at(tree.postfix(), [x, y], lin, "exact", scale=True)
    xs, ys = x[lin], y[lin]
    want = 1.5 * np.sqrt(np.abs(xs)) * np.abs(ys) + 2.0 * np.abs(xs) / (1.0 + np.abs(ys))
    # both sides are sums of positive terms, each term a handful of correctly
    # rounded operations (at most 8 along the oracle's rule chain, 4 here):
    # they agree to 12 units of roundoff; a dropped or doubled term is O(1)
    assert np.max(np.abs(S - want) / want) <= 12 * 2.0**-53
    assert np.max(np.abs(v - (np.sqrt(np.abs(xs)) * ys - xs / (1.0 + np.abs(ys))))) <= 1e-15 * np.max(want)


def test_leading_dimension_view(g):
    # an operand with ld > n_rows (a submatrix view) reads element (r, c) at r + c*ld
    big = np.asfortranarray(g.uniform(-1, 1, (10, 6)).astype(np.float32))
    sub = big[2:7, 1:5]  # 5 x 4 view, Fortran strides (4, 40)
    got = oracle.evaluate((2.5 * leaf(0)).postfix(), [synth.Mat(np.asfortranarray(sub), "f32")], "emu")
    assert np.array_equal(got, (np.float32(2.5) * sub).astype(np.float64))


def test_cfg1_tree_against_numpy_single(g):
    mats = synth.cfg1_inputs(40, 30)
    A, B, C, D = (mats[k].data for k in "ABCD")
    tree = synth.cfg1_trees()["Y"]
    got = oracle.evaluate(tree.postfix(), [mats[k] for k in "ABCD"], "emu")
    arith = np.float32(2.5) * A + B * C
    ex = np.exp(D.astype(np.float64)).astype(np.float32)  # correctly rounded single exp
    assert np.array_equal(got, (arith - ex).astype(np.float64))


def test_golden_hand_values():
    with open(os.path.join(HERE, "golden", "elementwise_small.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        mats = [synth.Mat(np.asfortranarray(np.array(m, np.float64).reshape(case["shape"], order="F")), "f64")
                for m in case["operands"]]
        tree = [synth.Node(n[0], n[1], n[2], n[3]) for n in case["tree"]]
        got = oracle.evaluate(tree, mats, "exact").reshape(-1, order="F")
        assert np.allclose(got, case["expect"], rtol=1e-15, atol=0), case["name"]


def test_conversion_node_rounds_to_target(g):
    x = f64mat(g, 40, 3, -100, 100)
    for dt in ("f32", "f16", "bf16"):
        got = oracle.evaluate(conv(leaf(0), dt).postfix(), [x], "exact")
        want = oracle.round_to(dt, x.data.reshape(-1, order="F")).reshape(x.shape, order="F")
        assert np.array_equal(got, want)


def test_round_to_f16_matches_numpy(g):
    v = np.concatenate([
        g.uniform(-70000, 70000, 20000),
        g.standard_normal(20000) * 1e-5,            # subnormal range of binary16
        np.array([65504.0, 65519.99, 65520.0, 1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11, 2 ** -25, 2 ** -24 * 1.5, 0.0, -0.0]),
    ])
    got = oracle.round_to("f16", v)
    want = v.astype(np.float16).astype(np.float64)
    assert np.array_equal(got, want)


def test_round_to_bf16_matches_torch(g):
    torch = pytest.importorskip("torch")
    v = np.concatenate([g.standard_normal(20000) * 10.0 ** g.integers(-30, 30, 20000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.3895313892515355e38, 1e-40])]).astype(np.float32)
    got = oracle.round_to("bf16", v.astype(np.float64))
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(got, want)


def test_round_to_f32_matches_numpy(g):
    v = g.standard_normal(10000) * 10.0 ** g.integers(-40, 38, 10000)
    assert np.array_equal(oracle.round_to("f32", v), v.astype(np.float32).astype(np.float64))


def test_widen16_matches_libraries(g):
    torch = pytest.importorskip("torch")
    bits = np.arange(65536, dtype=np.uint16)
    w = oracle.widen16("f16", bits)
    ref = bits.view(np.float16).astype(np.float64)
    assert np.array_equal(w[~np.isnan(ref)], ref[~np.isnan(ref)]) and np.all(np.isnan(w[np.isnan(ref)]))
    wb = oracle.widen16("bf16", bits)
    refb = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    nan = np.isnan(refb)
    assert np.array_equal(wb[~nan], refb[~nan]) and np.all(np.isnan(wb[nan]))


def test_sixteen_bit_leaves_compute_in_single(g):
    x = g.uniform(-3, 3, (20, 5))
    for dt in ("f16", "bf16"):
        M = synth.Mat(synth.store(np.asfortranarray(x), dt), dt)
        wide = oracle.widen16(dt, M.data.reshape(-1, order="F")).reshape(M.shape, order="F")
        got = oracle.evaluate((leaf(0) % leaf(0) + 0.1).postfix(), [M], "emu")
        w32 = wide.astype(np.float32)
        assert np.array_equal(got, (w32 * w32 + np.float32(0.1)).astype(np.float64))


def test_scale_bounds_emulation_error(g):
    """|EMU32 - EXACT| <= k * 2^-24 * S for a tree with k roundings on its longest path."""
    mats = [f32mat(g, 300, 10) for _ in range(3)]
    a, b, c = leaves(3)
    cases = [(a + b, 1), (a % b - c, 2), (2.5 * a + b % c, 2), (a / (1.0 + abs_(b)), 2),
             (sqrt(abs_(a)) % b - a / (1.0 + abs_(b)), 3), (trans(trans(a)) - 0.75 * b, 2)]
    u = 2.0 ** -24
    for t, k in cases:
        ex, S = oracle.evaluate(t.postfix(), mats, "exact", scale=True)
        em = oracle.evaluate(t.postfix(), mats, "emu")
        assert np.all(S >= np.abs(ex) * (1 - 1e-15))
        assert np.all(np.abs(em - ex) <= k * u * S * (1 + 1e-12))


def test_scale_equals_value_for_positive_sums_and_products(g):
    mats = [f64mat(g, 30, 4, 0.1, 3.0) for _ in range(3)]
    a, b, c = leaves(3)
    t = a % b + c % a + 2.0 * b
    ex, S = oracle.evaluate(t.postfix(), mats, "exact", scale=True)
    assert np.allclose(S, ex, rtol=1e-14)


def test_shape_and_precision_errors(g):
    A, B = f32mat(g, 3, 4), f32mat(g, 4, 3)
    with pytest.raises(oracle.OracleError) as e:
        oracle.evaluate((leaf(0) + leaf(1)).postfix(), [A, B])
    assert e.value.code == -2
    C = f64mat(g, 3, 4)
    with pytest.raises(oracle.OracleError):
        oracle.evaluate((leaf(0) + leaf(1)).postfix(), [A, C])
    # explicit conversion makes the mixed expression legal
    v = oracle.evaluate((conv(leaf(0), "f64") + leaf(1)).postfix(), [A, C], "exact")
    assert np.array_equal(v, A.data.astype(np.float64) + C.data)
