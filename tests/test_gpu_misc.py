"""GPU parity of Table 7's misc and trig functions in fused trees against the
CPU oracle.  Correctly rounded functions (square, floor, ceil, round, trunc,
sign) must equal the oracle's per-node rounded evaluation bit for bit; the
transcendental ones (pow, log10, log2, exp2, cos ... tanh) are within 1e-6
(FP32) or 1e-14 (FP64) of the exact FP64 value in the running-error scale S;
non-finite classes match (acos(2) is NaN, log10(0) is -inf)."""
import numpy as np
import pytest

import oracle
import synth
from synth import (acos, asin, atan, ceil, cos, cosh, exp2, floor, leaf, leaves, log2, log10, pow_, round_, sign,
                   sin, sinh, square, tan, tanh, trunc)

from gpu_util import classes_match, dev, empty, host, need_gpu, same, scaled_err, sum_gate, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

X = leaf(0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


@pytest.fixture(scope="module")
def g():
    return np.random.default_rng(7171)


def mat(g, shape, dt, lo, hi):
    return synth.Mat(synth.store(np.asfortranarray(g.uniform(lo, hi, shape)), dt), dt)


def run(tree, mats):
    r, c, p = oracle.shape(tree.postfix(), mats)
    Y = empty(r, c, "f64" if p == 64 else "f32")
    coot.eval(tree, [dev(m) for m in mats], Y)
    torch.cuda.synchronize()
    return host(Y), p


def check(tree, mats, exact):
    got, p = run(tree, mats)
    em = oracle.evaluate(tree.postfix(), mats, "emu")
    assert classes_match(got, em)
    if exact:
        assert same(got, em)
    ex, S = oracle.evaluate(tree.postfix(), mats, "exact", scale=True)
    fin = np.isfinite(ex) & np.isfinite(got)
    e = scaled_err(got[fin], ex[fin], S[fin])
    assert e <= (1e-6 if p == 32 else 1e-14), e


EXACT = [("square", square, -3, 3), ("floor", floor, -5, 5), ("ceil", ceil, -5, 5), ("round", round_, -5, 5),
         ("trunc", trunc, -5, 5), ("sign", sign, -1, 1)]
TRANSC = [("log10", log10, 0.01, 100), ("log2", log2, 0.01, 100), ("exp2", exp2, -20, 20),
          ("pow", lambda x: pow_(x, 2.5), 0.1, 10), ("pow_neg", lambda x: pow_(x, -1.5), 0.1, 10),
          ("cos", cos, -10, 10), ("sin", sin, -10, 10), ("tan", tan, -1.4, 1.4), ("acos", acos, -1, 1),
          ("asin", asin, -1, 1), ("atan", atan, -50, 50), ("cosh", cosh, -8, 8), ("sinh", sinh, -8, 8),
          ("tanh", tanh, -5, 5)]


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("name,f,lo,hi", EXACT, ids=[e[0] for e in EXACT])
def test_correctly_rounded_functions(g, dt, name, f, lo, hi):
    A = mat(g, (333, 77), dt, lo, hi)
    check(f(X), [A], True)
    check(f(X * 0.5 + 0.25), [A], True)


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
@pytest.mark.parametrize("name,f,lo,hi", TRANSC, ids=[e[0] for e in TRANSC])
def test_transcendental_functions(g, dt, name, f, lo, hi):
    A = mat(g, (333, 77), dt, lo, hi)
    check(f(X), [A], False)


def test_rounding_halfway_cases_and_signs():
    v = np.array([-2.5, -1.5, -0.5, 0.5, 1.5, 2.5, -0.0, 0.0, 3.0, -2.7, np.inf, -np.inf, np.nan], np.float32)
    A = synth.Mat(np.asfortranarray(v.reshape(-1, 1)), "f32")
    for f in (floor, ceil, round_, trunc, sign, square):
        got, _ = run(f(X), [A])
        em = oracle.evaluate(f(X).postfix(), [A], "emu")
        assert same(got, em), f.__name__
        assert np.array_equal(np.signbit(got[~np.isnan(got)]), np.signbit(em[~np.isnan(em)])), f.__name__


def test_out_of_domain_classes():
    v = np.array([2.0, -2.0, 0.0, -1.0, np.inf, np.nan], np.float32)
    A = synth.Mat(np.asfortranarray(v.reshape(-1, 1)), "f32")
    for f in (acos, asin, log10, log2, lambda x: pow_(x, 0.5), tan, exp2, cosh):
        got, _ = run(f(X), [A])
        assert classes_match(got, oracle.evaluate(f(X).postfix(), [A], "emu"))


def test_mixed_tree_and_reduction(g):
    A, B = mat(g, (500, 400), "f32", 0.1, 2.0), mat(g, (400, 500), "f32", -1, 1)
    x, y = leaves(2)
    t = sin(synth.trans(x)) % square(y) + pow_(synth.trans(x), 1.5) - floor(y * 4.0)
    check(t, [A, B], False)
    s = coot.reduce("accu", t, [dev(A), dev(B)]).double().item()
    o, _, asum = oracle.reduce("accu", t.postfix(), [A, B], mode="emu")
    sum_gate(s, o, asum, 500 * 400, 1e-6, what="accu of the mixed tree")
    # unfused per-node evaluation gives the same bits as the fused kernel
    Y1, Y2 = empty(400, 500, "f32"), empty(400, 500, "f32")
    coot.eval(t, [dev(A), dev(B)], Y1)
    coot.eval(t, [dev(A), dev(B)], Y2, unfused=True)
    torch.cuda.synchronize()
    assert same(host(Y1), host(Y2))
