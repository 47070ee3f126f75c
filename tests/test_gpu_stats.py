"""GPU parity of relational nodes (Table 5's all(A < x), Section 3's A > 0.3)
and of the statistics reductions (Table 6: mean, var, stddev; Table 5: all,
any; the count of nonzero elements) against the CPU oracle.

Gates: relational trees are bit-exact against the oracle's per-node rounded
evaluation (a comparison is exact for the operands it is given); count, all
and any are exact; the mean follows the sum gate (1e-6 relative for FP32
data, 1e-13 for FP64; the summed terms' scale stands in only for
ill-conditioned sums); var and stddev, accumulated in FP64 for every storage type, within
1e-12 relative of the oracle's two-pass variance of the same per-node rounded
values."""
import numpy as np
import pytest

import oracle
import synth
from synth import eq, leaf, leaves, ne, trans

from gpu_util import U_FP32, U_FP64, dev, empty, host, need_gpu, same, sum_gate, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

X = leaf(0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


@pytest.fixture(scope="module")
def g():
    return np.random.default_rng(6161)


def mat(g, shape, dt, lo=-1.0, hi=1.0):
    return synth.Mat(synth.store(np.asfortranarray(g.uniform(lo, hi, shape)), dt), dt)


def red(op, tree, mats, dim=-1, **kw):
    out = coot.reduce(op, tree, [dev(m) for m in mats], dim=dim, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check_exact_count(op, tree, mats, dim=-1):
    got = red(op, tree, mats, dim).astype(np.int64)
    _, want, _ = oracle.reduce(op, tree.postfix(), mats, dim=dim, mode="emu")
    assert np.array_equal(got, want), (op, dim, got[:6], want[:6])


def check_mean(tree, mats, dim=-1, f64=False):
    got = red("mean", tree, mats, dim).astype(np.float64)
    o, _, scale = oracle.reduce("mean", tree.postfix(), mats, dim=dim, mode="emu")
    tol = 1e-13 if f64 else 1e-6
    nan = np.isnan(o)
    assert np.array_equal(np.isnan(got), nan)
    r, c, prec = oracle.shape(tree, mats)
    n = r * c if dim < 0 else (r if dim == 0 else c)
    # the mean is a sum divided once: the sum's gate, with the oracle's mean of |terms|
    sum_gate(got[~nan], o[~nan], scale[~nan], n, tol, u=U_FP64 if prec == 64 else U_FP32, what=f"mean dim {dim}")


def check_var(op, tree, mats, dim=-1, tol=1e-12):
    got = red(op, tree, mats, dim).astype(np.float64)
    o, _, _ = oracle.reduce(op, tree.postfix(), mats, dim=dim, mode="emu")
    # the output is rounded once to its type (FP32 for FP32/16-bit trees)
    f32_out = mats[0].dtype != "f64"
    t = max(tol, 6e-8) if f32_out else tol
    for k in range(o.size):
        if np.isnan(o[k]):
            assert np.isnan(got[k])
            continue
        assert abs(got[k] - o[k]) <= t * abs(o[k]) or (o[k] == 0.0 and got[k] == 0.0), (op, k, got[k], o[k])


SPECIAL = np.array([-np.inf, -2.0, -0.0, 0.0, 0.3, 1.0, np.inf, np.nan])


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
def test_relational_nodes_bit_exact(dt):
    a = np.repeat(SPECIAL, 8).reshape(8, 8)
    b = np.tile(SPECIAL, 8).reshape(8, 8)
    A = synth.Mat(synth.store(np.asfortranarray(a), dt), dt)
    B = synth.Mat(synth.store(np.asfortranarray(b), dt), dt)
    x, y = leaves(2)
    odt = "f64" if dt == "f64" else "f32"
    for tree in (x > y, x < y, x >= y, x <= y, eq(x, y), ne(x, y), x > 0.3, 0.3 > x, x >= 0.0, x <= 1.0,
                 eq(x, 0.0), ne(x, 0.0), (x > y) % y + ne(x, 0.5) * 2.0 - (0.25 >= y)):
        Y = empty(8, 8, odt)
        coot.eval(tree, [dev(A), dev(B)], Y)
        torch.cuda.synchronize()
        em = oracle.evaluate(tree.postfix(), [A, B], "emu")
        assert same(host(Y), em), [n.op for n in tree.postfix()]


def test_relational_in_larger_and_transposed_trees(g):
    A, B = mat(g, (300, 700), "f32"), mat(g, (700, 300), "f32")
    x, y = leaves(2)
    for tree in ((trans(x) > y) % y, ne(trans(x) * 2.0, y) + (y <= 0.0)):
        Y = empty(700, 300, "f32")
        coot.eval(tree, [dev(A), dev(B)], Y)
        torch.cuda.synchronize()
        assert same(host(Y), oracle.evaluate(tree.postfix(), [A, B], "emu"))
    # unfused (one kernel per node) gives the same bits
    t = (x > 0.25) % x
    Y1, Y2 = empty(300, 700, "f32"), empty(300, 700, "f32")
    coot.eval(t, [dev(A)], Y1)
    coot.eval(t, [dev(A)], Y2, unfused=True)
    torch.cuda.synchronize()
    assert same(host(Y1), host(Y2))


@pytest.mark.parametrize("dt", ["f32", "f64", "f16", "bf16"])
@pytest.mark.parametrize("shape", [((1 << 20) + 3, 1), (1000, 300), (3, 100000), (100000, 3), (1000, 5000)])
def test_predicate_counts_exact(g, dt, shape):
    A = mat(g, shape, dt)
    for tree in (X > 0.3, 0.3 > X, ne(X, 0.0), X):
        for dim in (-1, 0, 1):
            if shape[1] == 1 and dim == 1 and shape[0] > 100000:
                continue
            check_exact_count("count", tree, [A], dim)
            check_exact_count("all", tree, [A], dim)
            check_exact_count("any", tree, [A], dim)


def test_all_any_on_all_true_and_all_false(g):
    A = mat(g, (513, 129), "f32", 0.5, 1.0)
    for dim in (-1, 0, 1):
        assert np.all(red("all", X > 0.25, [A], dim) == 1)
        assert np.all(red("any", X > 2.0, [A], dim) == 0)
        assert np.all(red("any", X > 0.75, [A], dim) == 1)
        assert np.all(red("all", X > 0.75, [A], dim) == 0)


@pytest.mark.parametrize("dt", ["f32", "f64", "f16", "bf16"])
@pytest.mark.parametrize("shape", [((1 << 20) + 3, 1), (1000, 300), (3, 100000), (100000, 3), (64, 64),
                                   (1000, 5000)])
def test_mean_var_stddev(g, dt, shape):
    """(1000, 5000) gives the per-row reductions 78 column splits: the
    combine of 16 to 255 splits by four waves per 64 rows."""
    A = mat(g, shape, dt, -2.0, 3.0)
    f64 = dt == "f64"
    for dim in (-1, 0, 1):
        check_mean(X, [A], dim, f64)
        check_var("var", X, [A], dim)
        check_var("stddev", X, [A], dim)
    check_mean(X > 0.5, [A], -1, f64)


def test_statistics_of_transposed_trees(g):
    A, B = mat(g, (90, 2000), "f32"), mat(g, (2000, 90), "f32")
    t = trans(leaf(0)) * 0.5 + leaf(1)
    for dim in (-1, 0, 1):
        check_mean(t, [A, B], dim)
        check_var("var", t, [A, B], dim)
        check_exact_count("count", trans(leaf(0)) > leaf(1), [A, B], dim)
    A2, B2 = mat(g, (3, 50000), "f64"), mat(g, (50000, 3), "f64")
    check_var("stddev", t, [A2, B2])


def test_variance_with_a_large_offset(g):
    # values near 1e4 with spread 1: the FP64 shifted sums keep the variance
    x = (1e4 + g.standard_normal(1 << 18)).astype(np.float32)
    A = synth.Mat(np.asfortranarray(x.reshape(-1, 1)), "f32")
    check_var("var", X, [A])
    D = synth.Mat(np.asfortranarray((1e8 + g.standard_normal(1 << 18)).reshape(-1, 1)), "f64")
    check_var("var", X, [D], tol=1e-9)


def test_statistics_special_cases(g):
    one = synth.Mat(np.asfortranarray(np.array([[3.5]], np.float32)), "f32")
    assert red("var", X, [one])[0] == 0.0
    assert red("mean", X, [one])[0] == 3.5
    const = synth.Mat(np.asfortranarray(np.full((4096, 3), 0.1, np.float32)), "f32")
    assert np.all(red("var", X, [const], 0) == 0.0)
    assert red("var", X, [const])[0] == 0.0
    withnan = mat(g, (5000, 2), "f32")
    withnan.data[777, 1] = np.nan
    v = red("var", X, [withnan], 0)
    assert v[0] == v[0] and np.isnan(v[1])
    assert red("count", ne(X, 0.0), [withnan])[0] == 10000
    e = torch.empty(0, device="cuda")
    assert np.isnan(coot.reduce("mean", X, [e]).item())
    assert np.isnan(coot.reduce("var", X, [e]).item())
    assert coot.reduce("count", X, [e]).item() == 0
    assert coot.reduce("all", X, [e]).item() == 1
    assert coot.reduce("any", X, [e]).item() == 0


def test_results_are_deterministic(g):
    A = mat(g, ((1 << 22) + 5, 1), "f32")
    for op in ("mean", "var", "count"):
        t = X > 0.1 if op == "count" else X
        r1 = red(op, t, [A])
        r2 = red(op, t, [A])
        assert np.array_equal(r1, r2)


def test_full_size_statistics_cfg2():
    """2^28-element FP32 x of the scale workload: mean, var, count(x > 0.3)."""
    d = synth.cfg2_inputs("f32")
    A = synth.Mat(np.asfortranarray(d["x"].reshape(-1, 1)), "f32")
    check_mean(X, [A])
    check_var("var", X, [A])
    check_exact_count("count", X > 0.3, [A])
