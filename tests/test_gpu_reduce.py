"""GPU parity of fused reductions against the CPU oracle.

Gates: FP32 sums within 1e-6 relative of the exact value (or, only where the
sum is ill-conditioned, kappa * n * u^2 > 1e-7, within 1e-6 of the sum of
|terms|); min/max values bit-exact against
the oracle's per-node rounded values; indices bit-exact (lowest index on ties);
FP64 sums within 1e-13 relative.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import abs_, exp, leaf, leaves, sqrt, trans

from gpu_util import U_FP32, U_FP64, dev, empty, host, need_gpu, rel, same, sum_gate, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

X = leaf(0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


@pytest.fixture(scope="module")
def g():
    return np.random.default_rng(4242)


def mat(g, shape, dt, lo=-1.0, hi=1.0):
    return synth.Mat(synth.store(np.asfortranarray(g.uniform(lo, hi, shape)), dt), dt)


def gpu_reduce(op, tree, mats, dim=-1, **kw):
    out = coot.reduce(op, tree, [dev(m) for m in mats], dim=dim, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check_sum(op, tree, mats, dim=-1, tol=1e-6, **kw):
    """The summation is gated against the exact sum of the tree values as the
    method evaluates them (rounded at every node); for trees that are exact in
    the compute precision this is the exact FP64 reference itself.  Relative
    error, except for ill-conditioned results (sum_gate)."""
    got = gpu_reduce(op, tree, mats, dim, **kw).astype(np.float64)
    o, _, asum = oracle.reduce(op, tree.postfix(), mats, dim=dim, mode="emu")
    r, c, prec = oracle.shape(tree, mats)
    n = r * c if dim < 0 else (r if dim == 0 else c)
    sum_gate(got, o, asum, n, tol, u=U_FP64 if prec == 64 else U_FP32, what=op,
             nonneg=op in ("norm1", "norm2"))
    return got


def check_sel(op, tree, mats, dim=-1):
    got = gpu_reduce(op, tree, mats, dim)
    v, i, _ = oracle.reduce(op, tree.postfix(), mats, dim=dim, mode="emu")
    if op.startswith("index"):
        assert np.array_equal(got.astype(np.int64), i), (got[:8], i[:8])
    else:
        assert same(got.astype(np.float64), v), (got[:8], v[:8])


@pytest.mark.parametrize("dt", ["f32", "f64", "f16", "bf16"])
def test_accu_of_ones_is_n(dt):
    n = (1 << 20) + 3
    ones = synth.store(np.ones(n), dt)
    M = synth.Mat(np.asfortranarray(ones.reshape(-1, 1)), dt)
    assert gpu_reduce("accu", X, [M])[0] == n
    assert gpu_reduce("accu", X, [M], pairwise=True)[0] == n


def test_sum_of_0_to_n_minus_1():
    n = 1 << 24
    v64 = synth.Mat(np.asfortranarray(np.arange(n, dtype=np.float64).reshape(-1, 1)), "f64")
    assert gpu_reduce("accu", X, [v64])[0] == n * (n - 1) / 2
    v32 = synth.Mat(np.asfortranarray(np.arange(n, dtype=np.float32).reshape(-1, 1)), "f32")
    assert rel(float(gpu_reduce("accu", X, [v32])[0]), n * (n - 1) / 2) <= 1e-6


@pytest.mark.parametrize("dt", ["f32", "f64", "f16", "bf16"])
@pytest.mark.parametrize("n", [1, 63, 4097, 1_000_003])
def test_sums_all(g, dt, n):
    a, b = mat(g, (n, 1), dt), mat(g, (n, 1), dt)
    tol = 1e-6 if dt != "f64" else 1e-13
    check_sum("accu", X, [a], tol=tol)
    check_sum("dot", leaf(0) % leaf(1), [a, b], tol=tol)
    check_sum("norm2", X, [a], tol=tol)
    check_sum("norm1", X, [a], tol=tol)
    check_sum("accu", sqrt(abs_(leaf(0))) % leaf(1) + 1.0, [a, b], tol=tol)


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
@pytest.mark.parametrize("op", ["min", "max", "index_min", "index_max", "norminf", "normneginf"])
def test_selections_all(g, dt, op):
    A = synth.Mat(synth.store(np.asfortranarray(g.integers(-50, 50, (1237, 311)).astype(np.float64)), dt), dt)
    check_sel(op, X, [A])
    check_sel(op, abs_(leaf(0)) * 0.5, [A])


@pytest.mark.parametrize("shape", [(1000, 1000), (5000, 7), (7, 5000), (63, 129), (64, 64), (3, 3), (1, 999), (999, 1)])
def test_dim_reductions(g, shape):
    A = mat(g, shape, "f32")
    for dim in (0, 1):
        check_sum("sum", X, [A], dim=dim)
        check_sum("sum", leaf(0) % leaf(0) - 0.25, [A], dim=dim)
        check_sel("max", X, [A], dim)
        check_sel("index_min", X, [A], dim)


@pytest.mark.parametrize("shape", [(100_003, 2), (1 << 20, 3), (300_001, 1), (4097, 17)])
def test_dim0_of_few_long_columns(g, shape):
    """Few long columns are cut into row segments combined in order."""
    for dt in ("f32", "bf16", "f64"):
        A = mat(g, shape, dt)
        tol = 1e-13 if dt == "f64" else 1e-6
        check_sum("sum", X, [A], dim=0, tol=tol)
        check_sel("index_max", X, [A], 0)
        check_sel("min", abs_(leaf(0)), [A], 0)
    A = synth.Mat(synth.store(np.asfortranarray(g.integers(-3, 4, shape).astype(np.float64)), "f32"), "f32")
    check_sel("index_min", X, [A], 0)   # many ties across segments: the lowest row must win


def test_dim_reductions_f64_and_16bit(g):
    for dt, tol in (("f64", 1e-13), ("bf16", 1e-6), ("f16", 1e-6)):
        A = mat(g, (700, 300), dt)
        for dim in (0, 1):
            check_sum("sum", X, [A], dim=dim, tol=tol)
            check_sel("min", X, [A], dim)


def test_dim_reduction_of_transposed_tree(g):
    A, B = mat(g, (90, 200), "f32"), mat(g, (200, 90), "f32")
    t = trans(leaf(0)) + 0.5 * leaf(1)
    for dim in (0, 1):
        check_sum("sum", t, [A, B], dim=dim)
        check_sel("index_max", t, [A, B], dim)
    check_sum("accu", t % t, [A, B])
    check_sel("max", t, [A, B])


@pytest.mark.parametrize("r,c", [(2, 3000), (3000, 2), (12, 300), (300, 12), (1, 70), (70, 1), (63, 65), (5, 7)])
def test_thin_transposed_reductions(g, r, c):
    """Full reductions over thin transposed trees (shape-adaptive tiles): sums,
    extrema and the linear index of the extremum."""
    A, B = mat(g, (r, c), "f32"), mat(g, (c, r), "f32")
    t = trans(leaf(0)) + 0.5 * leaf(1)
    check_sum("accu", t, [A, B])
    check_sum("accu", t % t, [A, B])
    check_sel("index_max", t, [A, B])
    check_sel("index_min", t, [A, B])
    check_sel("max", t, [A, B])
    A64, B64 = mat(g, (r, c), "f64"), mat(g, (c, r), "f64")
    check_sum("accu", t, [A64, B64], tol=1e-13)
    check_sel("index_max", t, [A64, B64])


@pytest.mark.parametrize("shape", [(524288, 4), (1000, 5000), (3, 100000), (4097, 17), (8, 524288), (300, 200000)])
def test_row_reductions_narrow_and_split(g, shape):
    """Per-row reductions: narrow rows in one pass; few long rows split over
    column ranges, the splits combined per row in order by one thread."""
    A = mat(g, shape, "f32")
    check_sum("sum", X, [A], dim=1)
    check_sel("index_max", X, [A], 1)
    check_sel("min", X, [A], 1)
    D = mat(g, shape, "f64")
    check_sum("sum", X % X, [D], dim=1, tol=1e-13)


def test_dim_reduction_with_ld_view(g):
    A = mat(g, (300, 50), "f32")
    dA = dev(A, ld=333)
    for dim in (0, 1):
        got = coot.reduce("sum", X, [dA], dim=dim).cpu().numpy().astype(np.float64)
        o, _, _ = oracle.reduce("sum", X.postfix(), [A], dim=dim)
        assert np.max(np.abs(got - o) / np.abs(o)) <= 1e-6


def test_index_ties_lowest_wins():
    d = synth.cfg2_inputs("f32", n=(1 << 20) + 17, n_ties=64)
    M = synth.Mat(np.asfortranarray(d["x"].reshape(-1, 1)), "f32")
    assert int(gpu_reduce("index_max", X, [M])[0]) == d["ties"].min()
    N = synth.Mat(np.asfortranarray((-d["x"]).reshape(-1, 1)), "f32")
    assert int(gpu_reduce("index_max", abs_(leaf(0)), [N])[0]) == d["ties"].min()
    assert int(gpu_reduce("index_min", X, [N])[0]) == d["ties"].min()


def test_nan_skipped():
    v = np.full(10_000, np.nan, np.float32)
    v[777] = 2.0
    v[5000] = 2.0
    v[9000] = -3.0
    M = synth.Mat(np.asfortranarray(v.reshape(-1, 1)), "f32")
    assert int(gpu_reduce("index_max", X, [M])[0]) == 777
    assert gpu_reduce("min", X, [M])[0] == -3.0
    allnan = synth.Mat(np.asfortranarray(np.full((100, 1), np.nan, np.float32)), "f32")
    assert np.isnan(gpu_reduce("max", X, [allnan])[0])
    assert int(gpu_reduce("index_max", X, [allnan])[0]) == 0


def test_empty_inputs():
    E0 = synth.Mat(np.zeros((0, 4), np.float32, order="F"), "f32")
    assert gpu_reduce("accu", X, [E0])[0] == 0.0
    s = gpu_reduce("sum", X, [E0], dim=0)
    assert np.array_equal(s, np.zeros(4, np.float32))
    with pytest.raises(coot.CootError) as e:
        gpu_reduce("max", X, [E0])
    assert e.value.code == -5


def test_host_output(g):
    A = mat(g, (12345, 1), "f32")
    out = torch.zeros(1, dtype=torch.float64)  # host memory
    coot.lib()
    e = coot.expr(X)
    arr, n = coot._ops([dev(A)])
    o = coot.operand(out, host=True)
    import ctypes as C

    rc = coot.lib().coot_reduce(coot.REDS["accu"], -1, C.byref(e), arr, n, C.byref(o), coot.current_stream())
    assert rc == 0, coot.last_error()
    o_, _, _ = oracle.reduce("accu", X.postfix(), [A])
    assert rel(out.item(), o_[0]) <= 1e-6


def test_deterministic(g):
    A = mat(g, (3_000_001, 1), "f32")
    B = mat(g, (3_000_001, 1), "f32")
    dA, dB = dev(A), dev(B)
    first = coot.reduce("dot", leaf(0) % leaf(1), [dA, dB]).item()
    for _ in range(10):
        assert coot.reduce("dot", leaf(0) % leaf(1), [dA, dB]).item() == first


def test_accu_of_product_equals_dot(g):
    A, B = mat(g, (100_000, 1), "f32"), mat(g, (100_000, 1), "f32")
    a = gpu_reduce("accu", leaf(0) % leaf(1), [A, B])[0]
    d = gpu_reduce("dot", leaf(0) % leaf(1), [A, B])[0]
    assert a == d


def test_dot_xx_vs_norm_squared(g):
    A = mat(g, (1_000_000, 1), "f32")
    d = float(gpu_reduce("dot", leaf(0) % leaf(0), [A])[0])
    n = float(gpu_reduce("norm2", X, [A])[0])
    assert abs(d - n * n) <= 3 * 2.0 ** -24 * d


def test_pairwise_variant_runs(g):
    A = mat(g, (2_000_000, 1), "f32")
    check_sum("accu", X, [A], tol=1e-4, pairwise=True)


def test_unfused_reductions(g):
    A, B = mat(g, (50_000, 1), "f32"), mat(g, (50_000, 1), "f32")
    check_sum("dot", leaf(0) % leaf(1), [A, B], unfused=True)
    got = gpu_reduce("index_max", abs_(leaf(0)), [A], unfused=True)
    _, i, _ = oracle.reduce("index_max", abs_(leaf(0)).postfix(), [A], mode="emu")
    assert int(got[0]) == i[0]
