"""GPU parity of the 32-bit integer element types (I32, U32) and the
conversions between every storage type, against the CPU oracle: integer
leaves widen exactly and trees with them compute in FP64, so element-wise
results are bit-exact against the oracle's per-node evaluation, with the
output stored by the oracle's conversion rule (fraction toward zero, clamp,
NaN to 0); integer sums below 2^53 are exact; index results bit-exact."""
import numpy as np
import pytest

import oracle
import synth
from synth import conv, leaf, leaves, trans

from gpu_util import dev, need_gpu, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

x, y = leaves(2)
X = leaf(0)
TD = {"i32": torch.int32, "u32": torch.int32, "f32": torch.float32, "f64": torch.float64}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


@pytest.fixture(scope="module")
def g():
    return np.random.default_rng(5151)


def imat(g, shape, dt, lo, hi):
    return synth.Mat(synth.store(np.asfortranarray(g.integers(lo, hi, shape).astype(np.float64)), dt), dt)


def to_dev(m):
    """column-major device copy of an integer (or float) synth.Mat"""
    d = m.data
    if d.dtype == np.uint32:
        d = d.view(np.int32)
    t = torch.from_numpy(np.ascontiguousarray(d.T)).cuda()
    return t.t() if d.ndim == 2 else t


def out(r, c, dt):
    return torch.empty(c, r, dtype=TD[dt], device="cuda").t()


def operand(t, dt):
    o = coot.operand(t)
    o.dtype = coot.DTYPE_CODES[dt]      # u32 data travels in int32 tensors
    return o


def values(t, dt):
    a = t.cpu().numpy()
    if dt == "u32":
        a = a.view(np.uint32)
    return a.astype(np.float64)


@pytest.mark.parametrize("idt", ["i32", "u32"])
@pytest.mark.parametrize("odt", ["i32", "u32", "f32", "f64"])
@pytest.mark.parametrize("shape", [(1000, 1), (333, 77), (77, 333)])
def test_integer_trees_bit_exact(g, idt, odt, shape):
    lo, hi = (-2 ** 31, 2 ** 31) if idt == "i32" else (0, 2 ** 32)
    A = imat(g, shape, idt, lo, hi)
    B = synth.Mat(np.asfortranarray(g.uniform(-3e9, 3e9, shape)), "f64")
    trees = [x * 0.5 + y, x - y, (x > y) + x / 3.0, x % y]
    dA, dB = to_dev(A), dev(B)          # kept alive: an Operand holds only the pointer
    for tree in trees:
        Y = out(shape[0], shape[1], odt)
        coot.eval(tree, [operand(dA, idt), dB], operand(Y, odt))
        torch.cuda.synchronize()
        ref = oracle.evaluate(tree.postfix(), [A, B], "emu")
        want = oracle.round_to(odt, ref.reshape(-1, order="F")).reshape(ref.shape, order="F") if odt != "f64" else ref
        assert np.array_equal(values(Y, odt), want), (tree.postfix(), idt, odt)


@pytest.mark.parametrize("dt", ["i32", "u32"])
def test_conversion_of_special_values(dt):
    v = np.array([2.5, -2.5, -0.7, 0.7, -0.0, 1e10, -1e10, 2147483647.4, 2147483647.6, -2147483648.9, 4294967295.9,
                  4294967296.0, -1.5, np.inf, -np.inf, np.nan, 123456789.99])
    V = synth.Mat(np.asfortranarray(v.reshape(-1, 1)), "f64")
    for tree, odt in ((X, dt), (conv(X, dt), "f64"), (conv(X * 1.0, dt) + 0.5, "f64")):
        Y = out(v.size, 1, odt)
        coot.eval(tree, [dev(V)], operand(Y, odt))
        torch.cuda.synchronize()
        ref = oracle.evaluate(tree.postfix(), [V], "emu")[:, 0]
        want = oracle.round_to(odt, ref) if odt != "f64" else ref
        assert np.array_equal(values(Y, odt).ravel(), want), (tree.postfix(), odt)
    # f32 data converts the same way (through FP64)
    F = synth.Mat(np.asfortranarray(v.astype(np.float32).reshape(-1, 1)), "f32")
    Y = out(v.size, 1, dt)
    coot.eval(X, [dev(F)], operand(Y, dt))
    torch.cuda.synchronize()
    want = oracle.round_to(dt, v.astype(np.float32).astype(np.float64))
    assert np.array_equal(values(Y, dt).ravel(), want)


def test_integer_reductions(g):
    n = (1 << 20) + 7
    A = imat(g, (n, 1), "i32", -2 ** 31, 2 ** 31)
    tA = to_dev(A)
    dA = operand(tA, "i32")
    s = coot.reduce("accu", X, [dA]).item()
    assert s == float(A.data.astype(np.int64).sum())
    assert coot.reduce("index_max", X, [dA]).item() == int(np.argmax(A.data))
    assert coot.reduce("min", X, [dA]).item() == float(A.data.min())
    M = imat(g, (513, 300), "u32", 0, 2 ** 32)
    tM = to_dev(M)
    dM = operand(tM, "u32")
    for dim in (0, 1):
        got = coot.reduce("sum", X, [dM], dim=dim).cpu().numpy()
        assert np.array_equal(got, M.data.astype(np.float64).sum(axis=dim)), dim   # exact: sums < 2^53
        got = coot.reduce("max", X, [dM], dim=dim).cpu().numpy()
        assert np.array_equal(got, M.data.astype(np.float64).max(axis=dim)), dim


def test_transposed_integer_reads_and_generators(g):
    A = imat(g, (300, 700), "i32", -1000, 1000)
    B = synth.Mat(np.asfortranarray(g.uniform(-1, 1, (700, 300))), "f64")
    Y = out(700, 300, "i32")
    tree = trans(x) * 3.0 + y
    tA, tB = to_dev(A), dev(B)
    coot.eval(tree, [operand(tA, "i32"), tB], operand(Y, "i32"))
    torch.cuda.synchronize()
    ref = oracle.evaluate(tree.postfix(), [A, B], "emu")
    want = oracle.round_to("i32", ref.reshape(-1, order="F")).reshape(ref.shape, order="F")
    assert np.array_equal(values(Y, "i32"), want)
    # an integer generator: fill(2.7) stored as I32 is 2
    Y = out(700, 300, "f64")
    coot.eval(x + y, [dev(B), coot.fill(700, 300, 2.7, "i32")], Y)
    torch.cuda.synchronize()
    assert np.array_equal(Y.cpu().numpy(), B.data + 2.0)


@pytest.mark.parametrize("idt", ["i32", "u32"])
@pytest.mark.parametrize("i0", [4, 1])
def test_integer_views_on_tall_tiles(g, idt, i0):
    """An integer view (3000 x 45 of a 3012 x 48 matrix, 4 rows in: 4-row
    accesses; one row in: single elements) read by tall tiles: element-wise
    results bit-exact against the oracle, the count of a predicate and the
    index of the maximum exact."""
    lo, hi = (-2 ** 31, 2 ** 31) if idt == "i32" else (0, 2 ** 32)
    R0, C0, r, c, j0 = 3012, 48, 3000, 45, 2
    M = imat(g, (R0, C0), idt, lo, hi)
    dM = to_dev(M)
    V = operand(dM, idt)
    V.ptr += (i0 + j0 * R0) * 4
    V.n_rows, V.n_cols = r, c
    sub = synth.Mat(np.asfortranarray(M.data[i0:i0 + r, j0:j0 + c]), idt)
    B = synth.Mat(np.asfortranarray(g.uniform(-3e9, 3e9, (r, c))), "f64")
    dB = dev(B)
    tree = x * 0.5 + y
    Y = out(r, c, "f64")
    src = coot.kernel_source(None, -1, tree, [V, dB], operand(Y, "f64"))
    assert "tall tile" in src
    coot.eval(tree, [V, dB], operand(Y, "f64"))
    torch.cuda.synchronize()
    assert np.array_equal(values(Y, "f64"), oracle.evaluate(tree.postfix(), [sub, B], "emu"))
    vals = sub.data.astype(np.float64)
    thr = float(np.median(vals))
    cnt = coot.reduce("count", X > thr, [V]).cpu().numpy()
    assert int(cnt[0]) == int((vals > thr).sum())
    im = int(coot.reduce("index_max", X, [V]).cpu().numpy()[0])
    assert im == int(np.argmax(vals.reshape(-1, order="F")))
