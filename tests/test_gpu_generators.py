"""GPU parity of generator operands (Table 1 fill / ones / zeros / eye, Table 4
eye / ones / zeros / linspace) and submatrix views (Table 1 .row, .col, .rows,
.cols, .submat, .diag; Table 5 trace; Table 6 diagvec) against the CPU oracle.

Generators hold no memory: the kernel forms each value from the element's
index.  Element-wise trees with generators are bit-exact against the
oracle's per-node rounded evaluation on the dense generator; reductions follow
the usual gates.  Views are strided operands of device buffers: reads match
the oracle on the numpy slice bit for bit, and writes through a view change
exactly the viewed elements."""
import numpy as np
import pytest

import oracle
import synth
from synth import leaf, leaves, trans

from gpu_util import U_FP32, U_FP64, dev, empty, host, need_gpu, same, sum_gate, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

X = leaf(0)
x, y = leaves(2)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


@pytest.fixture(scope="module")
def g():
    return np.random.default_rng(8181)


def mat(g, shape, dt, lo=-1.0, hi=1.0):
    return synth.Mat(synth.store(np.asfortranarray(g.uniform(lo, hi, shape)), dt), dt)


def run(tree, gpu_ops, shape, odt):
    Y = empty(shape[0], shape[1], odt)
    coot.eval(tree, gpu_ops, Y)
    torch.cuda.synchronize()
    return host(Y)


ODT = {"f32": "f32", "f64": "f64", "f16": "f32", "bf16": "f32"}


@pytest.mark.parametrize("dt", ["f32", "f64", "f16", "bf16"])
@pytest.mark.parametrize("shape", [(333, 77), (77, 333), (1, 1000), (1000, 1), (2, 5000), (5000, 3), (64, 64)])
def test_eye_and_fill_bit_exact(g, dt, shape):
    r, c = shape
    A = mat(g, shape, dt)
    for tree, gpu_gen, cpu_gen in ((x + y, coot.eye(r, c, dt), oracle.eye(r, c, dt)),
                                   (x % y - y, coot.fill(r, c, 0.1, dt), oracle.fill(r, c, 0.1, dt)),
                                   (y * 3.0 + x, coot.ones(r, c, dt), oracle.fill(r, c, 1.0, dt)),
                                   (x + y, coot.zeros(r, c, dt), oracle.fill(r, c, 0.0, dt))):
        got = run(tree, [dev(A), gpu_gen], shape, ODT[dt])
        assert same(got, oracle.evaluate(tree.postfix(), [A, cpu_gen], "emu")), (tree.postfix(), shape)


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
def test_transposed_generators(g, dt):
    A = mat(g, (300, 700), dt)
    for gpu_gen, cpu_gen in ((coot.eye(700, 300, dt), oracle.eye(700, 300, dt)),
                             (coot.fill(700, 300, -2.25, dt), oracle.fill(700, 300, -2.25, dt))):
        tree = trans(y) * 2.0 + x
        got = run(tree, [dev(A), gpu_gen], (300, 700), ODT[dt])
        assert same(got, oracle.evaluate(tree.postfix(), [A, cpu_gen], "emu"))
    v = mat(g, (1, 999), dt)
    tree = trans(x) + y
    got = run(tree, [dev(v), coot.linspace(-3.0, 5.0, 999, dt)], (999, 1), ODT[dt])
    assert same(got, oracle.evaluate(tree.postfix(), [v, oracle.linspace(-3.0, 5.0, 999, dt)], "emu"))


@pytest.mark.parametrize("dt", ["f32", "f64", "f16", "bf16"])
@pytest.mark.parametrize("n", [1, 2, 3, 1000, (1 << 20) + 3])
def test_linspace_bit_exact(g, dt, n):
    V = mat(g, (n, 1), dt)
    a, b = -1.5, 2.0 + 1.0 / 3.0
    for tree in (x * 0.5 + y, leaf(1) * 1.0):
        got = run(tree, [dev(V), coot.linspace(a, b, n, dt)], (n, 1), ODT[dt])
        assert same(got, oracle.evaluate(tree.postfix(), [V, oracle.linspace(a, b, n, dt)], "emu")), (n, dt)
    # a row vector (1 x n) through a strided operand takes the tiled kernel
    W = mat(g, (1, n), dt)
    got = run(x - y, [dev(W, ld=3), coot.linspace(a, b, n, dt, row=True)], (1, n), ODT[dt])
    assert same(got, oracle.evaluate((x - y).postfix(), [W, oracle.linspace(a, b, n, dt, row=True)], "emu"))


def test_generator_only_trees():
    """A tree of generators alone reads no memory."""
    got = run(leaf(0) + 0.0, [coot.eye(5, 7, "f32")], (5, 7), "f32")
    assert np.array_equal(got, np.eye(5, 7))
    got = run(leaf(0) + leaf(1), [coot.linspace(0.0, 1.0, 5, "f64"), coot.fill(5, 1, 1.0, "f64")], (5, 1), "f64")
    assert np.array_equal(got[:, 0], [1.0, 1.25, 1.5, 1.75, 2.0])
    n = 1000
    s = coot.reduce("accu", X, [coot.linspace(1.0, float(n), n, "f64")]).item()
    assert s == n * (n + 1) / 2
    assert coot.reduce("count", X, [coot.eye(300, 200, "f32")]).item() == 200
    assert coot.reduce("count", X, [coot.eye(300, 200, "f32")], dim=0).cpu().tolist() == [1] * 200
    assert coot.reduce("max", X, [coot.linspace(-2.0, 7.0, 10, "f32")]).item() == 7.0
    assert coot.reduce("index_max", X, [coot.linspace(-2.0, 7.0, 10, "f32")]).item() == 9
    assert coot.reduce("index_min", X, [coot.fill(50, 1, 3.0, "f32")]).item() == 0


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_reductions_of_trees_with_generators(g, dt):
    A = mat(g, (513, 300), dt)
    f64 = dt == "f64"
    tol = 1e-13 if f64 else 1e-6
    E, Eo = coot.eye(513, 300, dt), oracle.eye(513, 300, dt)
    for op, tree, dims in (("accu", x % y, (-1,)), ("sum", x + y, (-1, 0, 1)), ("max", x - y, (0, 1)),
                           ("index_max", x + y * 2.0, (-1, 0, 1)), ("mean", x + y, (0, 1))):
        for dim in dims:
            got = coot.reduce(op, tree, [dev(A), E], dim=dim)
            torch.cuda.synchronize()
            got = got.cpu().numpy().astype(np.float64).ravel()
            o, oi, asum = oracle.reduce(op, tree.postfix(), [A, Eo], dim=dim)
            if op.startswith("index"):
                assert np.array_equal(got.astype(np.int64), oi), (op, dim)
            elif op == "max":
                assert same(got, o), (op, dim)
            else:
                r_, c_ = 513, 300
                n = r_ * c_ if dim < 0 else (r_ if dim == 0 else c_)
                sum_gate(got, o, asum, n, tol, u=U_FP64 if f64 else U_FP32, what=f"{op} dim {dim}")
    # accu(A % eye) is the trace
    t = coot.reduce("accu", x % y, [dev(A), E]).item()
    assert abs(t - np.trace(host(dev(A)))) <= tol * np.sum(np.abs(np.diagonal(host(dev(A)))))
    # dot with a linspace of the flat kernel (a ragged tail)
    n = (1 << 20) + 5
    V = mat(g, (n, 1), dt)
    got = coot.reduce("dot", x % y, [dev(V), coot.linspace(-1.0, 1.0, n, dt)]).item()
    o, _, asum = oracle.reduce("dot", (x % y).postfix(), [V, oracle.linspace(-1.0, 1.0, n, dt)])
    sum_gate(got, o, asum, n, tol, u=U_FP64 if f64 else U_FP32, what="dot with linspace")


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
def test_submatrix_views_read_and_write(g, dt):
    Mm = mat(g, (200, 150), dt)
    M = dev(Mm)
    Mh = host(M)
    odt = ODT[dt]
    cases = ((coot.submat(M, 10, 20, 109, 79), (slice(10, 110), slice(20, 80))),
             (coot.rows(M, 5, 6), (slice(5, 7), slice(0, 150))),
             (coot.cols(M, 140, 149), (slice(0, 200), slice(140, 150))),
             (coot.row(M, 17), (slice(17, 18), slice(0, 150))),
             (coot.col(M, 3), (slice(0, 200), slice(3, 4))))
    for view, (rs, cs) in cases:
        sub = Mh[rs, cs]
        ref = synth.Mat(np.asfortranarray(Mm.data[rs, cs]), dt)
        got = run(X * 2.0 - 1.0 / 3.0, [view], sub.shape, odt)
        assert same(got, oracle.evaluate((X * 2.0 - 1.0 / 3.0).postfix(), [ref], "emu"))
        s = coot.reduce("sum", X, [view], dim=0).cpu().numpy().astype(np.float64)
        assert np.allclose(s, sub.sum(axis=0), rtol=1e-6, atol=1e-6)
    # writes through a view touch exactly the viewed elements
    Y = dev(synth.Mat(np.asfortranarray(np.zeros((200, 150))), "f64"))
    S = mat(g, (100, 60), "f64")
    coot.eval(X - 0.5, [dev(S)], coot.submat(Y, 10, 20, 109, 79))
    torch.cuda.synchronize()
    Yh = host(Y)
    assert np.array_equal(Yh[10:110, 20:80], S.data - 0.5)
    Yh[10:110, 20:80] = 0.0
    assert not np.any(Yh)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_diag_trace_diagvec(g, dt):
    for shape in ((300, 300), (257, 400), (400, 129)):
        Am = mat(g, shape, dt)
        A = dev(Am)
        Ah = host(A)
        for k in (0, 5, -7):
            d = np.diagonal(Ah, k)
            col = empty(d.size, 1, dt)
            coot.diagvec(A, col, k)
            torch.cuda.synchronize()
            assert np.array_equal(host(col)[:, 0], d), (shape, k)
            m = coot.reduce("max", X, [coot.diag(A, k)]).item()
            assert m == d.max()
        t = coot.trace(A).item()
        o, _, asum = oracle.reduce("accu", X.postfix(), [synth.Mat(np.asfortranarray(np.diagonal(Ah).reshape(1, -1)), "f64")])
        sum_gate(t, o, asum, np.diagonal(Ah).size, 1e-13 if dt == "f64" else 1e-6,
                 u=U_FP64 if dt == "f64" else U_FP32, what=f"trace {shape}")
    # in place through the diagonal: A.diag() += 1
    Am = mat(g, (50, 50), dt)
    A = dev(Am)
    before = host(A)
    D = coot.diag(A)
    coot.eval(X + 1.0, [D], D)
    torch.cuda.synchronize()
    after = host(A)
    want = np.diagonal(before) + 1.0            # exact in FP64, rounded once to the element type
    assert np.array_equal(np.diagonal(after), want.astype(np.float32) if dt == "f32" else want)
    off = ~np.eye(50, dtype=bool)
    assert np.array_equal(after[off], before[off])


def test_unfused_generators_match_fused(g):
    A = mat(g, (400, 300), "f32")
    tree = (x + y) % y - 0.25
    Y1, Y2 = empty(400, 300), empty(400, 300)
    coot.eval(tree, [dev(A), coot.eye(400, 300)], Y1)
    coot.eval(tree, [dev(A), coot.eye(400, 300)], Y2, unfused=True)
    torch.cuda.synchronize()
    assert same(host(Y1), host(Y2))
