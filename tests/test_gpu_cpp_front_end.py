"""GPU parity of the C++ expression-template front end (include/coot.hpp, the
paper's Section 7 interface): the cases in tests/cpp/front_end_cases.cpp run
front-end expressions on device memory owned here, and the results are
compared with the CPU oracle (same gates as the binding's tests) and, for the
small workload, with the Python binding's own call of the same tree (the same
fused kernel: identical bits)."""
import ctypes as C
import os

import numpy as np
import pytest

import oracle
import synth

from gpu_util import dev, empty, host, need_gpu, same, sum_gate, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FE = os.path.join(ROOT, "tests", "cpp", "libcoot_front_end_cases.so")
vp, i64, dbl = C.c_void_p, C.c_int64, C.c_double


@pytest.fixture(scope="module")
def fe():
    need_gpu()
    coot.init(0)
    coot.lib()
    assert os.path.exists(FE), "tests/cpp/libcoot_front_end_cases.so is missing: run __graft_entry__.build()"
    L = C.CDLL(FE)
    L.fe_last_error.restype = C.c_char_p
    sig = {"fe_small": [vp] * 5 + [i64, i64, vp, vp, vp, vp], "fe_in_place": [vp, vp, i64, vp],
           "fe_views": [vp, i64, i64, i64, vp, i64, vp, vp], "fe_generators": [vp, i64, i64, vp, i64, dbl, dbl, vp, vp],
           "fe_scalars": [vp, vp, i64, vp, vp], "fe_convert": [vp, vp, i64, i64, vp, vp, vp],
           "fe_owned": [vp, i64, i64, vp, vp], "fe_shape_error": [vp, vp, vp],
           "fe_integers": [vp, vp, i64, vp, vp, vp, vp, vp]}
    for name, args in sig.items():
        getattr(L, name).argtypes = args
    return L


def stream():
    return torch.cuda.current_stream().cuda_stream


def ptr(t):
    return t.data_ptr()


def run(L, name, *args):
    rc = getattr(L, name)(*args, stream())
    assert rc == 0, L.fe_last_error().decode()


@pytest.fixture(scope="module")
def g():
    return np.random.default_rng(9292)


def test_small_workload(fe):
    mats = synth.cfg1_inputs(67, 45)
    names = "ABCD"
    D = [dev(mats[k]) for k in names]
    Y = empty(67, 45)
    colsum = torch.empty(45, device="cuda")
    s = torch.empty(1, device="cuda")
    idx = torch.empty(1, dtype=torch.int64, device="cuda")
    run(fe, "fe_small", *[ptr(t) for t in D], ptr(Y), 67, 45, ptr(colsum), ptr(s), ptr(idx))
    trees = synth.cfg1_trees()
    ops = [mats[k] for k in names]
    # the binding's call of the same tree runs the same fused kernel
    Y2 = empty(67, 45)
    coot.eval(trees["Y"], D, Y2)
    torch.cuda.synchronize()
    assert same(host(Y), host(Y2))
    ex, S = oracle.evaluate(trees["Y"].postfix(), ops, "exact", scale=True)
    assert np.max(np.abs(host(Y) - ex) / np.maximum(S, 1e-300)) <= 1e-6
    o, _, _ = oracle.reduce("accu", trees["accu_AB"].postfix(), ops)
    assert abs(s.item() - o[0]) <= 1e-6 * abs(o[0])
    oc, _, asum = oracle.reduce("sum", synth.leaf(0).postfix(), [mats["A"]], dim=0)
    sum_gate(colsum.double().cpu().numpy(), oc, asum, 67, 1e-6, what="sum(A, 0)")
    _, oi, _ = oracle.reduce("index_max", trees["absB"].postfix(), ops, mode="emu")
    assert idx.item() == oi[0]


def test_in_place_updates(fe, g):
    n = 300
    A = g.uniform(-1, 1, (n, n)).astype(np.float32)
    B = g.uniform(-1, 1, (n, n)).astype(np.float32)
    Am, Bm = synth.Mat(np.asfortranarray(A), "f32"), synth.Mat(np.asfortranarray(B), "f32")
    dA, dB = dev(Am), dev(Bm)
    run(fe, "fe_in_place", ptr(dA), ptr(dB), n)
    # the statements one after the other, each evaluated by the oracle on the
    # values the previous one stored: a = trans(a) + 1; b += a; b %= a;
    # b *= 0.5; b -= 1
    x, y = synth.leaves(2)
    st = lambda v: synth.Mat(np.asfortranarray(v.astype(np.float32)), "f32")
    a = oracle.evaluate((synth.trans(x) + 1.0).postfix(), [Am], "emu")
    b = oracle.evaluate((y + x).postfix(), [st(a), Bm], "emu")
    b = oracle.evaluate((y % x).postfix(), [st(a), st(b)], "emu")
    b = oracle.evaluate((y * 0.5).postfix(), [st(a), st(b)], "emu")
    b = oracle.evaluate((y - 1.0).postfix(), [st(a), st(b)], "emu")
    assert np.array_equal(host(dA), a)
    assert np.array_equal(host(dB), b)


@pytest.mark.parametrize("k", [0, 4, -3])
def test_views(fe, g, k):
    r, c = 50, 40
    A = g.uniform(-1, 1, (r, c))
    dA = dev(synth.Mat(np.asfortranarray(A), "f64"))
    nd = np.diagonal(A, k).size
    dv = torch.empty(nd, dtype=torch.float64, device="cuda")
    t = torch.empty(1, dtype=torch.float64, device="cuda")
    run(fe, "fe_views", ptr(dA), r, c, k, ptr(dv), nd, ptr(t))
    W = A.copy()
    W[np.arange(min(r, c)), np.arange(min(r, c))] += 1.0
    W[1:4, 1:4] = 2.0 * W[0:3, 0:3].copy()        # the right side is read before the write
    W[r - 1, :] = W[0, :] - W[1, :]
    W[:, c - 1] = 7.0
    got = host(dA)
    assert np.array_equal(got, W)
    assert np.array_equal(dv.cpu().numpy(), np.diagonal(W, k))
    d = np.diagonal(W)
    assert abs(t.item() - np.trace(W)) <= 1e-13 * np.sum(np.abs(d))


def test_generators(fe):
    r, c, n = 37, 29, 1001
    Y = empty(r, c)
    L = torch.empty(n, dtype=torch.float64, device="cuda")
    H = np.empty((c, r), np.float32)                  # host, column-major r x c
    run(fe, "fe_generators", ptr(Y), r, c, ptr(L), n, -1.25, 3.5, H.ctypes.data)
    # y = 3 * eye(r, c) + ones(r, c) + trans(eye(c, r)), generators as the oracle's dense operands
    a, b, e = synth.leaves(3)
    want = oracle.evaluate((3.0 * a + b + synth.trans(e)).postfix(),
                           [oracle.eye(r, c, "f32"), oracle.fill(r, c, 1.0, "f32"), oracle.eye(c, r, "f32")], "emu")
    assert np.array_equal(host(Y), want)
    lw = oracle.evaluate(synth.leaf(0).postfix(), [oracle.linspace(-1.25, 3.5, n, "f64")], "emu")
    assert np.array_equal(L.cpu().numpy(), lw[:, 0])
    ew = oracle.evaluate(synth.leaf(0).postfix(), [oracle.eye(r, c, "f32")], "emu")
    assert np.array_equal(H.T.astype(np.float64), ew)


def test_scalar_functions(fe, g):
    n = 100003
    x = g.uniform(-2, 2, n)
    y = g.uniform(-2, 2, n)
    res = torch.empty(14, dtype=torch.float64)        # host
    dx, dy = dev(x), dev(y)
    run(fe, "fe_scalars", ptr(dx), ptr(dy), n, res.data_ptr())
    r = res.numpy()
    X, Y = synth.Mat(np.asfortranarray(x.reshape(-1, 1)), "f64"), synth.Mat(np.asfortranarray(y.reshape(-1, 1)), "f64")
    a, b = synth.leaves(2)

    def close(v, op, tree, ops, tol=1e-13):
        o, _, s = oracle.reduce(op, tree.postfix(), ops)
        assert abs(v - o[0]) <= tol * max(abs(o[0]), s[0]), (op, v, o[0])

    close(r[0], "dot", a % b, [X, Y])
    close(r[1], "norm2", a, [X])
    close(r[2], "norm1", a, [X])
    assert r[3] == np.max(np.abs(x)) and r[4] == np.min(np.abs(x))
    assert r[5] == x.max() and r[6] == np.min(x * y)
    assert r[7] == np.argmin(x) and r[8] == np.argmax(x - y)
    close(r[9], "mean", a, [X])
    assert abs(r[10] - np.var(x, ddof=1)) <= 1e-12 * np.var(x, ddof=1)
    assert r[11] == np.count_nonzero(x > 0.3)
    assert r[12] == 1.0 and r[13] == 0.0


def test_fused_conversion_and_dim_statistics(fe, g):
    r, c = 300, 77
    X = g.uniform(-1, 1, (r, c))
    dX = dev(synth.Mat(np.asfortranarray(X), "f64"))
    F = empty(r, c)
    cm = torch.empty(c, device="cuda")
    rv = torch.empty(r, device="cuda")
    run(fe, "fe_convert", ptr(dX), ptr(F), r, c, ptr(cm), ptr(rv))
    f = (2.0 * X + 1.0).astype(np.float32)            # one rounding, after the FP64 arithmetic
    assert np.array_equal(host(F), f.astype(np.float64))
    Fm = synth.Mat(np.asfortranarray(f), "f32")
    om, _, sm = oracle.reduce("mean", synth.leaf(0).postfix(), [Fm], dim=0)
    sum_gate(cm.double().cpu().numpy(), om, sm, r, 1e-6, what="mean(F, 0)")
    ov, _, _ = oracle.reduce("var", synth.leaf(0).postfix(), [Fm], dim=1)
    assert np.all(np.abs(rv.double().cpu().numpy() - ov) <= 2e-7 * np.abs(ov))


def test_owned_matrices(fe, g):
    r, c = 23, 31
    A = g.uniform(-1, 1, (r, c)).astype(np.float32)
    Hin = np.asfortranarray(A)
    H = np.empty((c, r), np.float32)
    run(fe, "fe_owned", Hin.ctypes.data, r, c, H.ctypes.data)
    b = A * np.float32(2.0) + np.float32(1.0)
    want = b * A - A
    assert np.array_equal(H.T, want)


def test_errors_become_exceptions(fe):
    A = torch.zeros(20, device="cuda")
    B = torch.zeros(20, device="cuda")
    rc = fe.fe_shape_error(ptr(A), ptr(B), stream())
    assert rc == -1
    assert "shape" in fe.fe_last_error().decode()


def test_integer_vectors(fe, g):
    """imat / ivec through the front end (Section 7's conv_to of an integer
    expression, fused): integers widen exactly to FP64, stores truncate and
    clamp."""
    n = 100001
    a = g.integers(-2 ** 20, 2 ** 20, n).astype(np.int32)
    b = g.integers(-2 ** 10, 2 ** 10, n).astype(np.int32)
    b[b == 0] = 3
    dA = torch.from_numpy(a).cuda()
    dB = torch.from_numpy(b).cuda()
    F = torch.empty(n, device="cuda")
    Q = torch.empty(n, dtype=torch.int32, device="cuda")
    U = torch.empty(n, dtype=torch.int32, device="cuda")          # u32 bits
    s = torch.empty(2, dtype=torch.float64)
    run(fe, "fe_integers", ptr(dA), ptr(dB), n, ptr(F), ptr(Q), ptr(U), s.data_ptr())
    a64, b64 = a.astype(np.int64), b.astype(np.int64)
    assert np.array_equal(F.cpu().numpy(), (2 * a64 + b64).astype(np.float32))
    q = np.trunc(a64 / b64).astype(np.int64)                    # exact: |a| < 2^21
    assert np.array_equal(Q.cpu().numpy().astype(np.int64), q)
    assert np.array_equal(U.cpu().numpy().view(np.uint32).astype(np.int64), np.maximum(a64 - b64, 0))
    assert s[0].item() == float(a64.sum())
    assert s[1].item() == float((a64 * b64).max())
