"""GPU parity of the thin-value kernels (a short side of at most 16 elements,
operands moved as whole vectors and transposed in registers) against the CPU
oracle.

Every short side 2..16 in both orientations, long sides ragged against the
vector width, 64- and 16-bit storage, element-wise trees bit-exact against the
oracle's per-node rounded evaluation (EMU), sums within the sum gate, extrema
and their linear indices bit-exact (ties planted), in-place updates, an
index-dependent generator, and views that do not fit whole vectors (which
take the shape-adaptive tiles instead).  Each case first asks the library
for its kernel text and checks that the intended kernel is the one launched.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import abs_, conv, leaf, leaves, trans

from gpu_util import U_FP32, U_FP64, dev, empty, host, mismatch_report, need_gpu, same, sum_gate, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

x, y = leaves(2)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


def mat(g, shape, dt, lo=-2.0, hi=2.0):
    return synth.Mat(synth.store(np.asfortranarray(g.uniform(lo, hi, shape)), dt), dt)


def is_thin(red, tree, ops, out, dim=-1):
    return "// thin value:" in coot.kernel_source(red, dim, tree, ops, out)


def eval_checked(tree, mats, ops, out_dt, expect_thin=True, out=None):
    r, c, _ = oracle.shape(tree.postfix(), mats)
    Y = out if out is not None else empty(r, c, out_dt)
    assert is_thin(None, tree, ops, Y) == expect_thin, (r, c, out_dt)
    coot.eval(tree, ops, Y)
    torch.cuda.synchronize()
    em = oracle.evaluate(tree.postfix(), mats, "emu")
    if out_dt != "f64":
        em = oracle.round_to(out_dt, em.reshape(-1, order="F")).reshape(em.shape, order="F")
    got = host(Y)
    assert same(got, em), (r, c, out_dt, mismatch_report(got, em))


LONG = [4 * 37 + 3, 4 * 64]   # a ragged and a whole number of 4-element groups


# (a short side of 1 is a vector: read transposed, a contiguous vector is the
# same linear order, so those trees take the flat kernels)
@pytest.mark.parametrize("k", list(range(2, 17)))
def test_every_short_side_both_orientations(k):
    g = np.random.default_rng(1600 + k)
    t = trans(x) % y - 2.5
    for ln in LONG:
        for r, c in ((k, ln), (ln, k)):
            A, B = mat(g, (c, r), "f32"), mat(g, (r, c), "f32")
            ops = [dev(A), dev(B)]
            # two reads and an output: 8/K groups x K vectors x 3 fit the
            # register budget up to K = 13
            eval_checked(t, [A, B], ops, "f32", expect_thin=k <= 13)
            assert is_thin("accu", t % t, ops, empty(1, 1, "f32"))
            got = coot.reduce("accu", t % t, ops).double().cpu().numpy()
            o, _, asum = oracle.reduce("accu", (t % t).postfix(), [A, B], mode="emu")
            sum_gate(got, o, asum, r * c, 1e-6, u=U_FP32, what="accu")


@pytest.mark.parametrize("dt", ["f64", "f16", "bf16"])
def test_storage_types(dt):
    g = np.random.default_rng(77)
    for r, c in ((2, 8 * 50 + 5), (8 * 50 + 5, 3), (12, 8 * 40), (8 * 40 + 1, 13)):
        # strided reads need leading dimensions that are whole vectors
        vec = 16 // {"f64": 8, "f16": 2, "bf16": 2}[dt]
        A, B = mat(g, (c, r), dt), mat(g, (r, c), dt)
        ldA = c + (-c) % vec
        ldB = r + (-r) % vec
        short_rows = r <= c
        dA = dev(A, ld=ldA if short_rows else c)
        dB = dev(B, ld=r if short_rows else ldB)
        t = trans(x) + y % y
        out_dt = dt
        O = empty(r, c, out_dt) if short_rows else empty(r, c, out_dt, ld=ldB)
        eval_checked(t, [A, B], [dA, dB], out_dt, expect_thin=True, out=O)
        # a sum over the same tree
        red_out = empty(1, 1, "f64" if dt == "f64" else "f32")
        assert is_thin("accu", t, [dA, dB], red_out)
        got = coot.reduce("accu", t, [dA, dB]).double().cpu().numpy()
        o, _, asum = oracle.reduce("accu", t.postfix(), [A, B], mode="emu")
        prec = 64 if dt == "f64" else 32
        sum_gate(got, o, asum, r * c, 1e-13 if prec == 64 else 1e-6, u=U_FP64 if prec == 64 else U_FP32, what=dt)


@pytest.mark.parametrize("r,c", [(3, 4 * 300 + 2), (4 * 300 + 2, 5), (16, 4 * 64 + 1)])
def test_extrema_and_indices_with_ties(r, c):
    """The largest value planted at several positions: the lowest linear index
    of the value wins, whatever thread or group holds it."""
    g = np.random.default_rng(5)
    A, B = mat(g, (c, r), "f32"), mat(g, (r, c), "f32")
    t = trans(x) + 0.5 * y
    flat = np.random.default_rng(9).choice(r * c, 6, replace=False)
    for p in flat:
        i, j = p % r, p // r
        A.data[j, i] = 6.0
        B.data[i, j] = 4.0   # value 6 + 0.5 * 4 = 8, above every other (|value| <= 3)
    ops = [dev(A), dev(B)]
    for op in ("index_max", "index_min", "max", "min"):
        odt = "u64" if op.startswith("index") else "f32"
        assert "// thin value:" in coot.kernel_source(op, -1, t, ops, coot.fake_operand(1, 1, odt))
        got = coot.reduce(op, t, ops).cpu().numpy()
        v, i, _ = oracle.reduce(op, t.postfix(), [A, B], mode="emu")
        if op.startswith("index"):
            assert int(got[0]) == int(i[0]), (op, got, i)
        else:
            assert same(got.astype(np.float64), v), (op, got, v)
    assert int(coot.reduce("index_max", t, ops).cpu().numpy()[0]) == int(np.min(flat))


def test_in_place_and_dot_and_statistics():
    g = np.random.default_rng(11)
    r, c = 6, 4 * 500 + 3
    A, B = mat(g, (c, r), "f32"), mat(g, (r, c), "f32")
    dA, dB = dev(A), dev(B)
    # B = trans(A) + 2 * B, the output being the straight operand itself
    t = trans(x) + 2.0 * y
    em = oracle.evaluate(t.postfix(), [A, B], "emu")
    assert is_thin(None, t, [dA, dB], dB)
    coot.eval(t, [dA, dB], dB)
    torch.cuda.synchronize()
    assert same(host(dB), em), mismatch_report(host(dB), em)
    # dot(trans(A), B') in product form, var and count over the thin value
    Bm = synth.Mat(np.asfortranarray(em.astype(np.float32)), "f32")
    for op, tree, tol in (("dot", trans(x) % y, 1e-6), ("var", trans(x) - y, 1e-6), ("count", trans(x) > y, 0.0)):
        got = coot.reduce(op, tree, [dA, dB]).double().cpu().numpy()
        o, _, asum = oracle.reduce(op, tree.postfix(), [A, Bm], mode="emu")
        if op == "count":
            assert got[0] == o[0]
        elif op == "var":
            assert abs(got[0] - o[0]) <= tol * abs(o[0])
        else:
            sum_gate(got, o, asum, r * c, tol, u=U_FP32, what=op)


def test_index_generator_and_conversions():
    """eye (needs each element's row and column) inside a thin tree, and a
    conversion node between storage precisions."""
    g = np.random.default_rng(13)
    r, c = 4, 4 * 200 + 1
    A, B = mat(g, (c, r), "f32"), mat(g, (r, c), "f64")
    E = oracle.eye(r, c, "f32")
    t = trans(leaf(0)) % leaf(2) + conv(leaf(1), "f32")
    ops = [dev(A), dev(B), coot.eye(r, c, "f32")]
    eval_checked(t, [A, B, E], ops, "f32", expect_thin=True)


def test_views_and_misaligned_operands():
    """Strided operands with any leading dimension and misaligned bases move
    element by element inside the thin kernel; a packed operand with padding
    (ld != K) cannot follow the thin layout and takes the shape-adaptive
    tiles.  Every case is exact."""
    g = np.random.default_rng(17)
    r, c = 3, 4 * 100 + 1
    A, B = mat(g, (c, r), "f32"), mat(g, (r, c), "f32")
    t = trans(x) - 0.25 * y
    for ldA, ldB, off in ((c, r, 0), (c + 3, r, 0), (c + 3, r + 1, 0), (c + (-c) % 4, r, 1), (c, r, 2)):
        dA, dB = dev(A, ld=ldA, offset=off), dev(B, ld=ldB)
        O = empty(r, c, "f32", offset=off)
        eval_checked(t, [A, B], [dA, dB], "f32", expect_thin=ldB == r, out=O)
        if ldB == r:
            # read 0 (A, strided): whole vectors when its base and ld are;
            # read 1 (B, packed) always; the output when its base is
            mask = (1 if ldA % 4 == 0 and off == 0 else 0) | 2 | ((1 << 31) if off == 0 else 0)
            assert f"(mask {mask}" in coot.kernel_source(None, -1, t, [dA, dB], O)
