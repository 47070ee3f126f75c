"""Tiled kernels on views that start inside a 128-byte line.  Trees that read
an operand transposed use 64 x 64 tiles whose grid starts as many rows above
the value as the output's columns start into a line (a launch argument), so
its first and last tile rows are partial; trees with straight reads only use
tall tiles that walk down each column.  Element-wise results must match the
oracle bit for bit, nothing outside the output view may change, and
reductions must keep the plain linear index (row + column * rows) of the
value."""
import numpy as np
import pytest

import oracle
import synth
from synth import leaves, trans

from gpu_util import TORCH_DT, dev, host, need_gpu, same, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

x, y = leaves(2)
R, C, LD = 200, 150, 256          # several tiles with ragged tails; LD keeps one phase per column
ODT = {"f32": "f32", "f64": "f64", "bf16": "f32"}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


def mat(g, shape, dt):
    return synth.Mat(synth.store(np.asfortranarray(g.uniform(-2, 2, shape)), dt), dt)


def out_buffer(dt, off):
    """NaN-filled buffer and an R x C view of it starting `off` elements in."""
    buf = torch.full((C * LD + off + 1,), float("nan"), dtype=TORCH_DT[dt], device="cuda")
    return buf, buf[off:off + C * LD].view(C, LD)[:, :R].t()


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
@pytest.mark.parametrize("offs", [(1, 1), (0, 3), (5, 0), (7, 7), (0, 0)])
def test_elementwise_into_offset_views(dt, offs):
    g = np.random.default_rng(500 + 100 * list(ODT).index(dt) + 10 * offs[0] + offs[1])
    ia, ib, io = offs[0], (offs[0] + 2) % 9, offs[1]
    A, B = mat(g, (R, C), dt), mat(g, (R, C), dt)
    T = mat(g, (C, R), dt)
    dA, dB = dev(A, ld=LD, offset=ia), dev(B, ld=LD, offset=ib)
    dT = dev(T, ld=LD, offset=ia)
    odt = ODT[dt]
    for tree, gops, cops in ((x * 2.0 - y, [dA, dB], [A, B]), (trans(x) + y * 0.5, [dT, dB], [T, B])):
        buf, Y = out_buffer(odt, io)
        coot.eval(tree, gops, Y)
        torch.cuda.synchronize()
        want = oracle.evaluate(tree.postfix(), cops, "emu")
        assert same(host(Y), want), (dt, offs, tree)
        # nothing outside the view was written
        full = buf[io:io + C * LD].view(C, LD)
        assert torch.isnan(full[:, R:]).all() and torch.isnan(buf[:io]).all() and torch.isnan(buf[io + C * LD:]).all()


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
@pytest.mark.parametrize("off", [1, 3, 0])
def test_reductions_over_offset_views(dt, off):
    g = np.random.default_rng(1000 + 10 * list(ODT).index(dt) + off)
    DA = g.uniform(-2, 2, (R, C))                  # draws; 16-bit Mats hold bit patterns
    A, B = synth.Mat(synth.store(np.asfortranarray(DA), dt), dt), mat(g, (R, C), dt)
    dA, dB = dev(A, ld=LD, offset=off), dev(B, ld=LD, offset=off)
    o, _, s = oracle.reduce("accu", (x % y).postfix(), [A, B])
    got = coot.reduce("accu", x % y, [dA, dB]).item()
    tol = 1e-6 if dt != "f64" else 1e-13
    assert abs(got - o[0]) <= tol * s[0]
    # a unique maximum planted at each tile boundary row of the shifted grid and elsewhere
    for (i, j) in ((0, 0), (R - 1, C - 1), (64 - off if off else 63, 70), (128 - off, 1), (17, 149)):
        M = DA.copy()
        M[i, j] = 50.0
        Am = synth.Mat(synth.store(np.asfortranarray(M), dt), dt)
        dM = dev(Am, ld=LD, offset=off)
        assert coot.reduce("index_max", x, [dM]).item() == i + j * R, (dt, off, i, j)
        assert coot.reduce("index_max", x % y, [dM, dB]).item() == \
            oracle.reduce("index_max", (x % y).postfix(), [Am, B], mode="emu")[1][0]


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
def test_tall_tiles_over_long_strided_views(dt):
    """Trees with no transposed read over strided views take tall tiles (up to
    4096 rows of one column): a 4097 x 70 view (a full and a one-row tile per
    column) starting inside a line, written into another offset view; the
    result bit-exact, nothing outside the view written, and extrema planted
    on either side of the 4096-row tile boundary keep their linear index."""
    r, c, ld = 4097, 70, 4101
    g = np.random.default_rng(4097 + list(ODT).index(dt))
    DA = g.uniform(-2, 2, (r, c))
    A = synth.Mat(synth.store(np.asfortranarray(DA), dt), dt)
    B = mat(g, (r, c), dt)
    dA, dB = dev(A, ld=ld, offset=3), dev(B, ld=ld + 2, offset=1)
    odt = ODT[dt]
    buf = torch.full((c * ld + 6,), float("nan"), dtype=TORCH_DT[odt], device="cuda")
    Y = buf[5:5 + c * ld].view(c, ld)[:, :r].t()
    tree = x * 2.0 - y
    coot.eval(tree, [dA, dB], Y)
    torch.cuda.synchronize()
    assert same(host(Y), oracle.evaluate(tree.postfix(), [A, B], "emu")), dt
    full = buf[5:5 + c * ld].view(c, ld)
    assert torch.isnan(full[:, r:]).all() and torch.isnan(buf[:5]).all()
    o, _, s = oracle.reduce("accu", (x % y).postfix(), [A, B])
    got = coot.reduce("accu", x % y, [dA, dB]).item()
    assert abs(got - o[0]) <= (1e-6 if dt != "f64" else 1e-13) * s[0]
    for (i, j) in ((4095, 3), (4096, 3), (0, 69), (4096, 69)):
        M = DA.copy()
        M[i, j] = 50.0
        dM = dev(synth.Mat(synth.store(np.asfortranarray(M), dt), dt), ld=ld, offset=3)
        assert coot.reduce("index_max", x, [dM]).item() == i + j * r, (dt, i, j)


# tall tiles of 4096 elements, 2^lr x 2^lc: several tile rows, so that some
# are whole with the grid shifted by the output's phase, and partial tiles at
# both ends of the columns
V4_SHAPES = [(9000, 19), (1024 * 6 + 5, 21), (256 * 9 + 3, 37), (64 * 20 + 7, 70), (128 * 11, 99)]


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
@pytest.mark.parametrize("r,c", V4_SHAPES)
def test_whole_tall_tiles_four_rows_per_access(dt, r, c):
    """Tall tiles start as many rows above the value as the output's columns
    start into a 128-byte line (else the straight reads' most common phase).
    Whole tiles move 4 consecutive rows per lane and access when every
    operand's columns then start on 4-element boundaries (views 4 rows in, or
    all one row in, leading dimensions multiples of 64), else single elements;
    partial tiles clamp their loads into the value.  A tree with eye (needs
    each element's row and column).  Results bit-exact, nothing outside the
    view written, sums within the gate, extrema planted on both sides of the
    4-row groups and the tile edges keep their index."""
    g = np.random.default_rng(7000 + r + c + list(ODT).index(dt))
    DA = g.uniform(-2, 2, (r, c))
    A = synth.Mat(synth.store(np.asfortranarray(DA), dt), dt)
    B = mat(g, (r, c), dt)
    odt = ODT[dt]
    ld = (r + 12 + 63) // 64 * 64
    # offsets of A, B, Y (elements); 4-row accesses expected for the
    # element-wise call (phase of Y) and the sum (phase of A on a tie)
    for off_a, off_b, off_y, v4_ew, v4_red in ((4, 8, 4, True, True), (4, 9, 4, False, False),
                                               (1, 1, 1, True, True), (1, 5, 2, False, True)):
        dA, dB = dev(A, ld=ld, offset=off_a), dev(B, ld=ld, offset=off_b)
        buf = torch.full((c * ld + off_y + 4,), float("nan"), dtype=TORCH_DT[odt], device="cuda")
        Y = buf[off_y:off_y + c * ld].view(c, ld)[:, :r].t()
        tree = x * 2.0 - y
        src = coot.kernel_source(None, -1, tree, [dA, dB], Y)
        assert ("4 rows per access" in src) == v4_ew and "whole tall tile" in src, (r, c, off_a, off_b)
        coot.eval(tree, [dA, dB], Y)
        torch.cuda.synchronize()
        assert same(host(Y), oracle.evaluate(tree.postfix(), [A, B], "emu")), (dt, r, c, off_a, off_b)
        full = buf[off_y:off_y + c * ld].view(c, ld)
        assert torch.isnan(full[:, r:]).all() and torch.isnan(buf[:off_y]).all()
        assert ("4 rows per access" in coot.kernel_source("accu", -1, x % y, [dA, dB],
                                                           coot.fake_operand(1, 1, "f64" if dt == "f64" else "f32"))) == v4_red
        o, _, s = oracle.reduce("accu", (x % y).postfix(), [A, B])
        got = coot.reduce("accu", x % y, [dA, dB]).item()
        assert abs(got - o[0]) <= (1e-6 if dt != "f64" else 1e-13) * s[0]
    # index reductions over views on one phase: maxima at group and tile
    # edges, a tie resolved to the lower linear index
    dB = dev(B, ld=ld, offset=8)
    for pts in (((3, 0),), ((4, 1),), ((r - 1, c - 1),), ((r - 4, c - 1), (r - 1, c - 2)),
                ((min(r - 1, 4091), 0), (5, c - 1)), ((min(r - 1, 4092), c // 2),)):
        M = DA.copy()
        for (i, j) in pts:
            M[i, j] = 50.0
        Am = synth.Mat(synth.store(np.asfortranarray(M), dt), dt)
        dM = dev(Am, ld=ld, offset=4)
        want = min(i + j * r for (i, j) in pts)
        assert coot.reduce("index_max", x, [dM]).item() == want, (dt, r, c, pts)
        assert coot.reduce("index_max", x % y, [dM, dB]).item() == \
            oracle.reduce("index_max", (x % y).postfix(), [Am, B], mode="emu")[1][0]
    # a generator needing each element's position, with an operand on the
    # output's phase
    E = oracle.eye(r, c, odt)
    t = x * 0.5 + synth.leaf(1)
    dA = dev(A, ld=ld, offset=0)
    Y = torch.empty(c, ld, dtype=TORCH_DT[odt], device="cuda")[:, :r].t()
    assert "4 rows per access" in coot.kernel_source(None, -1, t, [dA, coot.eye(r, c, odt)], Y)
    coot.eval(t, [dA, coot.eye(r, c, odt)], Y)
    torch.cuda.synchronize()
    assert same(host(Y), oracle.evaluate(t.postfix(), [A, E], "emu")), (dt, r, c)


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
@pytest.mark.parametrize("off", [(4, 2), (1, 1)])
def test_tall_tiles_in_place_on_a_view(dt, off):
    """V = 2*V + 1 in place on a 3000 x 45 view of a 3012 x 48 matrix (whole
    and partial tall tiles; 4 rows per access when the view starts 4 rows
    into aligned columns, single elements and cached loads one row in):
    every element of the view updated once, bit-exact, everything else
    unchanged."""
    R0, C0 = 3012, 48
    i0, j0 = off
    r, c = 3000, 45
    g = np.random.default_rng(3000 + i0 + list(ODT).index(dt))
    M = mat(g, (R0, C0), dt)
    dM = dev(M)
    before = host(dM)
    V = coot.submat(dM, i0, j0, i0 + r - 1, j0 + c - 1)
    tree = x * 2.0 + 1.0
    src = coot.kernel_source(None, -1, tree, [V], V)
    assert "whole tall tile" in src and (("4 rows per access" in src) == (i0 % 4 == 0)), off
    coot.eval(tree, [V], V)
    torch.cuda.synchronize()
    after = host(dM)
    sub = synth.Mat(np.asfortranarray(M.data[i0:i0 + r, j0:j0 + c]), dt)
    want = oracle.evaluate(tree.postfix(), [sub], "emu")
    got = after[i0:i0 + r, j0:j0 + c]
    if dt == "bf16":
        want = oracle.round_to("bf16", want.reshape(-1, order="F")).reshape(want.shape, order="F")
    assert same(got, want), (dt, off)
    mask = np.ones((R0, C0), dtype=bool)
    mask[i0:i0 + r, j0:j0 + c] = False
    assert np.array_equal(after[mask], before[mask])
