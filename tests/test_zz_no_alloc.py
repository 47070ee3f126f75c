"""The allocation-free reduction entry point (coot_reduce_noalloc) through the
C ABI: bit-identical to coot_reduce for the same call, on two calls in a row
(the second smaller, so stale partials of the first would show), for every
reduction kind that keeps block partials; host-side refusals (host output,
kernel not loaded yet, partials beyond the static array) return their error
codes before anything is launched."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from synth import leaf, leaves, trans

from gpu_util import dev, host, need_gpu, same, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

X = leaf(0)
A, B = leaves(2)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


def mat(g, shape, dt):
    return synth.Mat(synth.store(np.asfortranarray(g.uniform(-1.0, 1.0, shape)), dt), dt)


def out_like(op, tree, mats, dim):
    r, c, prec = oracle.shape(tree, mats)
    n_out = 1 if dim < 0 else (c if dim == 0 else r)
    if op in ("index_max", "index_min", "count"):
        dt = torch.int64
    else:
        dt = torch.float64 if prec == 64 else torch.float32
    return torch.full((n_out,), -7, dtype=dt, device="cuda")


def noalloc(op, tree, ops, out, dim=-1):
    e = coot.expr(tree)
    arr, n = coot._ops(ops)
    o = coot.operand(out)
    return coot.lib().coot_reduce_noalloc(coot._red_code(op, False), dim, C.byref(e), arr, n, C.byref(o),
                                          C.c_void_p(coot.current_stream()))


ERR_ARG, ERR_NOT_READY = -10, -12

CASES = [
    # (reduction, dim, tree, number of leaves, first leaf read transposed, dtype, first shape, second shape)
    ("accu", -1, A % B, 2, False, "f32", ((1 << 22) + 37, 1), (1003, 1)),   # flat, one partial per block
    ("index_max", -1, X, 1, False, "f64", (4099, 517), (67, 45)),          # flat, value + index partials
    ("var", -1, X, 1, False, "f32", ((1 << 21) + 5, 1), (333, 1)),         # flat, 32-byte partials
    ("accu", -1, trans(A) % B, 2, True, "f32", (700, 900), (65, 130)),    # tiled
    ("sum", 0, X, 1, False, "f32", (1 << 16, 40), (1000, 7)),             # per column, split columns
    ("sum", 1, X, 1, False, "f32", (1000, 5000), (70, 130)),              # per row, split rows
    ("stddev", 1, X, 1, False, "f64", (1000, 5000), (90, 300)),           # per row, variance partials
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}_dim{c[1]}_{c[5]}" for c in CASES])
def test_noalloc_matches_reduce_on_two_calls(case):
    op, dim, tree, nl, t0, dt, s1, s2 = case
    g = np.random.default_rng(909)
    for k, shape in enumerate((s1, s2)):
        mats = [mat(g, (shape[1], shape[0]) if (j == 0 and t0) else shape, dt) for j in range(nl)]
        ops = [dev(m) for m in mats]
        want = coot.reduce(op, tree, ops, dim=dim)
        got = out_like(op, tree, mats, dim)
        print(f"noalloc {op} dim={dim} {dt} shape={shape} call {k + 1}", flush=True)
        rc = noalloc(op, tree, ops, got, dim)
        assert rc == 0, (rc, coot.last_error())
        torch.cuda.synchronize()
        assert same(host(got), host(want)), (op, shape, host(got)[:4], host(want)[:4])
        if k == 1 and op in ("accu", "sum"):
            # and the values are the oracle's, within the sum gate of the per-call path
            o, _, _ = oracle.reduce(op, tree.postfix(), mats, dim=dim, mode="emu")
            rel = np.max(np.abs(host(got) - o) / np.maximum(np.abs(o), 1e-300))
            assert rel <= 1e-6, rel


def test_noalloc_refusals():
    g = np.random.default_rng(5)
    m = mat(g, (300, 20), "f32")
    a = dev(m)
    # host output
    hout = torch.zeros(1, dtype=torch.float32)
    o = coot.operand(hout, host=True)
    e = coot.expr(X)
    arr, n = coot._ops([a])
    rc = coot.lib().coot_reduce_noalloc(coot._red_code("accu", False), -1, C.byref(e), arr, n, C.byref(o),
                                        C.c_void_p(coot.current_stream()))
    assert rc == ERR_ARG, rc
    # a tree whose kernel has never been loaded in this process
    fresh = (X * 3.0625 + 1.8125) % X
    out = torch.zeros(1, dtype=torch.float32, device="cuda")
    assert noalloc("accu", fresh, [a], out) == ERR_NOT_READY
    assert "not loaded" in coot.last_error()
    want = coot.reduce("accu", fresh, [a])
    assert noalloc("accu", fresh, [a], out) == 0
    torch.cuda.synchronize()
    assert same(host(out), host(want))
    # partials beyond the static array: 2^19 + 4 rows in two column splits
    big = torch.zeros(128, (1 << 19) + 4, dtype=torch.float32, device="cuda").t()
    rows = coot.reduce("sum", X, [big], dim=1)
    torch.cuda.synchronize()
    before = rows.clone()
    assert noalloc("sum", X, [big], rows, dim=1) == ERR_ARG
    assert "static scratch" in coot.last_error()
    torch.cuda.synchronize()
    assert torch.equal(rows, before)
