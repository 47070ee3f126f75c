"""Operands beyond 2^31 elements: every kernel kind addresses memory and
tracks indices in 64 bits.  Inputs are built on the device in chunks from
integer patterns (exact in FP32), with extremes planted beyond element 2^31.
Element-wise results are checked at sampled indices (including both sides of
2^31 and the ragged tail) against the oracle evaluated on the sampled inputs;
reductions against exact closed forms of the patterns."""
import numpy as np
import pytest

import oracle
import synth
from synth import leaf, leaves, trans

from gpu_util import need_gpu, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

X = leaf(0)
x, y = leaves(2)
N = (1 << 31) + 37          # elements of the flat vectors
CH = 1 << 27                # generation chunk


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)
    free, _ = torch.cuda.mem_get_info()
    if free < 40 * (1 << 30):
        pytest.skip("needs 40 GiB of free device memory")


def pattern_vector(n, mod):
    """v[i] = i % mod as FP32, built in chunks on the device"""
    v = torch.empty(n, dtype=torch.float32, device="cuda")
    for s in range(0, n, CH):
        e = min(n, s + CH)
        v[s:e] = (torch.arange(s, e, device="cuda", dtype=torch.int64) % mod).to(torch.float32)
    return v


def samples(n, g):
    idx = {0, 1, (1 << 31) - 2, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, n - 2, n - 1}
    idx |= set(int(i) for i in g.integers(0, n, 2000))
    return np.array(sorted(idx), np.int64)


def test_flat_elementwise_and_reductions_beyond_2e31():
    g = np.random.default_rng(31)
    v = pattern_vector(N, 1000)
    top, bottom = (1 << 31) + 11, N - 1
    v[top] = 5000.0
    v[bottom] = -7.0
    w = torch.empty_like(v)
    tree = X * 2.0 - 0.5
    coot.eval(tree, [v], w)
    torch.cuda.synchronize()
    idx = samples(N, g)
    ti = torch.from_numpy(idx).cuda()
    xs = v[ti].double().cpu().numpy()
    got = w[ti].double().cpu().numpy()
    want = oracle.evaluate(tree.postfix(), [synth.Mat(np.asfortranarray(xs.astype(np.float32).reshape(-1, 1)), "f32")],
                           "emu")[:, 0]
    assert np.array_equal(got, want)
    # reductions over the whole vector: closed forms of i % 1000 with the planted values
    full, rest = divmod(N, 1000)
    exact = full * 499500 + rest * (rest - 1) // 2
    exact += 5000 - (top % 1000) + (-7) - (bottom % 1000)
    s = coot.reduce("accu", X, [v]).item()
    assert abs(s - exact) <= 1e-6 * exact
    assert coot.reduce("index_max", X, [v]).item() == top
    assert coot.reduce("index_min", X, [v]).item() == bottom
    assert coot.reduce("max", X, [v]).item() == 5000.0
    n999 = full + (1 if rest > 999 else 0) - (1 if top % 1000 == 999 else 0) - (1 if bottom % 1000 == 999 else 0)
    assert coot.reduce("count", X > 998.5, [v]).item() == n999 + 1          # + the planted 5000
    del v, w
    torch.cuda.empty_cache()


def test_transposed_read_and_column_sums_beyond_2e31():
    """A 65536 x 32771 matrix (2^31 + 3 * 2^16 elements) read transposed, and
    summed per column."""
    g = np.random.default_rng(32)
    R, C = 1 << 16, (1 << 15) + 3
    # A[r, c] = (7 r + 13 c) % 1009, column-major, built a column block at a time
    A = torch.empty(C, R, dtype=torch.float32, device="cuda")      # row c of this is column c of A
    rr = torch.arange(R, device="cuda", dtype=torch.int64)
    for c0 in range(0, C, 2048):
        c1 = min(C, c0 + 2048)
        cc = torch.arange(c0, c1, device="cuda", dtype=torch.int64)
        A[c0:c1] = ((7 * rr[None, :] + 13 * cc[:, None]) % 1009).to(torch.float32)
    Am = A.t()                                                      # R x C, ld = R
    Y = torch.empty(R, C, dtype=torch.float32, device="cuda").t()   # C x R, ld = C
    coot.eval(trans(x) * 1.0, [Am], Y)
    torch.cuda.synchronize()
    # sampled elements: Y[i, j] = A[j, i], on both sides of element 2^31 of Y
    i = g.integers(0, C, 3000)
    j = g.integers(0, R, 3000)
    i[:4] = [C - 1, C - 1, (1 << 31) % C, 0]
    j[:4] = [R - 1, 0, (1 << 31) // C, R - 1]
    ti, tj = torch.from_numpy(i).cuda(), torch.from_numpy(j).cuda()
    assert torch.equal(Y[ti, tj], Am[tj, ti])
    del Y
    torch.cuda.empty_cache()
    # per-column sums: the compensated sum of these integers is exact, rounded once to FP32
    cs = coot.reduce("sum", X, [Am], dim=0)
    cols = np.array([0, 1, C // 2, C - 2, C - 1], np.int64)
    r = np.arange(R, dtype=np.int64)
    for c in cols:
        col = ((7 * r + 13 * c) % 1009).astype(np.float32)
        o, _, _ = oracle.reduce("accu", X.postfix(), [synth.Mat(np.asfortranarray(col.reshape(-1, 1)), "f32")])
        assert cs[int(c)].item() == float(np.float32(o[0])), c
    # the index of the largest element, counted over all 2^31+ elements
    Am[R - 5, C - 2] = 2000.0
    assert coot.reduce("index_max", X, [Am]).item() == (R - 5) + (C - 2) * R
    del A, Am
    torch.cuda.empty_cache()


def test_thin_view_with_wide_stride_after_narrow_stride():
    """A 2 x 40 FP64 view whose column stride (2^24 + 8 elements) puts the
    per-lane offsets of a tile step beyond 32 bits, evaluated after the same
    tree on a 2 x 40 view with a stride of 3: each call must run the kernel
    built for its own offset width (the per-call kernel cache keys on it)."""
    g = np.random.default_rng(33)
    cols = 40
    tree = X * 2.0 - 0.5
    for ld in (3, (1 << 24) + 8):                    # the narrow stride first
        M = torch.empty(cols, ld, dtype=torch.float64, device="cuda").t()    # ld x cols, column-major
        vals = g.uniform(-4, 4, (2, cols))
        M[0:2, :] = torch.from_numpy(vals).cuda()
        view = M[0:2, :]
        assert coot.operand(view).ld == ld
        Y = torch.empty(cols, 2, dtype=torch.float64, device="cuda").t()
        coot.eval(tree, [view], Y)
        torch.cuda.synchronize()
        want = oracle.evaluate(tree.postfix(), [synth.Mat(np.asfortranarray(vals), "f64")], "emu")
        assert np.array_equal(Y.cpu().numpy(), want), ld
        del M, Y, view
        torch.cuda.empty_cache()
