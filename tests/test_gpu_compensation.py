"""The compensated accumulation of 16- and 32-bit data, told apart from plain
FP32 accumulation on a sum with no cancellation at all (condition number 1).

Input: n = 2^26 positive terms, the first half equal to L = 1 and the second
half equal to s = 1.75 * 2^-19, exact in FP32, BF16 and FP16 (an FP16
subnormal).  The exact sum is (n / 2)(1 + s).

Why plain FP32 loses it: the flat reduction used here (2 vectors per thread
per step, 512 threads per block, 512 blocks: the default for these calls)
walks the vector in grid-stride steps of 2^19 vectors, each thread folding
every other vector of a step into one of two running sums, 2^19 running sums
in all.  The first half's 2^25 terms are spread evenly over them, so each
running sum takes its 64 terms from the first half (all equal to 1) before
any from the second half: it holds exactly 64 when the first s arrives, and
s < 2^-18 = half an ulp of 64, so every s is rounded away.  The tree that
follows adds integers exactly, so plain accumulation returns n / 2, a
relative error of s / (1 + s) = 3.3e-6.  The compensated form keeps each lost
s in its correction term and returns the exact sum."""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import dev, need_gpu, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

N = 1 << 26
L = 1.0
S = 1.75 * 2.0 ** -19
FLAT_CFG = (2, 512, 1)


def crafted(dt):
    v = np.full(N, S)
    v[: N // 2] = L
    st = synth.store(v, dt)
    assert np.array_equal(st.astype(np.float64) if dt in ("f32", "f64") else oracle.widen16(dt, st), v)
    return synth.Mat(np.asfortranarray(st.reshape(-1, 1)), dt)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16"])
def test_compensated_sum_is_exact_where_plain_fp32_is_not(dt):
    M = crafted(dt)
    ones = synth.Mat(np.asfortranarray(synth.store(np.ones((N, 1)), dt)), dt)
    exact = (N // 2) * (L + S)
    X = synth.leaf(0)
    prod = synth.leaf(0) % synth.leaf(1)
    o, _, asum = oracle.reduce("accu", X.postfix(), [M])
    assert o[0] == exact and asum[0] == exact   # kappa = 1
    od, _, _ = oracle.reduce("dot", prod.postfix(), [M, ones])
    assert od[0] == exact
    dM, dO = dev(M), dev(ones)
    out = torch.empty(1, dtype=torch.float32, device="cuda")
    # the default launch is the one analysed above
    assert coot.config_of(coot.default_config("accu", -1, X, [dM], out)) == FLAT_CFG
    assert coot.config_of(coot.default_config("dot", -1, prod, [dM, dO], out)) == FLAT_CFG
    for op, tree, ops in (("accu", X, [dM]), ("dot", prod, [dM, dO])):
        comp = coot.reduce(op, tree, ops).double().item()
        plain = coot.reduce(op, tree, ops, pairwise=True).double().item()
        rc, rp = abs(comp - exact) / exact, abs(plain - exact) / exact
        assert rc <= 1e-7, (op, dt, comp, exact, rc)
        assert rp > 1e-6, (op, dt, plain, exact, rp)
        # with the launch configuration stated explicitly the results are the same
        assert coot.reduce(op, tree, ops, cfg=FLAT_CFG).double().item() == comp


def test_fp16_leaf_sums_special_values():
    """Compensated FP16 leaf sums (accu, per-column sum) add each half from
    its storage word through the mixed-precision FMA: infinities and NaNs
    propagate as in IEEE addition, subnormal halves count at their value and
    the largest half sums exactly."""
    g = np.random.default_rng(11)
    r, c = 4099, 6
    v = g.uniform(-1, 1, (r, c))
    v[:, 1] = 2.0 ** -24 * g.integers(1, 1024, r)   # subnormal halves only
    v[:, 2] = 65504.0                               # the largest half
    v[100, 3] = np.inf
    v[7, 4], v[3000, 4] = np.inf, -np.inf
    v[2048, 5] = np.nan
    M = synth.Mat(np.asfortranarray(synth.store(v, "f16")), "f16")
    w = oracle.widen16("f16", M.data)
    X = synth.leaf(0)
    dM = dev(M)
    col = coot.reduce("sum", X, [dM], dim=0).double().cpu().numpy().reshape(-1)
    for j in (0, 1, 2):
        exact = float(np.sum(w[:, j]))   # FP64 sums of halves: exact for these columns
        assert abs(col[j] - exact) <= 1e-6 * abs(exact), (j, col[j], exact)
    assert col[1] > 0 and col[2] == float(np.float32(r * 65504.0))
    assert col[3] == np.inf and np.isnan(col[4]) and np.isnan(col[5])
    for cols, expect in (([0, 1, 2], None), ([0, 3], np.inf), ([4], "nan"), ([5, 0], "nan")):
        sub = synth.Mat(np.asfortranarray(M.data[:, cols]), "f16")
        got = coot.reduce("accu", X, [dev(sub)]).double().item()
        if expect is None:
            exact = float(np.sum(w[:, cols]))
            assert abs(got - exact) <= 1e-6 * abs(exact), (cols, got, exact)
        elif expect == "nan":
            assert np.isnan(got), cols
        else:
            assert got == expect, (cols, got)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_compensated_sums_propagate_infinities(dt):
    """An infinite term makes every later TwoSum correction NaN; accu and the
    sums along either dimension (row sums through the per-row combine) still
    return inf for one infinity and NaN for both signs or a NaN."""
    g = np.random.default_rng(12)
    for r, c in ((5000, 8), (8, 300000)):
        v = g.uniform(-1, 1, (r, c))
        v[r // 2, 1] = np.inf                     # column 1 and row r//2: +inf
        v[1, 2], v[r - 1, 2] = np.inf, -np.inf    # column 2: NaN
        v[0, 3] = np.nan                          # column 3 and row 0: NaN
        M = synth.Mat(np.asfortranarray(synth.store(v, dt)), dt)
        X = synth.leaf(0)
        dM = dev(M)
        col = coot.reduce("sum", X, [dM], dim=0).double().cpu().numpy().reshape(-1)
        assert col[1] == np.inf and np.isnan(col[2]) and np.isnan(col[3]) and np.isfinite(col[0]), (r, c)
        row = coot.reduce("sum", X, [dM], dim=1).double().cpu().numpy().reshape(-1)
        assert np.isnan(row[0]) and row[1] == np.inf and row[r - 1] == -np.inf, (r, c)
        assert row[r // 2] == np.inf and np.isfinite(row[2]), (r, c)
        assert np.isnan(coot.reduce("accu", X, [dM]).double().item())
        one = synth.Mat(np.asfortranarray(M.data[:, :2]), dt)
        assert coot.reduce("accu", X, [dev(one)]).double().item() == np.inf
