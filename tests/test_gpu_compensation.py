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
