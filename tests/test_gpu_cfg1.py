"""Small plain-method workload at its full size: FP32 column-major 1000 x 1000
A, B, C ~ U[-1,1], D ~ U[-4,4]; Y = 2.5*A + B%C - exp(D) as one fused kernel,
s = accu(A%B), sum(A, dim=0), index_max(abs(B)).  Every output is compared
with the oracle element by element."""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import dev, empty, host, need_gpu, rel, scaled_err, classes_match, sum_gate, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402


@pytest.fixture(scope="module")
def data():
    need_gpu()
    coot.init(0)
    mats = synth.cfg1_inputs()
    ms = [mats[k] for k in "ABCD"]
    return ms, [dev(m) for m in ms], synth.cfg1_trees()


def test_Y_fused(data):
    ms, dv, trees = data
    Y = empty(1000, 1000)
    coot.eval(trees["Y"], dv, Y)
    torch.cuda.synchronize()
    g = host(Y)
    ex, S = oracle.evaluate(trees["Y"].postfix(), ms, "exact", scale=True)
    assert classes_match(g, ex)
    e = scaled_err(g, ex, S)
    assert e <= 1e-6, e
    # without exp the same tree is arithmetic only: bit-exact against per-node rounding
    A, B, C, D = synth.leaves(4)
    t2 = 2.5 * A + B % C - D
    Y2 = empty(1000, 1000)
    coot.eval(t2, dv, Y2)
    torch.cuda.synchronize()
    em = oracle.evaluate(t2.postfix(), ms, "emu")
    assert np.array_equal(host(Y2), em)


def test_accu_AB(data):
    ms, dv, trees = data
    s = coot.reduce("accu", trees["accu_AB"], dv).item()
    o, _, asum = oracle.reduce("accu", trees["accu_AB"].postfix(), ms)
    assert rel(s, o[0]) <= 1e-6, (s, o[0])


def test_sum_A_dim0(data):
    ms, dv, trees = data
    s = coot.reduce("sum", trees["sumA"], dv, dim=0).double().cpu().numpy()
    o, _, asum = oracle.reduce("sum", trees["sumA"].postfix(), ms, dim=0)
    # columns of 1000 terms: relative 1e-6 unless a column's sum is ill-conditioned
    gates = sum_gate(s, o, asum, 1000, 1e-6, what="sum(A, 0)")
    assert gates["relative"] >= 990, gates


def test_index_max_abs_B(data):
    ms, dv, trees = data
    i = int(coot.reduce("index_max", trees["absB"], dv).item())
    _, oi, _ = oracle.reduce("index_max", trees["absB"].postfix(), ms)
    assert i == oi[0]


def test_unfused_matches(data):
    ms, dv, trees = data
    Y = empty(1000, 1000)
    Yu = empty(1000, 1000)
    coot.eval(trees["Y"], dv, Y)
    coot.eval(trees["Y"], dv, Yu, unfused=True)
    torch.cuda.synchronize()
    assert torch.equal(Y, Yu)
