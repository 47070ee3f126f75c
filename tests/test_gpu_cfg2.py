"""Plain method at scale: FP32 and FP64 vectors of 2^28 elements, x, y ~
N(0,1) with 64 injected tied maxima in x.  axpy y = y + 0.75*x (in place),
z = sqrt(abs(x)) % y - x/(1+abs(y)), dot(x, y), norm(x), index_max(x), in the
launch configuration the benchmark uses.  Element-wise results are checked
bit-exactly on 2^20 sampled indices plus both ends of the vector; the
reductions against the oracle over all 2^28 elements."""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import host, need_gpu, rel, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

N = 1 << 28


@pytest.fixture(scope="module", params=["f32", "f64"])
def data(request):
    need_gpu()
    coot.init(0)
    dt = request.param
    d = synth.cfg2_inputs(dt, n=N)
    X = torch.from_numpy(d["x"]).cuda()
    Y = torch.from_numpy(d["y"]).cuda()
    g = np.random.default_rng(99)
    idx = np.unique(np.concatenate([g.integers(0, N, 1 << 20), np.arange(4096), np.arange(N - 4096, N),
                                    d["ties"]]))
    yield dt, d, X, Y, idx
    del X, Y
    torch.cuda.empty_cache()


def test_axpy_in_place(data):
    dt, d, X, Y, idx = data
    t = synth.cfg2_trees()["axpy"]
    Yw = Y.clone()
    coot.eval(t, [X, Yw], Yw)
    torch.cuda.synchronize()
    got = Yw[torch.from_numpy(idx).cuda()].double().cpu().numpy()
    want = oracle.evaluate_at(t.postfix(), [d["x"], d["y"]], idx, "emu")
    assert np.array_equal(got, want)


def test_z(data):
    dt, d, X, Y, idx = data
    t = synth.cfg2_trees()["z"]
    Z = torch.empty_like(X)
    coot.eval(t, [X, Y], Z)
    torch.cuda.synchronize()
    got = Z[torch.from_numpy(idx).cuda()].double().cpu().numpy()
    want = oracle.evaluate_at(t.postfix(), [d["x"], d["y"]], idx, "emu")
    assert np.array_equal(got, want)
    ex, S = oracle.evaluate_at(t.postfix(), [d["x"], d["y"]], idx, "exact", scale=True)
    tol = 2e-7 if dt == "f32" else 1e-15
    assert np.max(np.abs(got - ex) / S) <= tol


def test_dot(data):
    dt, d, X, Y, idx = data
    t = synth.cfg2_trees()["dot"]
    got = coot.reduce("dot", t, [X, Y]).item()
    o, _, asum = oracle.reduce("dot", t.postfix(), [d["x"], d["y"]])
    assert rel(got, o[0]) <= (1e-6 if dt == "f32" else 1e-13), (got, o[0], asum[0])


def test_norm(data):
    dt, d, X, Y, idx = data
    got = coot.reduce("norm2", synth.leaf(0), [X]).item()
    o, _, _ = oracle.reduce("norm2", [synth.Node("leaf", 0)], [d["x"]])
    assert rel(got, o[0]) <= (1e-6 if dt == "f32" else 1e-13)
    # dot(x, x) = norm(x)^2
    dd = coot.reduce("dot", synth.leaf(0) % synth.leaf(0), [X]).item()
    assert rel(dd, got * got) <= (3e-7 if dt == "f32" else 1e-15)


def test_index_max_ties(data):
    dt, d, X, Y, idx = data
    i = int(coot.reduce("index_max", synth.leaf(0), [X]).item())
    assert i == int(d["ties"].min())
