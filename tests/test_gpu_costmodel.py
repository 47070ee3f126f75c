"""The committed cost model inside the library: installed weights (coot_model_set,
or a stamped file through coot_set_tuning(COOT_TUNE_MODEL)) are run, at plan
time, by the MLP forward kernel on the call's features; its pick must be the argmin of the FP64 oracle forward of the
same weights on the same features (up to near-ties the FP32 kernel may order
differently), and the tuned call must still compute the right values."""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp

from gpu_util import need_gpu, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot, costmodel as cm  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2308_03120_amd", "data", "costmodel_weights.bin")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)
    if not os.path.exists(WEIGHTS):
        pytest.skip("no committed cost model")
    yield
    coot.set_tuning(coot.TUNE_DEFAULT)


def unpack(v):
    return {"W1": v[:2048].reshape(32, 64), "b1": v[2048:2112], "W2": v[2112:6208].reshape(64, 64),
            "b2": v[6208:6272]}


def test_library_inference_matches_oracle_forward():
    params, mean, std = cm.load_model(WEIGHTS)
    p = unpack(params.astype(np.float64))
    coot.model_set(params, mean, std)
    coot.set_tuning(coot.TUNE_MODEL)
    trees = synth.cfg5_trees(6000)
    _, te = synth.cfg5_split(6000, 5000)
    mismatches = 0
    for i in te[:80]:
        rt = trees[i]
        red, dim, ops, out = cm.fake_call(rt)
        f = np.asarray(coot.features(red, dim, rt.expr, ops, out), np.float64)
        x = (f.astype(np.float32) - mean) / std
        y, _ = mlp.forward(p, x.astype(np.float32).astype(np.float64)[None, :])
        y = y[0]
        want = int(np.argmin(y))
        got = coot.model_choose(red, dim, rt.expr, ops, out)
        if got != want:
            # accepted only where the FP32 kernel may order a near-tie differently
            assert y[got] - y[want] <= 1e-4 * max(1.0, abs(y[want])), (i, got, want, y[got], y[want])
            mismatches += 1
    assert mismatches <= 2


def test_stamped_file_loads(tmp_path):
    """A model file stamped with the library's kernels is accepted by
    coot_set_tuning and installed (its picks are the installed weights')."""
    params, mean, std = cm.load_model(WEIGHTS)
    path = str(tmp_path / "stamped.bin")
    cm.save_model(path, params, mean, std)
    coot.set_tuning(coot.TUNE_MODEL, path)
    rt = synth.cfg5_trees(6000)[int(synth.cfg5_split(6000, 5000)[1][0])]
    red, dim, ops, out = cm.fake_call(rt)
    a = coot.model_choose(red, dim, rt.expr, ops, out)
    coot.model_set(params, mean, std)
    assert coot.model_choose(red, dim, rt.expr, ops, out) == a
    coot.set_tuning(coot.TUNE_DEFAULT)


def test_model_tuned_calls_compute_the_same_values():
    coot.model_set(*cm.load_model(WEIGHTS))
    coot.set_tuning(coot.TUNE_MODEL)
    g = np.random.default_rng(17)
    x, y = synth.leaves(2)
    A = synth.Mat(np.asfortranarray(g.uniform(0.5, 2.0, (300, 700)).astype(np.float32)), "f32")
    B = synth.Mat(np.asfortranarray(g.uniform(0.5, 2.0, (700, 300)).astype(np.float32)), "f32")
    dA = torch.from_numpy(np.ascontiguousarray(A.data.T)).cuda().t()
    dB = torch.from_numpy(np.ascontiguousarray(B.data.T)).cuda().t()
    t = synth.trans(x) % y - synth.sqrt(y)
    Y = torch.empty(300, 700, device="cuda").t()
    coot.eval(t, [dA, dB], Y)
    s = coot.reduce("accu", t, [dA, dB]).double().item()
    torch.cuda.synchronize()
    em = oracle.evaluate(t.postfix(), [A, B], "emu")
    assert np.array_equal(Y.cpu().numpy().astype(np.float64), em)
    o, _, _ = oracle.reduce("accu", t.postfix(), [A, B], mode="emu")
    assert abs(s - o[0]) <= 1e-6 * abs(o[0])
    coot.set_tuning(coot.TUNE_DEFAULT)
