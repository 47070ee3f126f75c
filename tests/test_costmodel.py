"""What the learned launch-configuration model gains over the method without it.

The corpus table (exhaustive autotuner timings of all 64 configurations for
6,000 seeded random trees, their features and the default configuration) and
the trained weights were produced on the MI355X by
``python bench.py --workload costmodel`` and are committed with the package.
On the 1,000 held-out trees the model's picks (argmin of the FP64 oracle
forward of the committed weights) must beat the fixed default configuration
in mean regret against the exhaustive autotuner.  Parity unpinned: the gain is
an empirical property of the measured table, not a closed form.
"""
import os

import numpy as np
import pytest

import synth
from oracle import mlp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DATA = os.path.join(ROOT, "paper_2308_03120_amd", "data")
CORPUS = os.path.join(DATA, "costmodel_corpus.npz")
WEIGHTS = os.path.join(DATA, "costmodel_weights.bin")

pytestmark = pytest.mark.skipif(not (os.path.exists(CORPUS) and os.path.exists(WEIGHTS)),
                                reason="cost-model corpus not measured yet")


def unpack(v):
    return {"W1": v[:2048].reshape(32, 64), "b1": v[2048:2112], "W2": v[2112:6208].reshape(64, 64),
            "b2": v[6208:6272]}


@pytest.fixture(scope="module")
def data():
    z = np.load(CORPUS)
    w = np.fromfile(WEIGHTS, dtype=np.float32).astype(np.float64)
    assert w.size == 6272 + 64
    return z, unpack(w[:6272]), w[6272:6304], w[6304:6336]


def regret(times, picks):
    return times[np.arange(times.shape[0]), picks] / times.min(axis=1) - 1.0


def test_split_matches_seeded_split(data):
    z, *_ = data
    tr, te = synth.cfg5_split(6000, 5000)
    assert np.array_equal(z["train"], tr) and np.array_equal(z["test"], te)
    assert z["times"].shape == (6000, 64) and np.all(z["times"] > 0)


def test_model_beats_default_on_held_out(data):
    z, p, mean, std = data
    te = z["test"]
    X = (z["feats"][te].astype(np.float64) - mean) / std
    Y, _ = mlp.forward(p, X)
    picks = Y.argmin(axis=1)
    t = z["times"][te].astype(np.float64)
    r_model = regret(t, picks)
    r_def = regret(t, z["default"][te])
    assert r_model.mean() < r_def.mean(), (r_model.mean(), r_def.mean())
    # geometric-mean speedup of the model's choice over the default choice
    sp = np.exp(np.mean(np.log(t[np.arange(len(te)), z["default"][te]] / t[np.arange(len(te)), picks])))
    assert sp > 1.0
