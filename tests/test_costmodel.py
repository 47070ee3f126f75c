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


def read_weights(path):
    """The stamped cost-model file: "COOTMLP2", schema (u32), 0 (u32), kernel
    stamp (u64), then 6272 parameters, 32 feature means, 32 feature scales."""
    raw = open(path, "rb").read()
    assert raw[:8] == b"COOTMLP2"
    schema, zero = np.frombuffer(raw[8:16], np.uint32)
    stamp = int(np.frombuffer(raw[16:24], np.uint64)[0])
    w = np.frombuffer(raw[24:], np.float32).astype(np.float64)
    assert zero == 0 and w.size == 6272 + 64
    return w, int(schema), stamp


@pytest.fixture(scope="module")
def data():
    z = np.load(CORPUS)
    w, _, _ = read_weights(WEIGHTS)
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


def test_mismatched_model_files_are_rejected(tmp_path):
    """coot_set_tuning refuses a model file made for other kernels, another
    feature layout or an unstamped one, says why, and leaves no model
    installed (tuning falls back to the tuned cache, then the default).  Host
    only: the checks come before anything is copied to a device."""
    from paper_2308_03120_amd import coot, costmodel as cm

    schema, stamp = coot.kernel_stamp()
    params = np.zeros(cm.N_PARAMS, np.float32)
    mean, std = np.zeros(32, np.float32), np.ones(32, np.float32)
    cases = {
        "stale": (dict(stamp=stamp ^ 1, schema=schema), "retrain"),
        "schema": (dict(stamp=stamp, schema=schema + 1), "feature schema"),
    }
    x = synth.leaf(0)
    ops = [coot.fake_operand(1000, 1, "f32")]
    out = coot.fake_operand(1000, 1, "f32", ptr=3 << 40)
    for name, (kw, why) in cases.items():
        path = str(tmp_path / f"{name}.bin")
        cm.save_model(path, params, mean, std, **kw)
        with pytest.raises(coot.CootError) as e:
            coot.set_tuning(coot.TUNE_MODEL, path)
        assert e.value.code == -10 and why in e.value.msg and "falls back" in e.value.msg
        with pytest.raises(coot.CootError) as e:
            coot.model_choose(None, -1, x + 1.0, ops, out)
        assert "no cost model" in e.value.msg
    # the unstamped layout of earlier files
    raw = str(tmp_path / "raw.bin")
    np.concatenate([params, mean, std]).tofile(raw)
    with pytest.raises(coot.CootError) as e:
        coot.set_tuning(coot.TUNE_MODEL, raw)
    assert "not a stamped" in e.value.msg
    coot.set_tuning(coot.TUNE_DEFAULT)


def test_stamp_follows_the_kernels():
    """The stamp is a pure function of the library's generated kernels and
    launch geometry: stable across calls, and written into saved files."""
    from paper_2308_03120_amd import coot

    a = coot.kernel_stamp()
    assert a == coot.kernel_stamp() and a[0] == 1 and a[1] != 0


def test_committed_weights_match_the_kernels():
    """The committed model was trained on the kernels this library generates:
    its feature schema and kernel stamp equal the library's, so
    coot_set_tuning accepts it (a model timed on other kernels is refused)."""
    from paper_2308_03120_amd import coot

    _, schema, stamp = read_weights(WEIGHTS)
    assert (schema, stamp) == coot.kernel_stamp()
