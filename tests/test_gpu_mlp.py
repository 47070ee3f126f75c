"""The cost model's MLP kernels (FP32, on the GPU) against the FP64 oracle:
forward values, loss and every gradient, and one Adam step."""
import numpy as np
import pytest

from oracle import mlp

from gpu_util import need_gpu, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402


def pack(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"]])


def unpack(v):
    return {"W1": v[:2048].reshape(32, 64), "b1": v[2048:2112], "W2": v[2112:6208].reshape(64, 64), "b2": v[6208:]}


@pytest.fixture(scope="module")
def case():
    need_gpu()
    coot.init(0)
    g = np.random.default_rng(31)
    p = mlp.init_params(g)
    p["b1"] = g.standard_normal(64) * 0.1
    p["b2"] = g.standard_normal(64) * 0.1
    B = 517
    X = g.standard_normal((B, 32))
    T = g.standard_normal((B, 64))
    M = (g.random((B, 64)) < 0.9).astype(np.float64)
    # the GPU computes in FP32 from FP32 inputs: give the oracle the same rounded inputs
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    X, T = X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64)
    return p, X, T, M


def d(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_forward(case):
    p, X, T, M = case
    Y = torch.zeros(X.shape[0], 64, device="cuda")
    coot.mlp_forward(d(pack(p)), d(X), Y)
    Yo, _ = mlp.forward(p, X)
    assert rel(Y.cpu().numpy().astype(np.float64), Yo) <= 1e-6


def test_backward_and_loss(case):
    p, X, T, M = case
    B = X.shape[0]
    grad = torch.zeros(coot.MLP_N_PARAMS, device="cuda")
    loss = torch.zeros(1, device="cuda")
    ws = torch.zeros(coot.mlp_ws_floats(B), device="cuda")
    coot.mlp_backward(d(pack(p)), d(X), d(T), d(M), grad, loss, ws)
    Yo, cache = mlp.forward(p, X)
    go = mlp.backward(p, cache, Yo, T, M)
    assert abs(loss.item() - mlp.loss(Yo, T, M)) <= 1e-5 * mlp.loss(Yo, T, M)
    gg = unpack(grad.cpu().numpy().astype(np.float64))
    for k in ("W1", "b1", "W2", "b2"):
        assert rel(gg[k], go[k]) <= 1e-5, k


def test_adam_step(case):
    g = np.random.default_rng(8)
    w = g.standard_normal(coot.MLP_N_PARAMS)
    gr = g.standard_normal(coot.MLP_N_PARAMS)
    m = g.standard_normal(coot.MLP_N_PARAMS) * 0.01
    v = np.abs(g.standard_normal(coot.MLP_N_PARAMS)) * 0.01
    w, gr, m, v = (a.astype(np.float32).astype(np.float64) for a in (w, gr, m, v))
    W, GR, Mm, V = d(w), d(gr), d(m), d(v)
    coot.mlp_adam(W, GR, Mm, V, 7, lr=1e-3)
    # the kernel takes its hyper-parameters as floats: give the oracle the same values
    f = lambda x: float(np.float32(x))
    mlp.adam_step(w, gr, m, v, 7, lr=f(1e-3), b1=f(0.9), b2=f(0.999), eps=f(1e-8))
    assert np.max(np.abs(W.cpu().numpy() - w)) <= 1e-6
    assert rel(Mm.cpu().numpy().astype(np.float64), m) <= 1e-6
    assert rel(V.cpu().numpy().astype(np.float64), v) <= 1e-6


def test_library_inference_matches_forward(case):
    """The model the library consults at plan time picks the argmin of the same forward."""
    import synth
    from paper_2308_03120_amd import costmodel as cm

    p, X, T, M = case
    params = pack(p).astype(np.float32)
    mean, std = np.zeros(32, np.float32), np.ones(32, np.float32)
    coot.model_set(params, mean, std)
    g = np.random.default_rng(3)
    trees = synth.cfg5_trees(40)
    for rt in trees[:20]:
        red, dim, ops, out = cm.fake_call(rt)
        f = coot.features(red, dim, rt.expr, ops, out).astype(np.float64)
        Yo, _ = mlp.forward(p, f[None, :])
        assert coot.model_choose(red, dim, rt.expr, ops, out) == int(np.argmin(Yo[0]))
