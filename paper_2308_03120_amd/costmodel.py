"""Learned launch-configuration model: corpus timing, training, evaluation.

The pieces of the method live in the library: the features of a call
(coot_features), the exhaustive autotuner that times all 64 configurations
(coot_autotune), and the MLP forward / backward / Adam kernels
(coot_mlp_forward, coot_mlp_backward, coot_mlp_adam).  This module drives
them over a corpus of random expression trees and packs the trained weights
for coot_set_tuning(COOT_TUNE_MODEL, path).

Model: 32 standardised features -> 64 hidden (ReLU) -> 64 outputs, one per
configuration; the target of output c is log(t_c / t_best), the measured
slowdown of configuration c over the best one for that call.  The chosen
configuration is the argmin of the outputs.
"""
from __future__ import annotations

import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import coot

N_CFG = coot.N_CONFIGS
N_FEAT = coot.N_FEATURES
N_PARAMS = coot.MLP_N_PARAMS
G = 1 << 40


def _dt_code(dt: str) -> int:
    return coot.DTYPE_CODES[dt]


def call_of(rt):
    """(red_op, dim, out shape, out dtype) of a random tree's call."""
    rows, cols = rt.out_shape
    dt = rt.dtypes[0] if rt.dtypes else "f32"
    if rt.reduce is None:
        return None, -1, (rows, cols), dt
    acc = "f64" if dt == "f64" else "f32"
    if rt.reduce == "accu":
        return "accu", -1, (1, 1), acc
    if rt.dim == 0:
        return "sum", 0, (1, cols), acc
    return "sum", 1, (rows, 1), acc


def fake_call(rt):
    """Operand descriptors without memory for the host-only calls."""
    ops = [coot.fake_operand(r, c, dt, ptr=G * (i + 1)) for i, ((r, c), dt) in enumerate(zip(rt.shapes, rt.dtypes))]
    red, dim, (orow, ocol), odt = call_of(rt)
    out = coot.fake_operand(orow, ocol, odt, ld=1 if orow == 1 else orow, ptr=G * 20)
    return red, dim, ops, out


def precompile_corpus(trees, per_module: int = 64, workers: int = 16) -> int:
    """Compile every kernel the corpus needs (4 elements-per-thread variants
    per tree), many kernels per code object, in parallel processes."""
    import multiprocessing as mp

    if workers <= 1 or len(trees) < 2 * workers:
        return _precompile_slice(trees, per_module)
    chunks = [trees[i::workers] for i in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        return sum(pool.starmap(_precompile_slice, [(c, per_module) for c in chunks]))


def _precompile_slice(trees, per_module):
    coot.precompile_begin()
    for rt in trees:
        red, dim, ops, out = fake_call(rt)
        for ept in (1, 2, 4, 8):
            coot.precompile(red, dim, rt.expr, ops, out, cfg=(ept, 256, 8))
    return coot.precompile_end(per_module)


def allocate(rt, torch, gen):
    """Device operands (positive values: log and sqrt stay finite) and output."""
    tdt = {"f32": torch.float32, "f64": torch.float64, "f16": torch.float16, "bf16": torch.bfloat16}
    ops = []
    for (r, c), dt in zip(rt.shapes, rt.dtypes):
        t = torch.empty(c, r, dtype=tdt[dt], device="cuda")
        t.uniform_(0.5, 2.0, generator=gen)
        ops.append(t.t())
    red, dim, (orow, ocol), odt = call_of(rt)
    if red is None:
        out = torch.empty(ocol, orow, dtype=tdt[odt], device="cuda").t()
    else:
        out = torch.empty(orow * ocol, dtype=tdt[odt], device="cuda")
    return red, dim, ops, out


def time_corpus(trees, reps: int = 3, log=None):
    """Exhaustive autotuning of every tree: times (n, 64) in ms, features
    (n, 32), default-configuration index (n,)."""
    import torch

    gen = torch.Generator(device="cuda")
    gen.manual_seed(2308)
    n = len(trees)
    times = np.zeros((n, N_CFG), np.float32)
    feats = np.zeros((n, N_FEAT), np.float32)
    default = np.zeros(n, np.int32)
    t0 = time.time()
    for i, rt in enumerate(trees):
        red, dim, ops, out = allocate(rt, torch, gen)
        feats[i] = coot.features(red, dim, rt.expr, ops, out)
        default[i] = coot.default_config(red, dim, rt.expr, ops, out)
        _, times[i] = coot.autotune(red, dim, rt.expr, ops, out, reps=reps)
        del ops, out
        if log and (i + 1) % 250 == 0:
            log(f"timed {i + 1}/{n} trees, {time.time() - t0:.0f} s")
    return times, feats, default


def targets(times):
    return np.log(times / times.min(axis=1, keepdims=True)).astype(np.float32)


def init_params(seed: int = 5120) -> np.ndarray:
    """He-uniform first layer, Glorot-uniform second, zero biases (packed)."""
    g = np.random.default_rng(seed)
    l1 = np.sqrt(6.0 / 32)
    l2 = np.sqrt(6.0 / (64 + 64))
    W1 = g.uniform(-l1, l1, (32, 64))
    W2 = g.uniform(-l2, l2, (64, 64))
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64)]).astype(np.float32)


def train(X: np.ndarray, T: np.ndarray, steps: int = 3000, lr: float = 3e-3, seed: int = 5120, log=None):
    """Full-batch Adam on the GPU with the library's MLP kernels.
    Returns (params, feature mean, feature std, loss history)."""
    import torch

    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std == 0] = 1.0
    Xs = ((X - mean) / std).astype(np.float32)
    B = Xs.shape[0]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    P = d(init_params(seed))
    Xd, Td, Md = d(Xs), d(T), d(np.ones_like(T))
    grad = torch.zeros_like(P)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    ws = torch.zeros(coot.mlp_ws_floats(B), device="cuda")
    loss = torch.zeros(1, device="cuda")
    hist = []
    for t in range(1, steps + 1):
        coot.mlp_backward(P, Xd, Td, Md, grad, loss, ws)
        coot.mlp_adam(P, grad, m, v, t, lr=lr)
        if t == 1 or t % 250 == 0 or t == steps:
            hist.append((t, float(loss.item())))
            if log:
                log(f"step {t}: loss {hist[-1][1]:.5f}")
    return P.cpu().numpy(), mean.astype(np.float32), std.astype(np.float32), hist


def predict(params: np.ndarray, mean, std, X: np.ndarray) -> np.ndarray:
    """MLP outputs on the GPU (library forward kernel)."""
    import torch

    Xs = ((X - mean) / std).astype(np.float32)
    Pd = torch.from_numpy(np.ascontiguousarray(params, np.float32)).cuda()
    Xd = torch.from_numpy(np.ascontiguousarray(Xs)).cuda()
    Y = torch.zeros(X.shape[0], N_CFG, device="cuda")
    coot.mlp_forward(Pd, Xd, Y)
    return Y.cpu().numpy()


def regret(times: np.ndarray, picks: np.ndarray) -> np.ndarray:
    """t(pick) / t(best of 64) - 1 per call."""
    rows = np.arange(times.shape[0])
    return times[rows, picks] / times.min(axis=1) - 1.0


MODEL_MAGIC = b"COOTMLP2"


def save_model(path: str, params, mean, std, stamp: Optional[int] = None, schema: Optional[int] = None) -> None:
    """Write a cost-model file stamped with the library's feature schema and
    kernel stamp (coot_set_tuning rejects files made for other kernels)."""
    if stamp is None or schema is None:
        schema, stamp = coot.kernel_stamp()
    head = MODEL_MAGIC + np.array([schema, 0], np.uint32).tobytes() + np.array([stamp], np.uint64).tobytes()
    body = np.concatenate([np.asarray(params, np.float32), np.asarray(mean, np.float32),
                           np.asarray(std, np.float32)]).astype(np.float32).tobytes()
    with open(path, "wb") as f:
        f.write(head + body)


def read_model(path: str):
    """(params, mean, std, schema, stamp) of a cost-model file."""
    with open(path, "rb") as f:
        raw = f.read()
    assert raw[:8] == MODEL_MAGIC, "not a stamped cost-model file"
    schema, zero = np.frombuffer(raw[8:16], np.uint32)
    stamp = int(np.frombuffer(raw[16:24], np.uint64)[0])
    a = np.frombuffer(raw[24:], np.float32)
    assert zero == 0 and a.size == N_PARAMS + 64, "cost-model file has the wrong size"
    return a[:N_PARAMS].copy(), a[N_PARAMS:N_PARAMS + 32].copy(), a[N_PARAMS + 32:].copy(), int(schema), stamp


def load_model(path: str):
    return read_model(path)[:3]


def summarize(times, default, picks_model) -> Dict[str, float]:
    rd = regret(times, default)
    rm = regret(times, picks_model)
    rows = np.arange(times.shape[0])
    speed = times[rows, default] / times[rows, picks_model]
    return {
        "n": int(times.shape[0]),
        "regret_default_mean": float(rd.mean()), "regret_default_median": float(np.median(rd)),
        "regret_default_p90": float(np.percentile(rd, 90)),
        "regret_model_mean": float(rm.mean()), "regret_model_median": float(np.median(rm)),
        "regret_model_p90": float(np.percentile(rm, 90)),
        "model_over_default_geomean_speedup": float(np.exp(np.mean(np.log(speed)))),
        "model_exact_best_fraction": float(np.mean(rm == 0.0)),
    }
