"""Helpers shared by the GPU parity tests: moving seeded inputs to the device
in column-major layout, bringing results back, and the comparison metrics."""
from __future__ import annotations

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

TORCH_DT = {"f32": torch.float32, "f64": torch.float64, "f16": torch.float16, "bf16": torch.bfloat16}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def dev(m, ld: int | None = None, offset: int = 0):
    """Device copy of a synth.Mat (or a 1-D numpy vector) in column-major layout.

    ``ld`` > n_rows places the matrix inside a taller allocation (a submatrix
    view); ``offset`` shifts the start by that many elements (misalignment)."""
    if isinstance(m, synth.Mat):
        data, dt = m.data, m.dtype
    else:
        data = np.asarray(m)
        dt = {np.dtype(np.float32): "f32", np.dtype(np.float64): "f64"}[data.dtype]
        data = data.reshape(-1, 1)
    r, c = data.shape
    if dt in ("f16", "bf16"):
        host = torch.from_numpy(np.ascontiguousarray(data.T).view(np.int16)).view(TORCH_DT[dt])
    else:
        host = torch.from_numpy(np.ascontiguousarray(data.T))
    L = ld if ld is not None else max(1, r)
    buf = torch.zeros(c * L + offset + 1, dtype=TORCH_DT[dt], device="cuda")
    view = buf[offset:offset + c * L].view(c, L)[:, :r]
    view.copy_(host.cuda())
    t = view.t()
    if not isinstance(m, synth.Mat):
        return t[:, 0] if offset == 0 and ld is None else t
    return t


def empty(r: int, c: int, dt: str = "f32", ld: int | None = None, offset: int = 0):
    L = ld if ld is not None else max(1, r)
    buf = torch.full((c * L + offset + 1,), float("nan"), dtype=TORCH_DT[dt], device="cuda")
    return buf[offset:offset + c * L].view(c, L)[:, :r].t()


def host(t) -> np.ndarray:
    """float64 numpy copy (2-D results keep their (rows, cols) shape)."""
    return t.detach().to(torch.float64).cpu().numpy()


def same(g: np.ndarray, o: np.ndarray) -> bool:
    """Bit-for-bit equality of float64 values (NaN equals NaN, +0 != -0)."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    if g.shape != o.shape:
        return False
    # NaN payloads and signs carry no meaning (x86 and the GPU make different default NaNs)
    nan = np.isnan(g) | np.isnan(o)
    if not np.array_equal(np.isnan(g), np.isnan(o)):
        return False
    gv, ov = g[~nan], o[~nan]
    return bool(np.array_equal(gv.view(np.int64), ov.view(np.int64)))


def mismatch_report(g, o, k=5) -> str:
    g = np.asarray(g, np.float64).reshape(-1, order="F")
    o = np.asarray(o, np.float64).reshape(-1, order="F")
    bad = np.nonzero(~((g == o) | (np.isnan(g) & np.isnan(o))))[0]
    return f"{bad.size} mismatches; first: " + ", ".join(f"[{i}] gpu={g[i]!r} oracle={o[i]!r}" for i in bad[:k])


def scaled_err(g, ex, S) -> float:
    """max_i |g_i - x_i| / S_i over finite entries (S_i = 0 demands equality)."""
    g = np.asarray(g, np.float64)
    ex = np.asarray(ex, np.float64)
    S = np.asarray(S, np.float64)
    fin = np.isfinite(ex) & np.isfinite(g)
    d = np.abs(g[fin] - ex[fin])
    s = S[fin]
    zero = s == 0
    if np.any(d[zero] != 0):
        return float("inf")
    return float(np.max(d[~zero] / s[~zero])) if np.any(~zero) else 0.0


def classes_match(g, ex) -> bool:
    g = np.asarray(g, np.float64)
    ex = np.asarray(ex, np.float64)
    return bool(np.array_equal(np.isnan(g), np.isnan(ex)) and np.array_equal(np.isposinf(g), np.isposinf(ex))
                and np.array_equal(np.isneginf(g), np.isneginf(ex)))


def rel(g: float, o: float) -> float:
    return abs(g - o) / abs(o) if o != 0 else abs(g)
