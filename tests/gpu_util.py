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


# ---- gate of a compensated sum ------------------------------------------------
U_FP32 = 2.0 ** -24   # unit roundoff of the FP32 accumulation (F32, F16, BF16 data)
U_FP64 = 2.0 ** -53   # unit roundoff of the FP64 accumulation (F64 and integer data)
ILL_CONDITIONED = 1e-7


def sum_gate(got, o, asum, n_terms, tol, u=U_FP32, what="sum", nonneg=False):
    """Gate each result of a sum-like reduction against the exact sum o of its
    terms, whose absolute values add up to asum.

    The gate is the relative error |g - o| / |o| <= tol.  Only where the sum is
    ill-conditioned, kappa * n * u^2 > 1e-7 with the condition number
    kappa = asum / |o| and n the number of terms, may the normwise error
    |g - o| / asum <= tol stand in: a compensated sum in working precision u
    is accurate to about u |o| + n u^2 asum, so the relative gate is reachable
    wherever that second term stays well below tol |o|.  nonneg marks sums
    of nonnegative terms (norms, sums of squares): kappa = 1.  Raises
    AssertionError naming the result, the gate that applied and both errors;
    returns the number of results judged by each gate."""
    g = np.atleast_1d(np.asarray(got, np.float64))
    o = np.atleast_1d(np.asarray(o, np.float64))
    a = np.atleast_1d(np.asarray(asum, np.float64))
    err = np.abs(g - o)
    with np.errstate(divide="ignore", invalid="ignore"):
        kappa = np.where(nonneg, 1.0, np.where(o != 0, a / np.abs(o), np.inf))
        relerr = np.where(o != 0, err / np.abs(o), np.where(err == 0, 0.0, np.inf))
        normwise = np.where(a > 0, err / a, np.where(err == 0, 0.0, np.inf))
    fallback = kappa * float(n_terms) * u * u > ILL_CONDITIONED
    ok = np.where(fallback, normwise <= tol, relerr <= tol)
    if not np.all(ok):
        k = int(np.nonzero(~ok)[0][0])
        gate = "normwise (ill-conditioned)" if fallback[k] else "relative"
        raise AssertionError(
            f"{what}[{k}] fails the {gate} gate {tol:g}: gpu={g[k]!r} exact={o[k]!r} rel={relerr[k]:.3e} "
            f"normwise={normwise[k]:.3e} kappa={kappa[k]:.3e} n={n_terms} ({int(np.sum(~ok))} of {o.size} fail)")
    return {"relative": int(np.sum(~fallback)), "normwise": int(np.sum(fallback))}
