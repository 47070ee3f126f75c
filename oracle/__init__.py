"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, unfused FP64 reference for the element-wise expression trees and
reductions of the Bandicoot paper (arXiv:2308.03120; Tables 2, 5, 6, 7 and the
delayed evaluation of Section 7).  Only ``tests/``, the smoke check and the CPU
baseline of the benchmark may import this package; the GPU library never does.

The arithmetic lives in ``oracle.c`` (gcc, -ffp-contract=off) and ``mlp.py``
(numpy float64).  This module only marshals arguments: it maps the op names of
the shared tree description onto the oracle's own codes and numpy arrays onto
the C structs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OPS = {
    "leaf": 0, "plus": 1, "minus": 2, "schur": 3, "div": 4,
    "scal_plus": 5, "scal_minus_post": 6, "scal_minus_pre": 7, "scal_times": 8,
    "scal_div_post": 9, "scal_div_pre": 10,
    "exp": 11, "log": 12, "sqrt": 13, "abs": 14, "trans": 15, "conv": 16,
    "gt": 17, "lt": 18, "ge": 19, "le": 20, "eq": 21, "ne": 22,
    "scal_gt": 23, "scal_lt": 24, "scal_ge": 25, "scal_le": 26, "scal_eq": 27, "scal_ne": 28,
    "scal_pow": 29, "log10": 30, "log2": 31, "exp2": 32, "square": 33, "floor": 34, "ceil": 35, "round": 36,
    "trunc": 37, "sign": 38, "cos": 39, "sin": 40, "tan": 41, "acos": 42, "asin": 43, "atan": 44, "cosh": 45,
    "sinh": 46, "tanh": 47,
}
TYPES = {"f32": 0, "f64": 1, "f16": 2, "bf16": 3, "i32": 5, "u32": 6}
MODES = {"exact": 0, "emu": 1}
REDS = {
    "accu": 0, "sum": 1, "dot": 2, "norm1": 3, "norm2": 4, "norminf": 5, "normneginf": 6,
    "min": 7, "max": 8, "index_min": 9, "index_max": 10,
    "mean": 11, "var": 12, "stddev": 13, "count": 14, "all": 15, "any": 16,
}
ERRORS = {-1: "bad tree", -2: "shape mismatch", -5: "empty input", -9: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


class _Node(C.Structure):
    _fields_ = [("op", C.c_int32), ("a", C.c_int32), ("b", C.c_int32), ("pad", C.c_int32),
                ("k", C.c_double)]


class _Leaf(C.Structure):
    _fields_ = [("data", C.c_void_p), ("rows", C.c_int64), ("cols", C.c_int64), ("ld", C.c_int64),
                ("dtype", C.c_int32), ("pad", C.c_int32)]


def build(force: bool = False) -> str:
    """Compile the oracle library (plain gcc, strict IEEE flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int64)
        L.oracle_eval.argtypes = [C.POINTER(_Node), C.c_int, C.POINTER(_Leaf), C.c_int, C.c_int,
                                  dp, dp, ip, ip]
        L.oracle_eval_at.argtypes = [C.POINTER(_Node), C.c_int, C.POINTER(_Leaf), C.c_int, C.c_int,
                                     ip, C.c_int64, dp, dp]
        L.oracle_shape.argtypes = [C.POINTER(_Node), C.c_int, C.POINTER(_Leaf), C.c_int, ip, ip,
                                   C.POINTER(C.c_int32)]
        L.oracle_reduce.argtypes = [C.c_int, C.c_int, C.POINTER(_Node), C.c_int, C.POINTER(_Leaf), C.c_int,
                                    C.c_int, dp, ip, dp]
        L.oracle_sum2.argtypes = [dp, C.c_int64, dp]
        L.oracle_sum2.restype = C.c_double
        L.oracle_dot2.argtypes = [dp, dp, C.c_int64]
        L.oracle_dot2.restype = C.c_double
        L.oracle_round_to.argtypes = [C.c_int, C.c_double]
        L.oracle_round_to.restype = C.c_double
        L.oracle_round_array.argtypes = [C.c_int, dp, dp, C.c_int64]
        L.oracle_widen16_array.argtypes = [C.c_int, C.POINTER(C.c_uint16), dp, C.c_int64]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _nodes(tree) -> "C.Array":
    """tree: list of synth.Node (or an expression builder with .postfix())."""
    if hasattr(tree, "postfix"):
        tree = tree.postfix()
    arr = (_Node * len(tree))()
    for i, n in enumerate(tree):
        arr[i].op = OPS[n.op]
        arr[i].a = n.a
        arr[i].b = n.b
        arr[i].k = n.k
    return arr, len(tree)


def _leaves(mats: Sequence) -> Tuple["C.Array", List[np.ndarray]]:
    """mats: sequence of synth.Mat, or (array, dtype) pairs, or float arrays
    (1-D vectors are taken as n x 1 columns)."""
    keep = []
    arr = (_Leaf * max(1, len(mats)))()
    for i, m in enumerate(mats):
        if hasattr(m, "dtype") and hasattr(m, "data") and isinstance(getattr(m, "dtype"), str):
            data, dt = m.data, m.dtype
        elif isinstance(m, tuple):
            data, dt = m
        else:
            data = np.asarray(m)
            dt = {np.dtype(np.float32): "f32", np.dtype(np.float64): "f64"}[data.dtype]
        if data.ndim == 1:
            data = data.reshape(-1, 1)
        data = np.asfortranarray(data)
        keep.append(data)
        arr[i].data = data.ctypes.data
        arr[i].rows, arr[i].cols = data.shape
        arr[i].ld = data.shape[0]
        arr[i].dtype = TYPES[dt]
    return arr, keep


def shape(tree, mats) -> Tuple[int, int, int]:
    nd, nn = _nodes(tree)
    lv, keep = _leaves(mats)
    r, c, p = C.c_int64(), C.c_int64(), C.c_int32()
    rc = lib().oracle_shape(nd, nn, lv, len(mats), C.byref(r), C.byref(c), C.byref(p))
    if rc:
        raise OracleError(rc)
    return r.value, c.value, p.value


def evaluate(tree, mats, mode: str = "exact", scale: bool = False):
    """Unfused evaluation.  Returns the root values as a (rows, cols) float64
    Fortran-ordered array, and the error scale S if ``scale``."""
    r, c, _ = shape(tree, mats)
    nd, nn = _nodes(tree)
    lv, keep = _leaves(mats)
    out = np.empty(max(1, r * c), np.float64)
    sc = np.empty(max(1, r * c), np.float64) if scale else None
    rc = lib().oracle_eval(nd, nn, lv, len(mats), MODES[mode], _dp(out), _dp(sc) if scale else None, None, None)
    if rc:
        raise OracleError(rc)
    v = out[: r * c].reshape((r, c), order="F")
    if scale:
        return v, sc[: r * c].reshape((r, c), order="F")
    return v


def evaluate_at(tree, mats, lin: np.ndarray, mode: str = "exact", scale: bool = False):
    """Pointwise evaluation at column-major linear indices of the root (and the
    running-error scale S there if ``scale``)."""
    nd, nn = _nodes(tree)
    lv, keep = _leaves(mats)
    lin = np.ascontiguousarray(lin, dtype=np.int64)
    out = np.empty(max(1, lin.size), np.float64)
    sc = np.empty(max(1, lin.size), np.float64) if scale else None
    rc = lib().oracle_eval_at(nd, nn, lv, len(mats), MODES[mode], _ip(lin), lin.size, _dp(out),
                              _dp(sc) if scale else None)
    if rc:
        raise OracleError(rc)
    if scale:
        return out[: lin.size], sc[: lin.size]
    return out[: lin.size]


SUM_LIKE = ("accu", "sum", "dot", "norm1", "norm2", "mean", "var", "stddev")


def reduce(op: str, tree, mats, dim: int = -1, mode: str = None):
    """Reduction of a tree.  Returns (values, indices, abs_sums) as 1-D arrays
    (length 1 for dim=-1, n_cols for dim=0, n_rows for dim=1).

    ``mode`` is how the tree is evaluated before reducing: "exact" (FP64 at
    every node) or "emu" (rounded at every node to the compute precision).
    Default: exact for sums, emu for selections (min/max/index)."""
    if mode is None:
        mode = "exact" if op in SUM_LIKE else "emu"
    r, c, _ = shape(tree, mats)
    n_out = 1 if dim < 0 else (c if dim == 0 else r)
    vals = np.empty(max(1, n_out), np.float64)
    idx = np.empty(max(1, n_out), np.int64)
    asum = np.empty(max(1, n_out), np.float64)
    nd, nn = _nodes(tree)
    lv, keep = _leaves(mats)
    rc = lib().oracle_reduce(REDS[op], dim, nd, nn, lv, len(mats), MODES[mode], _dp(vals), _ip(idx), _dp(asum))
    if rc:
        raise OracleError(rc)
    return vals[:n_out], idx[:n_out], asum[:n_out]


def sum2(x: np.ndarray) -> Tuple[float, float]:
    x = np.ascontiguousarray(x, dtype=np.float64)
    a = C.c_double()
    s = lib().oracle_sum2(_dp(x), x.size, C.byref(a))
    return s, a.value


def dot2(x: np.ndarray, y: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().oracle_dot2(_dp(x), _dp(y), x.size)


def round_to(dtype: str, x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even of float64 values to ``dtype`` (returned as float64)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().oracle_round_array(TYPES[dtype], _dp(x), _dp(y), x.size)
    return y


def widen16(dtype: str, bits: np.ndarray) -> np.ndarray:
    bits = np.ascontiguousarray(bits, dtype=np.uint16)
    y = np.empty(bits.shape, np.float64)
    lib().oracle_widen16_array(TYPES[dtype], bits.ctypes.data_as(C.POINTER(C.c_uint16)), _dp(y), bits.size)
    return y


# ---- generators (Table 1 fill/ones/zeros/eye, Table 4 eye/ones/zeros/linspace)
# Dense operands with the values a memory-free generator leaf stands for.  Each
# value is formed in FP64 as defined below, then stored (round to nearest even)
# in the generator's element type, exactly like a value read from memory.
def _stored(values: np.ndarray, dtype: str):
    """(Fortran array in the storage representation, dtype) of FP64 values."""
    v = np.asfortranarray(np.asarray(values, dtype=np.float64))
    if dtype == "f64":
        return v, dtype
    r = round_to(dtype, v.reshape(-1, order="F")).reshape(v.shape, order="F")
    if dtype == "f32":
        return np.asfortranarray(r.astype(np.float32)), dtype
    if dtype == "f16":
        return np.asfortranarray(r.astype(np.float16).view(np.uint16)), dtype
    # bfloat16: the rounded value is exact in float32 with 16 zero low bits
    b = (r.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return np.asfortranarray(b), dtype


def fill(rows: int, cols: int, k: float, dtype: str = "f32"):
    """.fill(k) / ones / zeros: every element is k stored in the element type."""
    return _stored(np.full((rows, cols), float(k)), dtype)


def eye(rows: int, cols: int, dtype: str = "f32"):
    """eye(rows, cols): 1 where the row index equals the column index, else 0
    (a rectangular shape keeps the leading diagonal)."""
    r = np.arange(rows).reshape(-1, 1)
    c = np.arange(cols).reshape(1, -1)
    return _stored((r == c).astype(np.float64), dtype)


def linspace_values(start: float, end: float, n: int) -> np.ndarray:
    """linspace(start, end, n) in FP64: x_i = start + i * d for i < n - 1 with
    d = (end - start) / (n - 1), and the last element is end itself (the
    vector includes both end points; n = 1 gives end)."""
    if n <= 0:
        return np.zeros(0)
    x = np.empty(n)
    if n > 1:
        d = (float(end) - float(start)) / float(n - 1)
        i = np.arange(n - 1, dtype=np.float64)
        x[: n - 1] = float(start) + i * d
    x[n - 1] = float(end)
    return x


def linspace(start: float, end: float, n: int, dtype: str = "f64", row: bool = False):
    """linspace as an n x 1 column (or 1 x n row) operand stored in dtype."""
    x = linspace_values(start, end, n)
    return _stored(x.reshape(1, -1) if row else x.reshape(-1, 1), dtype)
