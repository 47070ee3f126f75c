"""ctypes binding of libcoot_mi355x.so (argument marshalling only).

Every function here packs its arguments into the C structs of
``include/coot.h`` and calls the entry point of the same name; all
computation happens in the library's HIP kernels.  torch tensors supply
device memory and the current HIP stream.

A matrix is a 2-D tensor in column-major layout, i.e. stride (1, ld), such
as ``torch.empty(n_cols, n_rows).t()``; a 1-D contiguous tensor is an n x 1
column.  Expression trees are sequences of nodes with ``op``, ``a``, ``b``,
``k`` (the op names below), or objects with a ``postfix()`` method.
"""
from __future__ import annotations

import collections
import ctypes as C
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoot_mi355x.so")
# run-time compiled kernels are cached next to the library unless told otherwise
os.environ.setdefault("COOT_CACHE_DIR", os.path.join(_HERE, "_kcache"))

# ---- codes (include/coot.h) ---------------------------------------------
OK = 0
ERRORS = {
    -1: "BAD_TREE", -2: "SHAPE", -3: "DTYPE", -4: "ALIAS", -5: "EMPTY", -6: "UNSUPPORTED",
    -7: "JIT", -8: "HIP", -9: "NOMEM", -10: "ARG", -11: "NOT_INIT", -12: "NOT_READY",
}
F32, F64, F16, BF16, U64, I32, U32 = 0, 1, 2, 3, 4, 5, 6
DTYPE_CODES = {"f32": F32, "f64": F64, "f16": F16, "bf16": BF16, "u64": U64, "i32": I32, "u32": U32}
OPS = {
    "leaf": 0, "plus": 1, "minus": 2, "schur": 3, "div": 4,
    "scal_plus": 10, "scal_minus_post": 11, "scal_minus_pre": 12, "scal_times": 13,
    "scal_div_post": 14, "scal_div_pre": 15,
    "exp": 20, "log": 21, "sqrt": 22, "abs": 23, "trans": 30, "conv": 31,
    "gt": 40, "lt": 41, "ge": 42, "le": 43, "eq": 44, "ne": 45,
    "scal_gt": 50, "scal_lt": 51, "scal_ge": 52, "scal_le": 53, "scal_eq": 54, "scal_ne": 55,
    "scal_pow": 16, "log10": 60, "log2": 61, "exp2": 62, "square": 63, "floor": 64, "ceil": 65, "round": 66,
    "trunc": 67, "sign": 68, "cos": 70, "sin": 71, "tan": 72, "acos": 73, "asin": 74, "atan": 75, "cosh": 76,
    "sinh": 77, "tanh": 78,
}
REDS = {
    "accu": 0, "sum": 1, "dot": 2, "norm1": 3, "norm2": 4, "norminf": 5, "normneginf": 6,
    "min": 7, "max": 8, "index_min": 9, "index_max": 10,
    "mean": 11, "var": 12, "stddev": 13, "count": 14, "all": 15, "any": 16,
}
U64_RESULTS = ("index_min", "index_max", "count", "all", "any")
RED_PAIRWISE = 0x100
OPERAND_HOST = 1
GEN_FILL, GEN_EYE, GEN_LINSPACE = 0x10, 0x20, 0x40
ITEMSIZE = {F32: 4, F64: 8, F16: 2, BF16: 2, U64: 8, I32: 4, U32: 4}
EXPR_UNFUSED = 1
PRINT_INFO = 1
TUNE_DEFAULT, TUNE_CACHE, TUNE_MODEL = 0, 1, 2
BATCH_NO_GRAPH, BATCH_PER_ITEM, BATCH_UNFUSED = 1, 2, 4
N_CONFIGS = 64
N_FEATURES = 32
MLP_N_PARAMS = 32 * 64 + 64 + 64 * 64 + 64


def mlp_ws_floats(B: int) -> int:
    return B * (64 + 64 + 64) + 64 + 8


class CootError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"coot error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code
        self.msg = msg


# ---- structs -------------------------------------------------------------
class Operand(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("n_rows", C.c_int64), ("n_cols", C.c_int64), ("ld", C.c_int64),
                ("dtype", C.c_int32), ("flags", C.c_uint32), ("gen", C.c_double * 2)]


class Node(C.Structure):
    _fields_ = [("op", C.c_int32), ("a", C.c_int32), ("b", C.c_int32), ("reserved", C.c_int32), ("k", C.c_double)]


class Config(C.Structure):
    _fields_ = [("ept", C.c_int32), ("block", C.c_int32), ("split", C.c_int32), ("reserved", C.c_int32)]


class Expr(C.Structure):
    _fields_ = [("nodes", C.POINTER(Node)), ("n_nodes", C.c_int32), ("flags", C.c_uint32), ("cfg", Config)]


class Batch(C.Structure):
    _fields_ = [("expr", C.POINTER(Expr)), ("n_slots", C.c_int32), ("n_items", C.c_int32),
                ("slot_dtypes", C.POINTER(C.c_int32)), ("leaf_ptrs", C.POINTER(C.c_void_p)),
                ("out_ptrs", C.POINTER(C.c_void_p)), ("out_dtype", C.c_int32), ("red_op", C.c_int32),
                ("shapes", C.POINTER(C.c_int64)), ("red_expr", C.POINTER(Expr)), ("red_out", C.c_void_p),
                ("red_dtype", C.c_int32), ("flags", C.c_uint32)]


class Stats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("jit_compiles", C.c_int64), ("jit_disk_hits", C.c_int64),
                ("jit_mem_hits", C.c_int64), ("jit_seconds", C.c_double)]


# ---- library -------------------------------------------------------------
_lib = None

EXPORTS = [
    "coot_init", "coot_finalize", "coot_eval", "coot_reduce", "coot_synchronise", "coot_last_error",
    "coot_validate", "coot_kernel_source", "coot_precompile", "coot_batch_create", "coot_batch_run",
    "coot_batch_destroy", "coot_config_of", "coot_set_tuning", "coot_features", "coot_autotune",
    "coot_mlp_forward", "coot_mlp_backward", "coot_mlp_adam", "coot_model_set", "coot_model_choose",
    "coot_get_stats", "coot_copy", "coot_precompile_begin", "coot_precompile_end",
    "coot_default_config", "coot_batch_kernel_source", "coot_eval_batched", "coot_bandwidth_probe",
    "coot_kernel_stamp",
]


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2308_03120_amd.build.build() "
                              "(there is no CPU fallback)")
        # The library and torch must share one HIP runtime (the binding passes
        # torch's streams and memory): load torch's first, so that the
        # library's libamdhip64.so.7 dependency resolves to it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        L.coot_init.argtypes = [i32, C.c_uint]
        L.coot_eval.argtypes = [P(Expr), P(Operand), i32, P(Operand), vp]
        L.coot_reduce.argtypes = [i32, i32, P(Expr), P(Operand), i32, P(Operand), vp]
        L.coot_reduce_noalloc.argtypes = [i32, i32, P(Expr), P(Operand), i32, P(Operand), vp]
        L.coot_synchronise.argtypes = [vp]
        L.coot_last_error.restype = C.c_char_p
        L.coot_validate.argtypes = [i32, i32, P(Expr), P(Operand), i32, P(Operand)]
        L.coot_kernel_source.argtypes = [i32, i32, P(Expr), P(Operand), i32, P(Operand), C.c_char_p, i64]
        L.coot_kernel_source.restype = i64
        L.coot_precompile.argtypes = [i32, i32, P(Expr), P(Operand), i32, P(Operand)]
        L.coot_batch_create.argtypes = [P(Batch), vp, P(vp)]
        L.coot_batch_run.argtypes = [vp, vp]
        L.coot_batch_kernel_source.argtypes = [P(Batch), C.c_char_p, i64]
        L.coot_batch_kernel_source.restype = i64
        L.coot_batch_destroy.argtypes = [vp]
        L.coot_eval_batched.argtypes = [P(Batch), vp]
        L.coot_config_of.argtypes = [i32, P(Config)]
        L.coot_set_tuning.argtypes = [i32, C.c_char_p]
        L.coot_features.argtypes = [i32, i32, P(Expr), P(Operand), i32, P(Operand), P(C.c_float)]
        L.coot_autotune.argtypes = [i32, i32, P(Expr), P(Operand), i32, P(Operand), i32, P(C.c_float), vp]
        fp = P(C.c_float)
        L.coot_mlp_forward.argtypes = [vp, vp, i32, vp, vp, vp]
        L.coot_mlp_backward.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp]
        L.coot_mlp_adam.argtypes = [vp, vp, vp, vp, i32, i32, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.coot_model_set.argtypes = [fp, fp, fp]
        L.coot_model_choose.argtypes = [i32, i32, P(Expr), P(Operand), i32, P(Operand)]
        L.coot_get_stats.argtypes = [P(Stats)]
        L.coot_copy.argtypes = [vp, vp, i64, vp]
        L.coot_bandwidth_probe.argtypes = [i32, vp, vp, i64, vp]
        L.coot_kernel_stamp.argtypes = [P(C.c_uint64)]
        L.coot_precompile_end.argtypes = [i32]
        L.coot_default_config.argtypes = [i32, i32, P(Expr), P(Operand), i32, P(Operand)]
        _lib = L
    return _lib


def last_error() -> str:
    return lib().coot_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise CootError(rc, last_error())
    return rc


# ---- marshalling ---------------------------------------------------------
def _torch():
    import torch

    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    m = {torch.float32: F32, torch.float64: F64, torch.float16: F16, torch.bfloat16: BF16, torch.int64: U64,
         torch.int32: I32, torch.uint32: U32}
    if t.dtype not in m:
        raise TypeError(f"unsupported tensor dtype {t.dtype}")
    return m[t.dtype]


def operand(t, host: bool = False) -> Operand:
    """Column-major operand view of a tensor (1-D -> n x 1; 2-D with stride (1, ld))."""
    if isinstance(t, Operand):
        return t
    if t.dim() == 1:
        if t.numel() > 1 and t.stride(0) != 1:
            raise ValueError("1-D operands must be contiguous")
        r, c, ld = t.shape[0], 1, max(1, t.shape[0])
    elif t.dim() == 2:
        r, c = t.shape
        if r > 1 and t.stride(0) != 1:
            raise ValueError("2-D operands must be column-major (stride (1, ld)), e.g. torch.empty(c, r).t()")
        ld = t.stride(1) if c > 1 else max(1, r)
        if r == 1 and c > 1:
            ld = t.stride(1)
    else:
        raise ValueError("operands are vectors or matrices")
    return Operand(t.data_ptr(), r, c, ld, _dtype_code(t), OPERAND_HOST if host else 0)


def fake_operand(n_rows: int, n_cols: int, dtype: str = "f32", ld: Optional[int] = None,
                 ptr: int = 0x100000, flags: int = 0) -> Operand:
    """Operand descriptor without memory, for the host-only calls."""
    return Operand(ptr, n_rows, n_cols, ld if ld is not None else max(1, n_rows), DTYPE_CODES[dtype], flags)


# ---- generators and views (Table 1, Table 4) --------------------------------
def _gen(rows: int, cols: int, dtype: str, flag: int, g0: float = 0.0, g1: float = 0.0) -> Operand:
    o = Operand(None, int(rows), int(cols), max(1, int(rows)), DTYPE_CODES[dtype], flag)
    o.gen[0] = float(g0)
    o.gen[1] = float(g1)
    return o


def fill(rows: int, cols: int, k: float, dtype: str = "f32") -> Operand:
    """Memory-free operand with every element k (stored once in dtype)."""
    return _gen(rows, cols, dtype, GEN_FILL, k)


def ones(rows: int, cols: int, dtype: str = "f32") -> Operand:
    return fill(rows, cols, 1.0, dtype)


def zeros(rows: int, cols: int, dtype: str = "f32") -> Operand:
    return fill(rows, cols, 0.0, dtype)


def eye(rows: int, cols: int, dtype: str = "f32") -> Operand:
    """Memory-free operand: 1 where row == column, else 0."""
    return _gen(rows, cols, dtype, GEN_EYE)


def linspace(start: float, end: float, n: int, dtype: str = "f64", row: bool = False) -> Operand:
    """Memory-free n x 1 (or 1 x n) vector from start to end inclusive."""
    return _gen(1 if row else n, n if row else 1, dtype, GEN_LINSPACE, start, end)


def _view(base: Operand, off: int, rows: int, cols: int, ld: int) -> Operand:
    ptr = (base.ptr or 0) + off * ITEMSIZE[base.dtype]
    return Operand(ptr if rows * cols > 0 else (base.ptr or None), rows, cols, ld, base.dtype, 0)


def submat(t, p: int, q: int, r: int, s: int) -> Operand:
    """.submat(p, q, r, s): rows p..r and columns q..s (inclusive) of t."""
    b = operand(t)
    if not (0 <= p <= r + 1 and r < b.n_rows and 0 <= q <= s + 1 and s < b.n_cols):
        raise ValueError(f"submat({p}, {q}, {r}, {s}) outside {b.n_rows} x {b.n_cols}")
    return _view(b, p + q * b.ld, r - p + 1, s - q + 1, b.ld)


def rows(t, a: int, b: int) -> Operand:
    o = operand(t)
    return submat(o, a, 0, b, o.n_cols - 1)


def cols(t, c: int, d: int) -> Operand:
    o = operand(t)
    return submat(o, 0, c, o.n_rows - 1, d)


def row(t, i: int) -> Operand:
    return rows(t, i, i)


def col(t, j: int) -> Operand:
    return cols(t, j, j)


def diag(t, k: int = 0) -> Operand:
    """.diag(k): the k-th diagonal of t as a 1 x n operand with ld + 1."""
    b = operand(t)
    r0, c0 = max(-k, 0), max(k, 0)
    n = max(0, min(b.n_rows - r0, b.n_cols - c0))
    return _view(b, r0 + c0 * b.ld, 1, n, b.ld + 1)


def trace(t, out=None, stream=None):
    """trace(A): sum of the leading diagonal (Table 5)."""
    return reduce("accu", [("leaf", 0, -1, 0.0)], [diag(t)], out=out, stream=stream)


def diagvec(t, out, k: int = 0, stream=None) -> None:
    """diagvec(A, k): the k-th diagonal as an n x 1 column, written to out (Table 6)."""
    eval([("leaf", 0, -1, 0.0), ("trans", 0, -1, 0.0)], [diag(t, k)], out, stream=stream)


# Converted node arrays of recently used tree objects (trees are immutable once
# built).  The entry holds the tree itself, so its id cannot be reused while
# cached.
_NODE_CACHE: "collections.OrderedDict[int, tuple]" = collections.OrderedDict()
_NODE_CACHE_MAX = 512


def _nodes(tree):
    if hasattr(tree, "postfix"):
        hit = _NODE_CACHE.get(id(tree))
        if hit is not None and hit[0] is tree:
            _NODE_CACHE.move_to_end(id(tree))
            return hit[1]
        arr = _convert(tree.postfix())
        _NODE_CACHE[id(tree)] = (tree, arr)
        if len(_NODE_CACHE) > _NODE_CACHE_MAX:
            _NODE_CACHE.popitem(last=False)
        return arr
    return _convert(tree)


def _convert(tree):
    arr = (Node * len(tree))()
    for i, n in enumerate(tree):
        if isinstance(n, (tuple, list)):
            op, a, b, k = (list(n) + [-1, -1, 0.0])[:4]
        else:
            op, a, b, k = n.op, n.a, n.b, n.k
        arr[i].op = OPS[op] if isinstance(op, str) else int(op)
        arr[i].a = int(a)
        arr[i].b = int(b)
        arr[i].k = float(k)
    return arr


def expr(tree, cfg=None, unfused: bool = False):
    """coot_expr for a tree; keeps the node array alive on the returned object."""
    nodes = _nodes(tree)
    e = Expr()
    e.nodes = C.cast(nodes, C.POINTER(Node))
    e.n_nodes = len(nodes)
    e.flags = EXPR_UNFUSED if unfused else 0
    if cfg is not None:
        if isinstance(cfg, int):
            cc = Config()
            _check(lib().coot_config_of(cfg, C.byref(cc)))
            cfg = (cc.ept, cc.block, cc.split)
        e.cfg = Config(cfg[0], cfg[1], cfg[2], 0)
    e._keep = nodes
    return e


def _ops(operands: Sequence):
    arr = (Operand * max(1, len(operands)))()
    for i, t in enumerate(operands):
        arr[i] = operand(t)
    return arr, len(operands)


def current_stream():
    torch = _torch()
    if torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


def _red_code(op, pairwise: bool) -> int:
    c = REDS[op] if isinstance(op, str) else int(op)
    return c | (RED_PAIRWISE if pairwise else 0)


# ---- entry points --------------------------------------------------------
def init(device: int = 0, print_info: bool = False) -> None:
    _check(lib().coot_init(device, PRINT_INFO if print_info else 0))


def finalize() -> None:
    _check(lib().coot_finalize())


def eval(tree, operands: Sequence, out, cfg=None, unfused: bool = False, stream=None):
    """out = value of the tree (fused into one kernel unless unfused=True)."""
    e = expr(tree, cfg, unfused)
    arr, n = _ops(operands)
    o = operand(out)
    _check(lib().coot_eval(C.byref(e), arr, n, C.byref(o), stream if stream is not None else current_stream()))
    return out


def reduce(op, tree, operands: Sequence, out=None, dim: int = -1, pairwise: bool = False, cfg=None,
           unfused: bool = False, out_dtype=None, stream=None):
    """Reduction of the tree's value.  Allocates ``out`` on the device if not given
    (float32/float64 by the tree's precision; int64 for indices, counts, all and any)."""
    torch = _torch()
    e = expr(tree, cfg, unfused)
    arr, n = _ops(operands)
    if out is None:
        opname = op if isinstance(op, str) else {v: k for k, v in REDS.items()}[op]
        rows, cols, prec = _root_shape(tree, operands)
        n_out = 1 if dim < 0 else (cols if dim == 0 else rows)
        if opname in U64_RESULTS:
            dt = torch.int64
        else:
            dt = out_dtype or (torch.float64 if prec == 64 else torch.float32)
        dev = next((t.device for t in operands if hasattr(t, "device")), "cuda")
        out = torch.empty(n_out, dtype=dt, device=dev)
    o = operand(out)
    _check(lib().coot_reduce(_red_code(op, pairwise), dim, C.byref(e), arr, n, C.byref(o),
                             stream if stream is not None else current_stream()))
    return out


def reduce_noalloc(op, tree, operands: Sequence, out, dim: int = -1, pairwise: bool = False, cfg=None,
                   stream=None):
    """coot_reduce_noalloc: ``reduce`` into a caller-given device ``out`` with no
    device allocation (partials in the library's static scratch array)."""
    e = expr(tree, cfg, False)
    arr, n = _ops(operands)
    o = operand(out)
    _check(lib().coot_reduce_noalloc(_red_code(op, pairwise), dim, C.byref(e), arr, n, C.byref(o),
                                     stream if stream is not None else current_stream()))
    return out


def _root_shape(tree, operands):
    """Shape and precision of the tree's value (host-side bookkeeping for allocation)."""
    nodes = tree.postfix() if hasattr(tree, "postfix") else tree
    info = []
    for n in nodes:
        op, a, b = (n.op, n.a, n.b) if not isinstance(n, (tuple, list)) else (n[0], n[1], n[2])
        if op == "leaf" or op == 0:
            o = operand(operands[a])
            info.append((o.n_rows, o.n_cols, 64 if o.dtype in (F64, I32, U32) else 32))
        elif op in ("trans", 30):
            r, c, p = info[a]
            info.append((c, r, p))
        elif op in ("conv", 31):
            r, c, p = info[a]
            info.append((r, c, 64 if b in (F64, I32, U32) else 32))
        else:
            info.append(info[a])
    return info[-1]


def synchronise(stream=None) -> None:
    _check(lib().coot_synchronise(stream if stream is not None else current_stream()))


def validate(red_op, dim, tree, operands: Sequence, out) -> int:
    """Host-only argument checks; returns 0 or raises CootError."""
    e = expr(tree)
    arr, n = _ops(operands)
    o = operand(out)
    rc = -1 if red_op is None else _red_code(red_op, False)
    return _check(lib().coot_validate(rc, dim, C.byref(e), arr, n, C.byref(o)))


def kernel_source(red_op, dim, tree, operands: Sequence, out, cfg=None, pairwise: bool = False) -> str:
    e = expr(tree, cfg)
    arr, n = _ops(operands)
    o = operand(out)
    rc = -1 if red_op is None else _red_code(red_op, pairwise)
    size = _check(lib().coot_kernel_source(rc, dim, C.byref(e), arr, n, C.byref(o), None, 0))
    buf = C.create_string_buffer(size + 1)
    _check(lib().coot_kernel_source(rc, dim, C.byref(e), arr, n, C.byref(o), buf, size + 1))
    return buf.value.decode()


def precompile(red_op, dim, tree, operands: Sequence, out, cfg=None, pairwise: bool = False) -> int:
    e = expr(tree, cfg)
    arr, n = _ops(operands)
    o = operand(out)
    rc = -1 if red_op is None else _red_code(red_op, pairwise)
    return _check(lib().coot_precompile(rc, dim, C.byref(e), arr, n, C.byref(o)))


def precompile_begin() -> None:
    _check(lib().coot_precompile_begin())


def precompile_end(kernels_per_module: int = 64) -> int:
    return _check(lib().coot_precompile_end(kernels_per_module))


def features(red_op, dim, tree, operands: Sequence, out):
    import numpy as np

    e = expr(tree)
    arr, n = _ops(operands)
    o = operand(out)
    f = np.zeros(N_FEATURES, np.float32)
    rc = -1 if red_op is None else _red_code(red_op, False)
    _check(lib().coot_features(rc, dim, C.byref(e), arr, n, C.byref(o), f.ctypes.data_as(C.POINTER(C.c_float))))
    return f


def autotune(red_op, dim, tree, operands: Sequence, out, reps: int = 5, stream=None):
    """Time all 64 configurations; returns (best index, times in ms)."""
    import numpy as np

    e = expr(tree)
    arr, n = _ops(operands)
    o = operand(out)
    t = np.zeros(N_CONFIGS, np.float32)
    rc = -1 if red_op is None else _red_code(red_op, False)
    best = _check(lib().coot_autotune(rc, dim, C.byref(e), arr, n, C.byref(o), reps,
                                      t.ctypes.data_as(C.POINTER(C.c_float)),
                                      stream if stream is not None else current_stream()))
    return best, t


def default_config(red_op, dim, tree, operands: Sequence, out) -> int:
    e = expr(tree)
    arr, n = _ops(operands)
    o = operand(out)
    rc = -1 if red_op is None else _red_code(red_op, False)
    return _check(lib().coot_default_config(rc, dim, C.byref(e), arr, n, C.byref(o)))


def config_of(index: int):
    c = Config()
    _check(lib().coot_config_of(index, C.byref(c)))
    return (c.ept, c.block, c.split)


def set_tuning(mode: int, model_path: Optional[str] = None) -> None:
    _check(lib().coot_set_tuning(mode, model_path.encode() if model_path else None))


def kernel_stamp():
    """(feature schema, kernel stamp) of the library (coot_kernel_stamp)."""
    st = C.c_uint64()
    schema = _check(lib().coot_kernel_stamp(C.byref(st)))
    return schema, st.value


def model_set(params, mean, std) -> None:
    import numpy as np

    p = np.ascontiguousarray(params, np.float32)
    m = np.ascontiguousarray(mean, np.float32)
    s = np.ascontiguousarray(std, np.float32)
    fp = C.POINTER(C.c_float)
    _check(lib().coot_model_set(p.ctypes.data_as(fp), m.ctypes.data_as(fp), s.ctypes.data_as(fp)))


def model_choose(red_op, dim, tree, operands: Sequence, out) -> int:
    e = expr(tree)
    arr, n = _ops(operands)
    o = operand(out)
    rc = -1 if red_op is None else _red_code(red_op, False)
    return _check(lib().coot_model_choose(rc, dim, C.byref(e), arr, n, C.byref(o)))


def mlp_forward(params, X, Y, ws=None, stream=None) -> None:
    B = X.shape[0]
    _check(lib().coot_mlp_forward(params.data_ptr(), X.data_ptr(), B, Y.data_ptr(),
                                  ws.data_ptr() if ws is not None else None,
                                  stream if stream is not None else current_stream()))


def mlp_backward(params, X, T, M, grad, loss, ws, stream=None) -> None:
    B = X.shape[0]
    _check(lib().coot_mlp_backward(params.data_ptr(), X.data_ptr(), T.data_ptr(), M.data_ptr(), B,
                                   grad.data_ptr(), loss.data_ptr() if loss is not None else None, ws.data_ptr(),
                                   stream if stream is not None else current_stream()))


def mlp_adam(params, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None) -> None:
    _check(lib().coot_mlp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), params.numel(), t,
                               lr, beta1, beta2, eps, stream if stream is not None else current_stream()))


def copy(dst, src, nbytes: Optional[int] = None, stream=None) -> None:
    n = nbytes if nbytes is not None else src.numel() * src.element_size()
    _check(lib().coot_copy(dst.data_ptr(), src.data_ptr(), n, stream if stream is not None else current_stream()))


PROBE_COPY, PROBE_READ, PROBE_WRITE, PROBE_READ2_WRITE1 = 0, 1, 2, 3
PROBE_TILED_COPY, PROBE_TILED_READ2_WRITE1 = 4, 5


def bandwidth_probe(kind: int, dst, src, nbytes: int, stream=None) -> None:
    """Streaming probe of a read/write mix (coot_bandwidth_probe)."""
    _check(lib().coot_bandwidth_probe(kind, dst.data_ptr() if dst is not None else None,
                                      src.data_ptr() if src is not None else None, nbytes,
                                      stream if stream is not None else current_stream()))


def stats() -> dict:
    s = Stats()
    _check(lib().coot_get_stats(C.byref(s)))
    return {k: getattr(s, k) for k, _ in Stats._fields_}


# ---- batched evaluation ---------------------------------------------------
class BatchDescriptor:
    """A marshalled coot_batch (see coot.h): one tree over many matrices."""

    def __init__(self, tree, slot_dtypes, leaf_ptrs, shapes, out_ptrs=None, out_dtype=F32, red_tree=None,
                 red_op="accu", red_out=None, red_dtype=F32, flags=0, split=None):
        import numpy as np

        # split: 4*split blocks per CU for the tile pass (None: library default)
        self._e = expr(tree, None if split is None else (1, 256, split))
        self._re = expr(red_tree) if red_tree is not None else None
        n_items = len(shapes)
        n_slots = len(slot_dtypes)
        self._sd = (C.c_int32 * n_slots)(*slot_dtypes)
        lp = np.ascontiguousarray(np.asarray(leaf_ptrs, dtype=np.uint64).reshape(-1))
        self._lp = (C.c_void_p * lp.size)(*[int(x) for x in lp])
        self._op = None
        if out_ptrs is not None:
            self._op = (C.c_void_p * n_items)(*[int(x) for x in out_ptrs])
        sh = np.ascontiguousarray(np.asarray(shapes, dtype=np.int64).reshape(-1))
        self._sh = (C.c_int64 * sh.size)(*[int(x) for x in sh])
        red_out_ptr = red_out if (red_out is None or isinstance(red_out, int)) else red_out.data_ptr()
        b = Batch()
        b.expr = C.pointer(self._e)
        b.n_slots = n_slots
        b.n_items = n_items
        b.slot_dtypes = C.cast(self._sd, C.POINTER(C.c_int32))
        b.leaf_ptrs = C.cast(self._lp, C.POINTER(C.c_void_p))
        b.out_ptrs = C.cast(self._op, C.POINTER(C.c_void_p)) if self._op is not None else None
        b.out_dtype = out_dtype
        b.red_op = _red_code(red_op, False)
        b.shapes = C.cast(self._sh, C.POINTER(C.c_int64))
        b.red_expr = C.pointer(self._re) if self._re is not None else None
        b.red_out = red_out_ptr
        b.red_dtype = red_dtype
        b.flags = flags
        self.struct = b


def eval_batched(desc: BatchDescriptor, stream=None) -> None:
    """coot_eval_batched: build (first call) or replay the batch's launch."""
    _check(lib().coot_eval_batched(C.byref(desc.struct), stream if stream is not None else current_stream()))


class BatchPlan:
    """One persistent launch for many matrices (see coot_batch in coot.h)."""

    def __init__(self, tree, slot_dtypes, leaf_ptrs, shapes, out_ptrs=None, out_dtype=F32, red_tree=None,
                 red_op="accu", red_out=None, red_dtype=F32, flags=0, stream=None, split=None):
        self.handle = C.c_void_p()
        self.desc = BatchDescriptor(tree, slot_dtypes, leaf_ptrs, shapes, out_ptrs, out_dtype, red_tree, red_op,
                                    red_out, red_dtype, flags, split)
        _check(lib().coot_batch_create(C.byref(self.desc.struct), stream if stream is not None else current_stream(),
                                       C.byref(self.handle)))

    @staticmethod
    def kernel_source(tree, slot_dtypes, shapes, out=True, out_dtype=F32, red_tree=None, red_op="accu",
                      red_dtype=F32) -> str:
        """Host only: the HIP source of the batched kernels (pointers are placeholders)."""
        G = 1 << 40
        n = len(shapes)
        d = BatchDescriptor(tree, slot_dtypes, [[G * (s + 1) for s in range(len(slot_dtypes))]] * n, shapes,
                            [G * 9] * n if out else None, out_dtype, red_tree, red_op,
                            G * 10 if red_tree is not None else None, red_dtype, 0, None)
        size = _check(lib().coot_batch_kernel_source(C.byref(d.struct), None, 0))
        buf = C.create_string_buffer(size + 1)
        _check(lib().coot_batch_kernel_source(C.byref(d.struct), buf, size + 1))
        return buf.value.decode()

    def run(self, stream=None) -> None:
        _check(lib().coot_batch_run(self.handle, stream if stream is not None else current_stream()))

    def close(self) -> None:
        if self.handle:
            _check(lib().coot_batch_destroy(self.handle))
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
