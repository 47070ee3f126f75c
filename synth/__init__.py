"""Seeded synthetic inputs and expression-tree structures.

This module is shared by the test oracle and by the GPU path; it therefore
holds *no* arithmetic of the method itself (no element-wise evaluation, no
reductions, no type conversion of its own).  It only

  * draws seeded random numbers (numpy ``default_rng``),
  * stores them in the storage element type through library conversions
    (numpy ``astype`` for float32/float16, torch's CPU ``to(bfloat16)``),
  * describes expression trees as plain data.

Matrices follow the paper's storage rule (Section 2, Table 1): elements are
laid out column by column.  A matrix is a ``Mat`` whose ``data`` is a numpy
array of shape (n_rows, n_cols) in Fortran (column-major) order; 16-bit
types are carried as their raw ``uint16`` bit patterns.

Expression trees (Section 7: ``Op``/``eOp``/``eGlue``/``mtOp`` nodes) are
written with the small builder below and flattened to a post-order list of
``Node(op, a, b, k)`` records, where ``a``/``b`` index earlier nodes (or, for
a ``leaf``, ``a`` is an operand slot).  Each side (the oracle and the C-ABI
binding) maps the op *names* onto its own codes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

SEED_ROOT = (2308, 3120)

DTYPES = ("f32", "f64", "f16", "bf16")
ITEMSIZE = {"f32": 4, "f64": 8, "f16": 2, "bf16": 2, "u64": 8}


def rng(cfg: int, operand: int) -> np.random.Generator:
    """Generator for operand ``operand`` of workload ``cfg`` (independent streams)."""
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT[0], SEED_ROOT[1], cfg, operand]))


# ----------------------------------------------------------------------------
# storage
# ----------------------------------------------------------------------------
@dataclass
class Mat:
    data: np.ndarray  # (n_rows, n_cols), Fortran order; uint16 bits for f16/bf16
    dtype: str

    @property
    def shape(self) -> Tuple[int, int]:
        return (int(self.data.shape[0]), int(self.data.shape[1]))

    @property
    def n_elem(self) -> int:
        return int(self.data.shape[0]) * int(self.data.shape[1])

    def flat(self) -> np.ndarray:
        """Storage in memory order (column-major)."""
        return self.data.reshape(-1, order="F")


def store(draws: np.ndarray, dtype: str) -> np.ndarray:
    """Store FP64 draws in ``dtype`` with a library round-to-nearest-even.

    float16 rounds directly from float64 (numpy); bfloat16 goes through
    torch's float32 -> bfloat16 conversion (float64 -> float32 -> bfloat16).
    Whatever the rounding path, both sides read the same stored bits.
    """
    order = "F" if draws.ndim == 2 else "C"
    if dtype == "f64":
        return np.asarray(draws, dtype=np.float64, order=order)
    if dtype == "f32":
        return np.asarray(draws.astype(np.float32), order=order)
    if dtype == "f16":
        return np.asarray(draws.astype(np.float16).view(np.uint16), order=order)
    if dtype == "bf16":
        import torch

        flat = np.ascontiguousarray(draws.reshape(-1, order="F") if draws.ndim == 2 else draws)
        t = torch.from_numpy(flat.astype(np.float32)).to(torch.bfloat16)
        bits = t.view(torch.int16).numpy().view(np.uint16)
        if draws.ndim == 2:
            return np.asarray(bits.reshape(draws.shape, order="F"), order="F")
        return bits.copy()
    if dtype in ("i32", "u32"):
        # integer draws only (the test inputs are integer-valued): stored exactly
        info = np.iinfo(np.int32 if dtype == "i32" else np.uint32)
        if not (np.all(draws == np.round(draws)) and np.all(draws >= info.min) and np.all(draws <= info.max)):
            raise ValueError(f"{dtype} storage takes integer draws within range")
        return np.asarray(draws.astype(np.int32 if dtype == "i32" else np.uint32), order=order)
    raise ValueError(dtype)


def mat_from_draws(draws_flat: np.ndarray, n_rows: int, n_cols: int, dtype: str) -> Mat:
    """Column-major matrix from a flat vector of draws (draw k -> linear index k)."""
    m = draws_flat.reshape((n_rows, n_cols), order="F")
    return Mat(store(m, dtype), dtype)


# ----------------------------------------------------------------------------
# expression trees (structure only)
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Node:
    op: str
    a: int = -1
    b: int = -1
    k: float = 0.0


UNARY = ("exp", "log", "sqrt", "abs", "trans")
BINARY = ("plus", "minus", "schur", "div")
SCALAR = ("scal_plus", "scal_minus_post", "scal_minus_pre", "scal_times",
          "scal_div_post", "scal_div_pre")
ALL_OPS = ("leaf",) + BINARY + SCALAR + UNARY + ("conv",)
CONV_TARGET = {"f32": 0, "f64": 1, "f16": 2, "bf16": 3, "i32": 5, "u32": 6}


class E:
    """Tiny expression builder mirroring the paper's operator overloads
    (Table 2: ``A+k``, ``k-A``, ``A%B``, ``A/B``...; Table 7: ``trans``, ``exp``...)."""

    __slots__ = ("op", "kids", "k", "slot")

    def __init__(self, op: str, kids: Sequence["E"] = (), k: float = 0.0, slot: int = -1):
        self.op, self.kids, self.k, self.slot = op, tuple(kids), float(k), slot

    # binary element-wise / scalar forms
    def __add__(self, o):
        return E("plus", (self, o)) if isinstance(o, E) else E("scal_plus", (self,), o)

    def __radd__(self, o):
        return E("scal_plus", (self,), o)

    def __sub__(self, o):
        return E("minus", (self, o)) if isinstance(o, E) else E("scal_minus_post", (self,), o)

    def __rsub__(self, o):
        return E("scal_minus_pre", (self,), o)

    def __mul__(self, o):
        if isinstance(o, E):
            raise TypeError("matrix multiplication is not an element-wise operation")
        return E("scal_times", (self,), o)

    def __rmul__(self, o):
        return E("scal_times", (self,), o)

    def __mod__(self, o):
        return E("schur", (self, o))

    def __truediv__(self, o):
        return E("div", (self, o)) if isinstance(o, E) else E("scal_div_post", (self,), o)

    def __rtruediv__(self, o):
        return E("scal_div_pre", (self,), o)

    # relational expressions (1 where true, else 0): A < x, A > B ... (Table 5,
    # Section 3's counting example).  k > A is A < k.  == and != are the
    # functions eq() and ne(), so that trees keep ordinary identity comparison.
    def __gt__(self, o):
        return E("gt", (self, o)) if isinstance(o, E) else E("scal_gt", (self,), o)

    def __lt__(self, o):
        return E("lt", (self, o)) if isinstance(o, E) else E("scal_lt", (self,), o)

    def __ge__(self, o):
        return E("ge", (self, o)) if isinstance(o, E) else E("scal_ge", (self,), o)

    def __le__(self, o):
        return E("le", (self, o)) if isinstance(o, E) else E("scal_le", (self,), o)

    __hash__ = object.__hash__

    def t(self):
        return E("trans", (self,))

    def postfix(self) -> List[Node]:
        out: List[Node] = []

        def walk(e: E) -> int:
            if e.op == "leaf":
                out.append(Node("leaf", e.slot))
                return len(out) - 1
            idx = [walk(c) for c in e.kids]
            a = idx[0]
            b = idx[1] if len(idx) > 1 else -1
            if e.op == "conv":
                b = e.slot
            out.append(Node(e.op, a, b, e.k))
            return len(out) - 1

        walk(self)
        return out


def leaf(slot: int) -> E:
    return E("leaf", slot=slot)


def leaves(n: int) -> List[E]:
    return [leaf(i) for i in range(n)]


def exp(x: E) -> E:
    return E("exp", (x,))


def log(x: E) -> E:
    return E("log", (x,))


def sqrt(x: E) -> E:
    return E("sqrt", (x,))


def abs_(x: E) -> E:
    return E("abs", (x,))


def trans(x: E) -> E:
    return E("trans", (x,))


# misc and trig functions (Table 7)
def pow_(x: E, k: float) -> E:
    return E("scal_pow", (x,), k)


def _unary(name):
    def f(x: E) -> E:
        return E(name, (x,))

    f.__name__ = name
    return f


log10, log2, exp2, square, floor, ceil, round_, trunc, sign = (
    _unary(n) for n in ("log10", "log2", "exp2", "square", "floor", "ceil", "round", "trunc", "sign"))
cos, sin, tan, acos, asin, atan, cosh, sinh, tanh = (
    _unary(n) for n in ("cos", "sin", "tan", "acos", "asin", "atan", "cosh", "sinh", "tanh"))


def eq(a: E, b) -> E:
    """1 where a == b (b a tree or a scalar), else 0"""
    return E("eq", (a, b)) if isinstance(b, E) else E("scal_eq", (a,), b)


def ne(a: E, b) -> E:
    """1 where a != b (b a tree or a scalar), else 0"""
    return E("ne", (a, b)) if isinstance(b, E) else E("scal_ne", (a,), b)


def conv(x: E, dtype: str) -> E:
    return E("conv", (x,), slot=CONV_TARGET[dtype])


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def cfg1_inputs(n_rows: int = 1000, n_cols: int = 1000) -> Dict[str, Mat]:
    """Small plain method: A, B, C ~ U[-1,1], D ~ U[-4,4], FP32, column-major."""
    n = n_rows * n_cols
    out = {}
    for i, (name, lo, hi) in enumerate((("A", -1, 1), ("B", -1, 1), ("C", -1, 1), ("D", -4, 4))):
        d = rng(1, i).uniform(lo, hi, n)
        out[name] = mat_from_draws(d, n_rows, n_cols, "f32")
    return out


def cfg1_trees():
    A, B, C, D = leaves(4)
    return {
        "Y": 2.5 * A + B % C - exp(D),     # slots A,B,C,D
        "accu_AB": A % B,                    # slots A,B
        "sumA": A,                           # slot A
        "absB": abs_(B),                     # slot B (slot index 1 in the A,B,C,D operand list)
    }


def cfg2_inputs(dtype: str, n: int = 1 << 28, n_ties: int = 64) -> Dict[str, np.ndarray]:
    """Plain method at scale: x, y ~ N(0,1) (FP64 draws; FP32 is their RNE).

    ``n_ties`` distinct positions of x (sampled without replacement) are set
    to 8.0 after checking that the natural maximum is below 8.
    Returns vectors (1-D, storage dtype) and the sorted tie positions.
    """
    x = rng(2, 0).standard_normal(n)
    y = rng(2, 1).standard_normal(n)
    ties = np.sort(rng(2, 2).choice(n, size=min(n_ties, n), replace=False)) if n_ties else np.zeros(0, np.int64)
    if n_ties:
        assert float(np.max(x)) < 8.0
        x[ties] = 8.0
    return {"x": store(x, dtype), "y": store(y, dtype), "ties": ties.astype(np.int64)}


def cfg2_trees():
    x, y = leaves(2)
    return {
        "axpy": y + 0.75 * x,                               # y = y + 0.75*x (in place)
        "z": sqrt(abs_(x)) % y - x / (1 + abs_(y)),
        "dot": x % y,
        "x": x,
    }


FP16_CLIP = math.log(1e4) / 3.0  # |z| clip so |x| = exp(3 z) stays in [1e-4, 1e4]


def cfg3_inputs(dtype: str, n_rows: int = 16384, n_cols: int = 16384) -> Dict[str, Mat]:
    """Precision: |x| = exp(3 z), z ~ N(0,1) clipped to +-ln(1e4)/3, random signs."""
    out = {}
    n = n_rows * n_cols
    for i, name in enumerate(("A", "B")):
        g = rng(3, i)
        z = np.clip(g.standard_normal(n), -FP16_CLIP, FP16_CLIP)
        s = np.where(g.integers(0, 2, n) == 1, 1.0, -1.0)
        d = s * np.exp(3.0 * z)
        out[name] = mat_from_draws(d, n_rows, n_cols, dtype)
    return out


def cfg4_shapes(count: int = 10000, lo: int = 8, hi: int = 512) -> np.ndarray:
    """(count, 2) int64 of (rows, cols), each independently log-uniform in [lo, hi]."""
    g = rng(4, 0)
    u = g.uniform(math.log(lo), math.log(hi), (count, 2))
    return np.clip(np.rint(np.exp(u)), lo, hi).astype(np.int64)


def cfg4_inputs(count: int = 10000, lo: int = 8, hi: int = 512, align: int = 64):
    """Batching: A_i (r_i x c_i) and Bp_i (c_i x r_i) ~ U[-1,1], FP32.

    Every matrix lives in one flat buffer per operand kind at an offset that is
    a multiple of ``align`` elements.  Returns shapes, offsets and buffers.
    """
    shapes = cfg4_shapes(count, lo, hi)
    sizes = shapes[:, 0] * shapes[:, 1]
    padded = (sizes + align - 1) // align * align
    offs = np.zeros(count, np.int64)
    offs[1:] = np.cumsum(padded)[:-1]
    total = int(padded.sum())
    bufs = {}
    for i, name in enumerate(("A", "Bp")):
        d = rng(4, 1 + i).uniform(-1.0, 1.0, int(sizes.sum())).astype(np.float32)
        buf = np.zeros(total, np.float32)
        # scatter the draws matrix by matrix into the padded layout
        src = np.zeros(count + 1, np.int64)
        src[1:] = np.cumsum(sizes)
        idx = np.repeat(offs - src[:-1], sizes) + np.arange(int(sizes.sum()))
        buf[idx] = d
        bufs[name] = buf
    return {"shapes": shapes, "offsets": offs, "total": total, **bufs}


def cfg4_tree():
    A, Bp = leaves(2)
    Y = trans(A) + 0.5 * Bp
    return Y


# ----------------------------------------------------------------------------
# random trees for the cost-model corpus
# ----------------------------------------------------------------------------
TREE_OPS = ("plus", "minus", "schur", "div", "scal_times", "exp", "log", "sqrt", "abs", "trans")
TREE_ROOT_RED = (None, "sum", "accu")


@dataclass
class RandomTree:
    expr: E
    shapes: List[Tuple[int, int]]   # per operand slot
    dtypes: List[str]               # per operand slot
    out_shape: Tuple[int, int]
    reduce: Optional[str]           # None, "accu", "sum"
    dim: int
    depth: int


def random_tree(g: np.random.Generator, max_depth: int = 6, k_lo: int = 10, k_hi: int = 26,
                max_operands: int = 8) -> RandomTree:
    """One random expression tree: depth 1..max_depth, n = 2^k elements, one
    element type per tree (F64/F32/F16/BF16), reductions only at the root."""
    depth = int(g.integers(1, max_depth + 1))
    k = int(g.integers(k_lo, k_hi + 1))
    a = int(g.integers(0, k + 1))
    rows, cols = 1 << a, 1 << (k - a)
    dtype = DTYPES[int(g.integers(0, 4))]
    shapes: List[Tuple[int, int]] = []

    def new_leaf(shape):
        same = [i for i, s in enumerate(shapes) if s == shape]
        if same and (len(shapes) >= max_operands or g.random() < 0.25):
            return leaf(int(g.choice(same)))
        if len(shapes) >= max_operands:
            # fall back to any operand of the transposed shape through a trans node
            tsame = [i for i, s in enumerate(shapes) if s == (shape[1], shape[0])]
            return trans(leaf(int(g.choice(tsame)))) if tsame else leaf(0)
        shapes.append(shape)
        return leaf(len(shapes) - 1)

    def gen(shape, d):
        if d <= 1:
            return new_leaf(shape)
        op = TREE_OPS[int(g.integers(0, len(TREE_OPS)))]
        if op in ("plus", "minus", "schur", "div"):
            dl = d - 1
            dr = int(g.integers(1, d))
            l, r = gen(shape, dl), gen(shape, dr)
            return E(op, (l, r))
        if op == "scal_times":
            return E(op, (gen(shape, d - 1),), float(g.choice([0.5, 0.75, 1.5, 2.5, 3.0, -1.25])))
        if op == "trans":
            return trans(gen((shape[1], shape[0]), d - 1))
        return E(op, (gen(shape, d - 1),))

    expr = gen((rows, cols), depth)
    if not shapes:
        shapes.append((rows, cols))
    red = TREE_ROOT_RED[int(g.integers(0, 3))]
    dim = int(g.integers(0, 2)) if red == "sum" else -1
    return RandomTree(expr, shapes, [dtype] * len(shapes), (rows, cols), red, dim, depth)


def cfg5_trees(count: int = 6000, **kw) -> List[RandomTree]:
    g = rng(5, 0)
    return [random_tree(g, **kw) for _ in range(count)]


def cfg5_split(count: int = 6000, n_train: int = 5000):
    """Train / held-out index split (seeded permutation)."""
    p = rng(5, 1).permutation(count)
    return np.sort(p[:n_train]), np.sort(p[n_train:])
