"""Host-only checks of the C++ expression-template front end (include/coot.hpp,
the paper's Section 7 interface).  A small program (tests/cpp/
front_end_describe.cpp) builds expressions with the front end and prints the
node array and operand table each expression type flattens to; here every
one is evaluated by the CPU oracle next to the same expression built with the
Python tree helpers, on the same seeded data, and must agree bit for bit.
Compile-time rewrites (trans(trans(A)) is A, trans(eye) is eye) are
static_asserts of that program; misuse (A * B, mixed element types) must not
compile."""
import json
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from synth import abs_, conv, exp, leaf, log, ne, pow_, sqrt, tanh, trans

from paper_2308_03120_amd import coot

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2308_03120_amd")
CXX = ["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
       "-I" + os.path.join(ROOT, "include")]
LINK = ["-L" + LIBDIR, "-lcoot_mi355x", "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath," + LIBDIR]

P, Q, IP = 1 << 40, 1 << 41, 1 << 42   # stand-in device addresses: float, double, int32 memory
CODE_TO_NAME = {v: k for k, v in coot.OPS.items()}


@pytest.fixture(scope="module")
def described(tmp_path_factory):
    if not os.path.exists(coot.LIB_PATH):
        pytest.skip("library not built")
    exe = str(tmp_path_factory.mktemp("fe") / "describe")
    subprocess.check_call(CXX + [os.path.join(ROOT, "tests", "cpp", "front_end_describe.cpp"), "-o", exe] + LINK)
    out = subprocess.check_output([exe], text=True)
    return {d["name"]: d for d in map(json.loads, out.strip().splitlines())}


def memory(g):
    """Seeded contents of the program's stand-in float and double memory."""
    return {P: ("f32", g.uniform(-2, 2, 6000).astype(np.float32)), Q: ("f64", g.uniform(-2, 2, 1000)),
            IP: ("i32", g.integers(-2 ** 31, 2 ** 31, 2000).astype(np.int32))}


def operand_of(mem, op):
    """Dense oracle operand for one row of the operand table."""
    rows, cols, ld, dtype, flags, g0, g1, ptr = op
    dt = {0: "f32", 1: "f64", 5: "i32"}[dtype]
    if flags == coot.GEN_EYE:
        return oracle.eye(rows, cols, dt)
    if flags == coot.GEN_FILL:
        return oracle.fill(rows, cols, g0, dt)
    if flags == coot.GEN_LINSPACE:
        return oracle.linspace(g0, g1, rows * cols, dt, row=rows == 1)
    base = P if ptr < Q else (Q if ptr < IP else IP)
    _, buf = mem[base]
    off = (ptr - base) // buf.itemsize
    idx = off + np.arange(rows)[:, None] + ld * np.arange(cols)[None, :]
    return synth.Mat(np.asfortranarray(buf[idx]), dt)


def cpp_value(mem, d):
    nodes = [synth.Node(CODE_TO_NAME[op], a, b, k) for op, a, b, k in d["nodes"]]
    return oracle.evaluate(nodes, [operand_of(mem, o) for o in d["ops"]], "emu")


def mat_at(mem, base, off, rows, cols, ld=None):
    dt, buf = mem[base]
    ld = ld or rows
    idx = off + np.arange(rows)[:, None] + ld * np.arange(cols)[None, :]
    return synth.Mat(np.asfortranarray(buf[idx]), dt)


def test_compile_time_rewrites_and_expressions(described):
    g = np.random.default_rng(2024)
    mem = memory(g)
    A, B, C, D = (mat_at(mem, P, 1000 * i, 30, 20) for i in range(4))
    T = mat_at(mem, P, 4000, 20, 30)
    X = mat_at(mem, Q, 0, 30, 20)
    a, b, c, d = (leaf(i) for i in range(4))
    cases = {
        "small_Y": (2.5 * a + b % c - exp(d), [A, B, C, D]),
        "accu_AB": (a % b, [A, B]),
        "trans_sum": (trans(a) + 0.5 * b, [T, B]),
        "double_trans": (a % a, [A]),
        "scalars": (1.0 - a / 2.0 + (3.0 / b) - (a - 4.0), [A, B]),
        "relational": ((a > 0.3) % (0.3 > b) + (a <= b) - ne(a, 2.0), [A, B]),
        "funcs": (sqrt(abs_(a)) % log(abs_(b) + 1.0) + pow_(abs_(c), 1.5) - tanh(d), [A, B, C, D]),
        "conv": (conv(a * 2.0, "f32") + b, [X, A]),
        "neg": (a * -1.0 + b, [A, B]),
        "eye_fill": (a + 3.0 * b - c + trans(d),
                     [A, oracle.eye(30, 20, "f32"), oracle.fill(30, 20, 1.0, "f32"), oracle.eye(20, 30, "f32")]),
        "linspace": (a * 2.0, [oracle.linspace(-1.0, 2.0, 30, "f32")]),
        "views": (a + b, [mat_at(mem, P, 1 + 2 * 30, 10, 11, 30), mat_at(mem, P, 1000, 10, 11, 30)]),
        "diag": (trans(a), [mat_at(mem, P, 3 * 30, 1, 17, 31)]),
        "integers": (conv(a * 2.0 + b / 3.0, "f32") + c, [mat_at(mem, IP, 0, 30, 20), mat_at(mem, IP, 1000, 30, 20), A]),
        "integer_conv": (conv(a * 1000.0, "i32") + b, [A, mat_at(mem, IP, 0, 30, 20)]),
    }
    assert set(cases) == set(described)
    for name, (tree, ops) in cases.items():
        want = oracle.evaluate(tree.postfix(), ops, "emu")
        got = cpp_value(mem, described[name])
        assert got.shape == want.shape, name
        assert np.array_equal(got, want, equal_nan=True), name


def test_operand_slots(described):
    # a matrix read twice is one operand; trans(trans(A)) leaves no transpose node
    d = described["double_trans"]
    assert len(d["ops"]) == 1 and all(n[0] != coot.OPS["trans"] for n in d["nodes"])
    # trans of a generator is the generator with its shape swapped: no transpose node
    d = described["eye_fill"]
    assert all(n[0] != coot.OPS["trans"] for n in d["nodes"])
    assert sorted((o[0], o[1]) for o in d["ops"] if o[4] == coot.GEN_EYE) == [(30, 20), (30, 20)]
    # the diagonal view: 1 x n with the parent's ld + 1, starting k columns in
    d = described["diag"]
    assert d["ops"][0][:3] == [1, 17, 31] and d["ops"][0][7] == P + 3 * 30 * 4


@pytest.mark.parametrize("snippet", [
    "fmat A(nullptr, 2, 2), B(nullptr, 2, 2); auto C = A * B;",        # a matrix product is not element-wise
    "fmat A(nullptr, 2, 2); mat B(nullptr, 2, 2); auto C = A + B;",     # mixed element types need conv_to
    "fmat A(nullptr, 2, 2); auto C = A + std::string(\"x\");",          # not a scalar
])
def test_misuse_does_not_compile(tmp_path, snippet):
    src = tmp_path / "bad.cpp"
    src.write_text('#include <string>\n#include "coot.hpp"\nusing namespace coot;\nint main() { ' + snippet +
                   " (void)C; return 0; }\n")
    r = subprocess.run(CXX + ["-fsyntax-only", str(src)], capture_output=True, text=True)
    assert r.returncode != 0, snippet
