"""Host-only checks of the C ABI: the library loads without a GPU, exports every
entry point of include/coot.h, validates arguments before touching a device,
and generates kernels that compile for gfx950 under strict floating-point
rules."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from synth import abs_, exp, leaf, leaves, sqrt, trans, conv

from paper_2308_03120_amd import coot

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
F = coot.fake_operand
G = 1 << 40


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2308_03120_amd import build

    if not os.path.exists(coot.LIB_PATH):
        build.build()
    coot.lib()


def header_functions():
    with open(os.path.join(ROOT, "include", "coot.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(coot_\w+)\s*\(", text, re.M)))


def test_every_declared_function_is_exported():
    out = subprocess.check_output(["nm", "-D", "--defined-only", coot.LIB_PATH], text=True)
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    declared = header_functions()
    assert len(declared) >= 20
    missing = [f for f in declared if f not in syms]
    assert not missing, missing
    assert set(coot.EXPORTS) <= set(declared)


def code(fn):
    try:
        fn()
    except coot.CootError as e:
        return e.code
    return 0


def test_validation_errors():
    A = F(10, 20, ptr=G)
    B = F(20, 10, ptr=2 * G)
    O = F(10, 20, ptr=3 * G)
    x, y = leaves(2)
    assert code(lambda: coot.validate(None, -1, x + y, [A, A], O)) == 0
    assert code(lambda: coot.validate(None, -1, x + y, [A, B], O)) == -2          # shape
    assert code(lambda: coot.validate(None, -1, trans(y) + x, [A, B], O)) == 0
    assert code(lambda: coot.validate(None, -1, x + y, [A], O)) == -1             # slot out of range
    assert code(lambda: coot.validate(None, -1, [("plus", 0, 1, 0)], [A], O)) == -1  # child not earlier
    assert code(lambda: coot.validate(None, -1, [("leaf", 0, -1, 0), (99, 0, -1, 0)], [A], O)) == -1
    assert code(lambda: coot.validate(None, -1, x + y, [A, F(10, 20, "f64", ptr=4 * G)], O)) == -3  # mixed precision
    assert code(lambda: coot.validate(None, -1, x, [A], F(20, 10, ptr=3 * G))) == -2  # out shape
    assert code(lambda: coot.validate(None, -1, x, [F(10, 20, ld=5, ptr=G)], O)) == -10  # ld < rows
    assert code(lambda: coot.validate(None, -1, x, [F(10, 20, ptr=0)], O)) == -10      # NULL with elements
    assert code(lambda: coot.validate(None, -1, x, [A], F(10, 20, "u64", ptr=3 * G))) == -3
    # aliasing: exact in-place is fine, a transposed read of the output is not
    assert code(lambda: coot.validate(None, -1, x + y, [A, O], O)) == 0
    S = F(10, 10, ptr=5 * G)
    assert code(lambda: coot.validate(None, -1, trans(x) + x, [S], S)) == -4
    assert code(lambda: coot.validate(None, -1, x + 1.0, [F(10, 20, ptr=3 * G + 4)], O)) == -4  # shifted overlap
    # reductions
    assert code(lambda: coot.validate("accu", -1, x, [A], F(1, 1, ptr=3 * G))) == 0
    assert code(lambda: coot.validate("accu", 0, x, [A], F(1, 20, ld=1, ptr=3 * G))) == -10
    assert code(lambda: coot.validate("sum", 0, x, [A], F(1, 20, ld=1, ptr=3 * G))) == 0
    assert code(lambda: coot.validate("sum", 1, x, [A], F(10, 1, ptr=3 * G))) == 0
    assert code(lambda: coot.validate("sum", 1, x, [A], F(20, 1, ptr=3 * G))) == -2
    assert code(lambda: coot.validate("dot", -1, x + y, [A, A], F(1, 1, ptr=3 * G))) == -1
    assert code(lambda: coot.validate("index_max", -1, x, [A], F(1, 1, ptr=3 * G))) == -3
    assert code(lambda: coot.validate("index_max", -1, x, [A], F(1, 1, "u64", ptr=3 * G))) == 0
    assert code(lambda: coot.validate("max", -1, x, [F(0, 5, ptr=0)], F(1, 1, ptr=3 * G))) == -5
    assert code(lambda: coot.validate("accu", -1, x, [F(0, 5, ptr=0)], F(1, 1, ptr=3 * G))) == 0
    assert code(lambda: coot.validate("accu", -1, x, [A], F(1, 1, ptr=G + 8))) == -4  # result inside an operand


def test_generator_and_view_validation():
    """Generators (memory-free operands) and views are checked on the host."""
    x, y = leaves(2)
    A = F(10, 20, ptr=G)
    O = F(10, 20, ptr=3 * G)
    assert code(lambda: coot.validate(None, -1, x + y, [A, coot.eye(10, 20)], O)) == 0
    assert code(lambda: coot.validate(None, -1, x + y, [A, coot.fill(10, 20, 0.5)], O)) == 0
    assert code(lambda: coot.validate(None, -1, trans(y) + x, [A, coot.eye(20, 10)], O)) == 0
    assert code(lambda: coot.validate(None, -1, x + y, [A, coot.eye(20, 10)], O)) == -2             # shape
    assert code(lambda: coot.validate(None, -1, x + y, [A, coot.eye(10, 20, "f64")], O)) == -3      # precision
    V = F(100, 1, ptr=G)
    OV = F(100, 1, ptr=3 * G)
    assert code(lambda: coot.validate(None, -1, x + y, [V, coot.linspace(0, 1, 100, "f32")], OV)) == 0
    bad = coot.linspace(0, 1, 100, "f32")
    bad.n_cols, bad.n_rows, bad.ld = 10, 10, 10
    assert code(lambda: coot.validate(None, -1, x, [bad], O)) == -2                                   # linspace is a vector
    g = coot.eye(10, 20)
    g.ptr = G
    assert code(lambda: coot.validate(None, -1, x, [g], O)) == -10                                    # generator with memory
    g = coot.eye(10, 20)
    g.flags |= coot.GEN_FILL
    assert code(lambda: coot.validate(None, -1, x, [g], O)) == -10                                    # two kinds
    assert code(lambda: coot.validate(None, -1, x + 1.0, [A], coot.eye(10, 20))) == -10              # not an output
    # views: a diagonal is 1 x n with ld + 1, a submatrix keeps the parent's ld
    M = F(10, 20, ptr=G)
    d = coot.diag(M, 3)
    assert (d.n_rows, d.n_cols, d.ld, d.ptr) == (1, 10, 11, G + 3 * 10 * 4)
    d = coot.diag(M, -4)
    assert (d.n_rows, d.n_cols, d.ld, d.ptr) == (1, 6, 11, G + 4 * 4)
    s = coot.submat(M, 2, 3, 5, 9)
    assert (s.n_rows, s.n_cols, s.ld, s.ptr) == (4, 7, 10, G + (2 + 3 * 10) * 4)
    assert code(lambda: coot.validate(None, -1, x + 1.0, [s], s)) == 0                                # in place
    assert code(lambda: coot.validate(None, -1, x + 1.0, [coot.submat(M, 2, 4, 5, 10)], s)) == -4    # overlap


def test_bad_config_rejected():
    A = F(10, 20, ptr=G)
    O = F(10, 20, ptr=3 * G)
    e = coot.expr(leaf(0) + 1.0, cfg=(3, 256, 1))
    import ctypes as C
    arr, n = coot._ops([A])
    assert coot.lib().coot_validate(-1, -1, C.byref(e), arr, n, C.byref(O)) == -10
    assert coot.config_of(0) == (1, 64, 1) and coot.config_of(63) == (8, 512, 8)


def test_generated_source_is_strict_ieee():
    x, y = leaves(2)
    src = coot.kernel_source(None, -1, sqrt(abs_(x)) % y - x / (1 + abs_(y)),
                             [F(1 << 20, 1, ptr=G), F(1 << 20, 1, ptr=2 * G)], F(1 << 20, 1, ptr=3 * G))
    assert "#pragma clang fp contract(off)" in src
    body = src[src.find("CD float x_eval"):]
    body = body[: body.find("}")]
    assert "fma" not in body and "__f" not in body.replace("__builtin_fabsf", "")
    assert "sqrtf(" in body and " / " in body


def test_rewrites_move_trans_to_operands_and_merge_reads():
    x, y = leaves(2)
    A = F(30, 40, ptr=G)
    B = F(40, 30, ptr=2 * G)
    src = coot.kernel_source(None, -1, trans(trans(x) + y) - x, [A, B], F(30, 40, ptr=3 * G))
    tree = [l for l in src.splitlines() if l.startswith("// tree:")][0]
    reads = re.findall(r"r(f32|f64|f16|bf16)(S|T)", tree)
    assert reads == [("f32", "S"), ("f32", "T")]   # x read once, y read transposed
    assert ",30," not in tree                       # no transpose node left
    s2 = coot.kernel_source(None, -1, x % x + x, [A], F(30, 40, ptr=3 * G))
    assert len(re.findall(r"r(f32)(S)", [l for l in s2.splitlines() if l.startswith("// tree:")][0])) == 1


def test_features_shape_and_content():
    x, y = leaves(2)
    f = coot.features(None, -1, exp(x) + y % y, [F(1024, 64, ptr=G), F(1024, 64, ptr=2 * G)], F(1024, 64, ptr=3 * G))
    assert f.shape == (32,)
    assert f[0] == pytest.approx(np.log2(65536 + 1))
    assert f[5] == 2 and f[18] == 1 and f[15] == 1 and f[14] == 1 and f[23] == 0
    fr = coot.features("sum", 1, x, [F(1024, 64, ptr=G)], F(1024, 1, ptr=3 * G))
    assert fr[23] == 1 and fr[24] == 1 and fr[27] == 1


@pytest.mark.parametrize("red,dim,tree,ops,out", [
    (None, -1, "Y", [(1000, 1000)] * 4, (1000, 1000)),
    ("accu", -1, "AB", [(1000, 1000)] * 4, (1, 1)),
    ("sum", 0, "A", [(1000, 1000)] * 4, (1, 1000)),
    ("sum", 1, "A", [(1000, 1000)] * 4, (1000, 1)),
    ("index_max", -1, "absB", [(1000, 1000)] * 4, (1, 1)),
    (None, -1, "T", [(37, 211), (211, 37)], (211, 37)),
    ("accu", -1, "T", [(37, 211), (211, 37)], (1, 1)),
    (None, -1, "T", [(3001, 2), (2, 3001)], (2, 3001)),        # thin value, short rows
    ("index_max", -1, "T", [(12, 300), (300, 12)], (1, 1)),   # thin value, short columns
])
def test_generated_kernels_compile_for_gfx950(tmp_path, monkeypatch, red, dim, tree, ops, out):
    monkeypatch.setenv("COOT_CACHE_DIR", str(tmp_path))
    A, B, C, D = leaves(4)
    trees = {"Y": 2.5 * A + B % C - exp(D), "AB": A % B, "A": A, "absB": abs_(B), "T": trans(A) + 0.5 * B}
    opnds = [F(r, c, ptr=(i + 1) * G) for i, (r, c) in enumerate(ops)]
    odt = "u64" if red == "index_max" else "f32"
    o = F(out[0], out[1], odt, ld=1 if out[0] == 1 else out[0], ptr=9 * G)
    assert coot.precompile(red, dim, trees[tree], opnds, o) in (0, 1)


def test_batched_kernels_compile_for_gfx950(tmp_path):
    """The batched tile pass and its per-item combine, generated on the host,
    compile for gfx950 with the library's strict floating-point options."""
    import shutil
    import subprocess

    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    import synth
    src = coot.BatchPlan.kernel_source(synth.cfg4_tree(), [coot.F32, coot.F32], [[5, 7], [64, 64], [0, 3]],
                                       red_tree=synth.leaf(0) % synth.leaf(0))
    names = re.findall(r"__global__ void __launch_bounds__\(256\) (coot_batch_[0-9a-f]{16}(?:_comb)?)\(", src)
    assert len(names) == 2 and names[1] == names[0] + "_comb"
    f = tmp_path / "batch.hip"
    f.write_text("#include <hip/hip_runtime.h>\n" + src)
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang",
                        "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-c", str(f), "-o",
                        str(tmp_path / "batch.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    # without a reduction there is no combine kernel
    src2 = coot.BatchPlan.kernel_source(synth.cfg4_tree(), [coot.F32, coot.F32], [[5, 7]])
    assert "_comb" not in src2


def test_fp16_leaf_sums_add_from_the_storage_word(tmp_path):
    """Compensated sums whose tree is one FP16 leaf (accu, per-column sum) add
    each half with the mixed-precision FMA straight from its storage word;
    BF16 leaves, the pairwise variant and FP16 products keep the conversion
    first.  The FP16 kernels compile for gfx950."""
    import shutil

    n = 4096
    acc_out, col_out = F(1, 1, "f32", ptr=9 * G), F(1, n, "f32", ptr=9 * G)
    x, y = leaves(2)
    fused = [coot.kernel_source("accu", -1, x, [F(n, n, "f16", ptr=G)], acc_out),
             coot.kernel_source("sum", 0, x, [F(n, n, "f16", ptr=G)], col_out)]
    for s in fused:
        assert "acc_add_f16<1>" in s and "v_fma_mix_f32" in s
    plain = [coot.kernel_source("accu", -1, x, [F(n, n, "bf16", ptr=G)], acc_out),
             coot.kernel_source("accu", -1, x, [F(n, n, "f16", ptr=G)], acc_out, pairwise=True),
             coot.kernel_source("accu", -1, x % y, [F(n, n, "f16", ptr=G), F(n, n, "f16", ptr=2 * G)], acc_out)]
    for s in plain:
        assert "acc_add_f16" not in s
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    for i, src in enumerate(fused):
        f = tmp_path / f"k{i}.hip"
        f.write_text("#include <hip/hip_runtime.h>\n" + src)
        r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang",
                            "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", str(f), "-o",
                            str(tmp_path / f"k{i}.s")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        asm = (tmp_path / f"k{i}.s").read_text()
        assert "v_fma_mix_f32" in asm and "v_cvt_f32_f16_sdwa" not in asm


def test_batch_aliasing_rejected_before_any_device_work():
    """coot_batch_create checks every item's output against the memory the
    launch reads and writes before it allocates or launches anything, so the
    checks run without a device.  Y_i = trans(A_i) + 0.5 * B_i' (A_i r x c,
    B_i' and Y_i c x r)."""
    import ctypes as C

    tree = synth.cfg4_tree()
    r, c = 6, 4
    n = r * c * 4  # bytes of one FP32 item

    def create(ptrs, outs, shapes=((c, r), (c, r)), red_out=None):
        d = coot.BatchDescriptor(tree, [coot.F32, coot.F32], ptrs, [list(s) for s in shapes], out_ptrs=outs,
                                 red_tree=leaf(0) % leaf(0) if red_out else None, red_out=red_out)
        h = C.c_void_p()
        return coot.lib().coot_batch_create(C.byref(d.struct), None, C.byref(h))

    A0, B0, A1, B1, Y0, Y1 = (G * k for k in range(1, 7))
    ALIAS = -4
    # the output is an operand read through trans()
    assert create([[A0, B0], [A1, B1]], [A0, Y1]) == ALIAS
    # the output overlaps another item's operand
    assert create([[A0, B0], [A1, B1]], [Y0, B0 + 8]) == ALIAS
    # two outputs overlap
    assert create([[A0, B0], [A1, B1]], [Y0, Y0 + n - 4]) == ALIAS
    # the reduction results overlap an output
    assert create([[A0, B0], [A1, B1]], [Y0, Y1], red_out=Y1 + 4) == ALIAS
    # the output is the item's own straight slot, but starts elsewhere inside it
    assert create([[A0, B0], [A1, B1]], [B0 + 4, Y1]) == ALIAS
    assert "overlaps" in coot.last_error()
    # in place on the straight slot (same extent and type) and disjoint outputs pass the
    # check; without a device the call then fails at the device step instead
    assert create([[A0, B0], [A1, B1]], [B0, B1]) != ALIAS
    assert create([[A0, B0], [A1, B1]], [Y0, Y1], red_out=G * 7) != ALIAS
    # items of no elements touch no memory
    assert create([[A0, B0], [A1, B1]], [A0, Y1], shapes=((0, 3), (c, r))) != ALIAS


def test_probe_arguments_checked_on_the_host():
    """coot_bandwidth_probe rejects unknown kinds and launch shapes, lengths
    that are not whole vectors and misaligned pointers before touching a
    device."""
    L = coot.lib()
    d, s = C.c_void_p(G), C.c_void_p(2 * G)
    ERR_ARG = -10
    assert L.coot_bandwidth_probe(7, d, s, 1024, None) == ERR_ARG
    assert L.coot_bandwidth_probe(coot.PROBE_READ | (4 << 8), d, s, 1024, None) == ERR_ARG
    assert "shape" in coot.last_error()
    assert L.coot_bandwidth_probe(coot.PROBE_READ | (1 << 8), d, s, 1000, None) == ERR_ARG
    assert L.coot_bandwidth_probe(coot.PROBE_COPY | (3 << 8), C.c_void_p(G + 8), s, 1024, None) == ERR_ARG
    # tiled probes: whole 64-column blocks of 16384 rows only
    assert L.coot_bandwidth_probe(coot.PROBE_TILED_COPY, d, s, (4 << 20) + 16, None) == ERR_ARG
    assert "4 MiB" in coot.last_error()
    assert L.coot_bandwidth_probe(coot.PROBE_TILED_READ2_WRITE1 | (2 << 8), d, s, 1 << 20, None) == ERR_ARG
    assert L.coot_bandwidth_probe(coot.PROBE_TILED_COPY | (4 << 8), d, s, 4 << 20, None) == ERR_ARG


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
def test_tall_tile_kernels_compile_for_gfx950(tmp_path, monkeypatch, dt):
    """Trees with straight reads only over strided views take tall tiles:
    whole tiles with 4-row accesses (operands on a common 4-element phase),
    whole tiles element by element (phases differ), partial tiles (clamped
    loads, tested stores), and an index generator; element-wise and index
    reductions."""
    monkeypatch.setenv("COOT_CACHE_DIR", str(tmp_path))
    x, y = leaves(2)
    es = {"f32": 4, "f64": 8, "bf16": 2}[dt]
    odt = "f64" if dt == "f64" else "f32"
    r, c, ld = 9000, 40, 9024
    for offs in ((4, 8, 4), (1, 6, 1)):
        A = F(r, c, dt, ld=ld, ptr=G + offs[0] * es)
        B = F(r, c, dt, ld=ld, ptr=2 * G + offs[1] * es)
        Y = F(r, c, odt, ld=ld, ptr=3 * G + offs[2] * (8 if odt == "f64" else 4))
        assert coot.precompile(None, -1, x * 2.0 - y, [A, B], Y) in (0, 1)
        assert coot.precompile("index_max", -1, x % y, [A, B], F(1, 1, "u64", ptr=9 * G)) in (0, 1)
    E = coot.eye(r, c, odt)
    assert coot.precompile(None, -1, x * 0.5 + leaves(2)[1], [F(r, c, dt, ld=ld, ptr=G), E], F(r, c, odt, ptr=3 * G)) in (0, 1)


def test_fp16_leaf_sums_share_a_module():
    """Many kernels compiled into one code object each sit in a namespace of
    their own, so every FP16 leaf sum carries its own copy of the
    mixed-precision helpers (a shared include guard left the second kernel
    without them)."""
    from synth import leaf as lf

    coot.precompile_begin()
    for ept in (1, 2, 4, 8):
        coot.precompile("accu", -1, lf(0), [F(1 << 20, 1, "f16", ptr=G)], F(1, 1, "f32", ptr=9 * G), cfg=(ept, 256, 8))
        coot.precompile("sum", 0, lf(0), [F(4096, 64, "f16", ptr=G)], F(1, 64, "f32", ptr=9 * G), cfg=(ept, 256, 8))
    assert coot.precompile_end(64) == 8
