"""Batching extension: many matrices of different shapes in one persistent
launch replayed from a hipGraph.  Per matrix Y_i = trans(A_i) + 0.5*B_i'
(B_i' a matrix of its own with the shape of trans(A_i)) and
r_i = accu(Y_i % Y_i).  Y_i is checked bit for bit against the oracle's per-node
rounded evaluation, r_i within 1e-6 of the exact sum of y^2 over those values;
graph replays, the per-matrix launches and the unfused per-node form are
compared with the one-launch result."""
import numpy as np
import pytest

import oracle
import synth
from synth import leaf

from gpu_util import TORCH_DT, need_gpu, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402

Ytree = synth.cfg4_tree()
Rtree = leaf(0) % leaf(0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


def make_batch(shapes, g, dt="f32", align=64):
    """Flat device buffers for A_i (r x c), Bp_i (c x r), Y_i (c x r)."""
    sizes = shapes[:, 0] * shapes[:, 1]
    padded = (sizes + align - 1) // align * align
    offs = np.zeros(len(shapes), np.int64)
    offs[1:] = np.cumsum(padded)[:-1]
    total = int(padded.sum()) + align
    npdt = np.float32 if dt == "f32" else np.float64
    A = g.uniform(-1, 1, total).astype(npdt)
    B = g.uniform(-1, 1, total).astype(npdt)
    return offs, total, A, B


def host_mats(shapes, offs, A, B, i, dt="f32"):
    r, c = shapes[i]
    n = r * c
    Am = synth.Mat(np.asfortranarray(A[offs[i]:offs[i] + n].reshape((r, c), order="F")), dt)
    Bm = synth.Mat(np.asfortranarray(B[offs[i]:offs[i] + n].reshape((c, r), order="F")), dt)
    return Am, Bm


def run_batch(shapes, offs, dA, dB, dY, red, flags=0, red_dtype=coot.F32, out=True):
    es = dA.element_size()
    ptrs = [[dA.data_ptr() + int(o) * es, dB.data_ptr() + int(o) * es] for o in offs]
    outs = [dY.data_ptr() + int(o) * es for o in offs] if out else None
    plan = coot.BatchPlan(Ytree, [coot.F32 if dA.dtype == torch.float32 else coot.F64] * 2, ptrs,
                          [[int(c), int(r)] for r, c in shapes],  # Y_i is c x r
                          out_ptrs=outs, out_dtype=coot.F32 if dA.dtype == torch.float32 else coot.F64,
                          red_tree=Rtree, red_op="accu", red_out=red, red_dtype=red_dtype, flags=flags)
    return plan


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_small_ragged_batch_against_oracle(dt):
    g = np.random.default_rng(5)
    shapes = np.concatenate([np.array([[1, 1], [1, 70], [70, 1], [64, 64], [65, 63], [130, 7]]),
                             g.integers(1, 200, (60, 2))])
    offs, total, A, B = make_batch(shapes, g, dt)
    tdt = torch.float32 if dt == "f32" else torch.float64
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dY = torch.full((total,), float("nan"), dtype=tdt, device="cuda")
    red = torch.zeros(len(shapes), dtype=tdt, device="cuda")
    plan = run_batch(shapes, offs, dA, dB, dY, red, red_dtype=coot.F32 if dt == "f32" else coot.F64)
    plan.run()
    torch.cuda.synchronize()
    Yh = dY.cpu().numpy().astype(np.float64)
    rh = red.cpu().numpy().astype(np.float64)
    for i, (r, c) in enumerate(shapes):
        Am, Bm = host_mats(shapes, offs, A, B, i, dt)
        em = oracle.evaluate(Ytree.postfix(), [Am, Bm], "emu")
        got = Yh[offs[i]:offs[i] + r * c].reshape((c, r), order="F")
        assert np.array_equal(got, em), i
        o, _, _ = oracle.reduce("accu", (Ytree % Ytree).postfix(), [Am, Bm], mode="emu")
        assert abs(rh[i] - o[0]) <= (1e-6 if dt == "f32" else 1e-13) * abs(o[0]), (i, rh[i], o[0])
    plan.close()


@pytest.mark.parametrize("dts", [("f32", "bf16"), ("f16", "f16")])
def test_sixteen_bit_operands(dts):
    """16-bit A_i (staged through LDS) and B_i (read straight and widened on
    load, every element of a unit's last pass loading the unit's first when it
    falls past the unit): Y_i in FP32 bit for bit, r_i within 1e-6."""
    g = np.random.default_rng(9)
    shapes = np.concatenate([np.array([[1, 1], [1, 70], [70, 1], [64, 64], [65, 63], [130, 7], [300, 41]]),
                             g.integers(1, 200, (40, 2))])
    sizes = shapes[:, 0] * shapes[:, 1]
    padded = (sizes + 63) // 64 * 64
    offs = np.zeros(len(shapes), np.int64)
    offs[1:] = np.cumsum(padded)[:-1]
    total = int(padded.sum()) + 64
    host = [synth.store(g.uniform(-1, 1, total), dt) for dt in dts]
    devs = []
    for h, dt in zip(host, dts):
        t = torch.from_numpy(h.view(np.int16)).view(TORCH_DT[dt]) if dt != "f32" else torch.from_numpy(h)
        devs.append(t.cuda())
    dY = torch.full((total,), float("nan"), dtype=torch.float32, device="cuda")
    red = torch.zeros(len(shapes), dtype=torch.float32, device="cuda")
    ptrs = [[devs[0].data_ptr() + int(o) * devs[0].element_size(), devs[1].data_ptr() + int(o) * devs[1].element_size()]
            for o in offs]
    code = {"f32": coot.F32, "bf16": coot.BF16, "f16": coot.F16}
    plan = coot.BatchPlan(Ytree, [code[dts[0]], code[dts[1]]], ptrs, [[int(c), int(r)] for r, c in shapes],
                          out_ptrs=[dY.data_ptr() + int(o) * 4 for o in offs], out_dtype=coot.F32,
                          red_tree=Rtree, red_op="accu", red_out=red, red_dtype=coot.F32)
    plan.run()
    torch.cuda.synchronize()
    Yh = dY.cpu().numpy().astype(np.float64)
    rh = red.cpu().numpy().astype(np.float64)
    for i, (r, c) in enumerate(shapes):
        n = r * c
        Am = synth.Mat(np.asfortranarray(host[0][offs[i]:offs[i] + n].reshape((r, c), order="F")), dts[0])
        Bm = synth.Mat(np.asfortranarray(host[1][offs[i]:offs[i] + n].reshape((c, r), order="F")), dts[1])
        em = oracle.evaluate(Ytree.postfix(), [Am, Bm], "emu")
        got = Yh[offs[i]:offs[i] + n].reshape((c, r), order="F")
        assert np.array_equal(got, em), (dts, i)
        o, _, _ = oracle.reduce("accu", (Ytree % Ytree).postfix(), [Am, Bm], mode="emu")
        assert abs(rh[i] - o[0]) <= 1e-6 * abs(o[0]), (dts, i, rh[i], o[0])
    plan.close()


def test_results_do_not_depend_on_the_batch():
    """Items are cut into units by their shape alone and each item's unit
    partials are added in unit order, so Y_i and r_i are bit-identical
    whatever else is in the batch and wherever the item sits in it (here: the
    batch, the batch reversed, and every third item alone)."""
    g = np.random.default_rng(8)
    shapes = np.concatenate([np.array([[512, 512], [300, 500], [1, 4000], [4000, 1], [65, 65], [20000, 3]]),
                             g.integers(1, 300, (200, 2))])
    offs, total, A, B = make_batch(shapes, g)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    es = 4
    n = len(shapes)
    res = []
    for order in (np.arange(n), np.arange(n)[::-1], np.arange(n)[::3]):
        dY = torch.full((total,), float("nan"), device="cuda")
        red = torch.full((n,), float("nan"), device="cuda")
        plan = coot.BatchPlan(Ytree, [coot.F32, coot.F32],
                              [[dA.data_ptr() + int(offs[i]) * es, dB.data_ptr() + int(offs[i]) * es] for i in order],
                              [[int(shapes[i][1]), int(shapes[i][0])] for i in order],
                              out_ptrs=[dY.data_ptr() + int(offs[i]) * es for i in order], red_tree=Rtree,
                              red_op="accu", red_out=red)
        plan.run()
        torch.cuda.synchronize()
        r = torch.full((n,), float("nan"), device="cuda")
        r[torch.from_numpy(np.ascontiguousarray(order)).cuda()] = red[:len(order)]
        res.append((order, dY.clone(), r))
        plan.close()
    for order, y, r in res[1:]:
        for i in order:
            a, b_ = int(offs[i]), int(offs[i] + shapes[i].prod())
            assert torch.equal(y[a:b_], res[0][1][a:b_]), i
        idx = torch.from_numpy(np.ascontiguousarray(order)).cuda()
        assert torch.equal(r[idx], res[0][2][idx])
    rh = res[0][2].cpu().numpy().astype(np.float64)
    for i in (0, 1, 2, 3, 5):
        Am, Bm = host_mats(shapes, offs, A, B, i)
        o, _, _ = oracle.reduce("accu", (Ytree % Ytree).postfix(), [Am, Bm], mode="emu")
        assert abs(rh[i] - o[0]) <= 1e-6 * abs(o[0]), (i, rh[i], o[0])


def test_reduction_only_and_empty_items():
    g = np.random.default_rng(6)
    shapes = np.array([[5, 9], [0, 4], [33, 0], [100, 100], [1, 1]])
    offs, total, A, B = make_batch(shapes, g)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    red = torch.full((len(shapes),), float("nan"), device="cuda")
    es = 4
    ptrs = [[dA.data_ptr() + int(o) * es, dB.data_ptr() + int(o) * es] for o in offs]
    plan = coot.BatchPlan(Ytree, [coot.F32, coot.F32], ptrs, [[int(c), int(r)] for r, c in shapes], out_ptrs=None,
                          red_tree=leaf(0), red_op="norm2", red_out=red)
    plan.run()
    torch.cuda.synchronize()
    rh = red.cpu().numpy()
    assert rh[1] == 0.0 and rh[2] == 0.0
    for i in (0, 3, 4):
        Am, Bm = host_mats(shapes, offs, A, B, i)
        o, _, _ = oracle.reduce("norm2", Ytree.postfix(), [Am, Bm], mode="emu")
        assert abs(rh[i] - o[0]) <= 1e-6 * o[0]
    plan.close()


def test_batch_rejects_bad_input():
    dA = torch.zeros(64, device="cuda")
    with pytest.raises(coot.CootError):
        coot.BatchPlan(Ytree, [coot.F32, coot.F32], [[dA.data_ptr(), 0]], [[4, 4]], out_ptrs=[dA.data_ptr()])
    # A + trans(A) needs square items
    with pytest.raises(coot.CootError) as e:
        coot.BatchPlan(leaf(0) + synth.trans(leaf(0)), [coot.F32], [[dA.data_ptr()]], [[2, 3]],
                       out_ptrs=[dA.data_ptr() + 4096])
    assert e.value.code == -2


@pytest.fixture(scope="module")
def full():
    d = synth.cfg4_inputs()
    shapes, offs = d["shapes"], d["offsets"]
    dA, dB = torch.from_numpy(d["A"]).cuda(), torch.from_numpy(d["Bp"]).cuda()
    dY = torch.zeros(d["total"], device="cuda")
    red = torch.zeros(len(shapes), device="cuda")
    plan = run_batch(shapes, offs, dA, dB, dY, red)
    yield d, dA, dB, dY, red, plan
    plan.close()


def test_full_batch_graph_replays(full):
    d, dA, dB, dY, red, plan = full
    shapes, offs = d["shapes"], d["offsets"]
    plan.run()
    torch.cuda.synchronize()
    r1, y1 = red.clone(), dY.clone()
    plan.run()
    plan.run()
    torch.cuda.synchronize()
    assert torch.equal(red, r1) and torch.equal(dY, y1)
    g = np.random.default_rng(7)
    sample = np.unique(np.concatenate([g.choice(len(shapes), 300, replace=False),
                                       [int(np.argmax(shapes.prod(1))), int(np.argmin(shapes.prod(1)))]]))
    Yh = dY.cpu().numpy().astype(np.float64)
    rh = red.cpu().numpy().astype(np.float64)
    for i in sample:
        r, c = shapes[i]
        Am, Bm = host_mats(shapes, offs, d["A"], d["Bp"], i)
        em = oracle.evaluate(Ytree.postfix(), [Am, Bm], "emu")
        assert np.array_equal(Yh[offs[i]:offs[i] + r * c].reshape((c, r), order="F"), em), i
        o, _, _ = oracle.reduce("accu", (Ytree % Ytree).postfix(), [Am, Bm], mode="emu")
        assert abs(rh[i] - o[0]) <= 1e-6 * o[0], (i, rh[i], o[0])
    # every r_i is a sum of squares of the stored Y_i: positive and equal to its norm squared
    assert np.all(rh > 0)


def test_per_matrix_calls_match(full):
    """The baseline without batching (fused coot_eval + coot_reduce per matrix)
    gives the same Y_i bit for bit and r_i within the reduction gate."""
    d, dA, dB, dY, red, plan = full
    shapes, offs = d["shapes"], d["offsets"]
    n = 1500
    plan.run()
    torch.cuda.synchronize()
    red2 = torch.zeros(n, device="cuda")
    dY2 = torch.zeros_like(dY)
    p2 = run_batch(shapes[:n], offs[:n], dA, dB, dY2, red2, flags=coot.BATCH_PER_ITEM)
    p2.run()
    torch.cuda.synchronize()
    end = int(offs[n - 1] + shapes[n - 1].prod())
    assert torch.equal(dY2[:end], dY[:end])
    assert ((red2 - red[:n]).abs() / red[:n]).max().item() <= 1e-6
    p2.close()


def test_unfused_baseline_matches(full):
    d, dA, dB, dY, red, plan = full
    shapes, offs = d["shapes"], d["offsets"]
    n = 400  # a prefix of the batch: the unfused form is ~5 launches per matrix
    red3 = torch.zeros(n, device="cuda")
    dY3 = torch.zeros_like(dY)
    p3 = run_batch(shapes[:n], offs[:n], dA, dB, dY3, red3, flags=coot.BATCH_UNFUSED)
    p3.run()
    plan.run()
    torch.cuda.synchronize()
    end = int(offs[n - 1] + shapes[n - 1].prod())
    assert torch.equal(dY3[:end], dY[:end])
    rel = ((red3 - red[:n]).abs() / red[:n]).max().item()
    assert rel <= 1e-6
    p3.close()


def test_one_call_batched_entry(full):
    """coot_eval_batched through the C ABI: the first call builds the plan,
    later calls with the same descriptor replay its graph; Y_i bit-exact
    against the oracle's per-node rounding, r_i within 1e-6 of the oracle, and
    both bit-identical to coot_batch_run of an explicitly created plan."""
    import ctypes as C

    d, dA, dB, dY, red, plan = full
    shapes, offs = d["shapes"], d["offsets"]
    plan.run()
    torch.cuda.synchronize()
    y_ref, r_ref = dY.clone(), red.clone()
    es = 4
    dY2 = torch.full_like(dY, float("nan"))
    red2 = torch.full_like(red, float("nan"))
    desc = coot.BatchDescriptor(Ytree, [coot.F32, coot.F32],
                                [[dA.data_ptr() + int(o) * es, dB.data_ptr() + int(o) * es] for o in offs],
                                [[int(c), int(r)] for r, c in shapes],
                                out_ptrs=[dY2.data_ptr() + int(o) * es for o in offs], out_dtype=coot.F32,
                                red_tree=Rtree, red_op="accu", red_out=red2, red_dtype=coot.F32)
    # the items' elements (the padding between items is never written)
    inside = np.zeros(dY.numel(), bool)
    for o, (r, c) in zip(offs, shapes):
        inside[int(o):int(o) + int(r * c)] = True
    inside = torch.from_numpy(inside).cuda()
    launches0 = coot.stats()["launches"]
    rc = coot.lib().coot_eval_batched(C.byref(desc.struct), C.c_void_p(coot.current_stream()))
    assert rc == 0, coot.last_error()
    torch.cuda.synchronize()
    assert torch.equal(dY2[inside], y_ref[inside]) and torch.equal(red2, r_ref)
    assert torch.isnan(dY2[~inside]).all()
    # a replay of the cached plan: one graph launch, the same bits
    dY2.fill_(float("nan"))
    red2.fill_(float("nan"))
    launches1 = coot.stats()["launches"]
    assert coot.lib().coot_eval_batched(C.byref(desc.struct), C.c_void_p(coot.current_stream())) == 0
    torch.cuda.synchronize()
    assert coot.stats()["launches"] - launches1 == 1 and launches1 - launches0 == 1
    assert torch.equal(dY2[inside], y_ref[inside]) and torch.equal(red2, r_ref)
    Yh = dY2.cpu().numpy().astype(np.float64)
    rh = red2.cpu().numpy().astype(np.float64)
    g = np.random.default_rng(17)
    for i in g.choice(len(shapes), 100, replace=False):
        r, c = shapes[i]
        Am, Bm = host_mats(shapes, offs, d["A"], d["Bp"], i)
        em = oracle.evaluate(Ytree.postfix(), [Am, Bm], "emu")
        assert np.array_equal(Yh[offs[i]:offs[i] + r * c].reshape((c, r), order="F"), em), i
        o, _, _ = oracle.reduce("accu", (Ytree % Ytree).postfix(), [Am, Bm], mode="emu")
        assert abs(rh[i] - o[0]) <= 1e-6 * o[0], (i, rh[i], o[0])


def test_one_call_batched_entry_follows_the_descriptor():
    """A descriptor whose contents change gets a plan of its own (new pointers
    give new results); more descriptors than the library keeps evict the
    oldest plan, which is rebuilt when used again."""
    g = np.random.default_rng(21)
    shapes = g.integers(1, 90, (40, 2))
    offs, total, A, B = make_batch(shapes, g)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    es = 4
    ptrs = [[dA.data_ptr() + int(o) * es, dB.data_ptr() + int(o) * es] for o in offs]
    outs = [torch.full((total,), float("nan"), device="cuda") for _ in range(18)]
    reds = [torch.zeros(len(shapes), device="cuda") for _ in range(18)]
    descs = [coot.BatchDescriptor(Ytree, [coot.F32, coot.F32], ptrs, [[int(c), int(r)] for r, c in shapes],
                                  out_ptrs=[outs[k].data_ptr() + int(o) * es for o in offs], red_tree=Rtree,
                                  red_out=reds[k]) for k in range(18)]
    for k in range(18):
        coot.eval_batched(descs[k])
    coot.eval_batched(descs[0])   # evicted by the 17th descriptor: rebuilt
    torch.cuda.synchronize()
    for k in range(1, 18):
        assert torch.equal(torch.nan_to_num(outs[k], nan=3.0), torch.nan_to_num(outs[0], nan=3.0))
        assert torch.equal(reds[k], reds[0])
    Yh = outs[0].cpu().numpy().astype(np.float64)
    for i in (0, 7, 39):
        r, c = shapes[i]
        Am, Bm = host_mats(shapes, offs, A, B, i)
        assert np.array_equal(Yh[offs[i]:offs[i] + r * c].reshape((c, r), order="F"),
                              oracle.evaluate(Ytree.postfix(), [Am, Bm], "emu"))
