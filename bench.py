"""Benchmark of the fused element-wise + reduction hot path on one MI355X.

Workload (the plain method at scale): FP32 and FP64 vectors x, y of 2^28
elements, seeded N(0,1), 64 tied maxima injected in x.  One step runs, for
each precision, the five calls of that workload as fused kernels:
    axpy   y = y + 0.75*x          (in place, the paper's Task 2 form)
    z      sqrt(abs(x)) % y - x/(1+abs(y))
    dot    dot(x, y)
    norm   norm(x)
    index  index_max(x)
Inputs are resident in HBM before the timed region.  The value is effective
bandwidth: algorithmic bytes (each distinct operand read once, each output
written once) over wall time of the K timed steps.  The same step with one
kernel per node and temporaries gives the unfused baseline.

Prints one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBS = 8000.0
N = 1 << 28


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ops_of(synth):
    x, y = synth.leaves(2)
    t = synth.cfg2_trees()
    # (name, kind, tree, operand slots, algorithmic bytes per element in units of the item size)
    return [
        ("axpy", "eval", t["axpy"], 3),
        ("z", "eval", t["z"], 3),
        ("dot", "dot", t["dot"], 2),
        ("norm", "norm2", x, 1),
        ("index_max", "index_max", x, 1),
    ]


def build_step(coot, synth, torch, dt, X, Y, Yw, Z, unfused=False):
    """List of (name, bytes, callable) for one precision."""
    sz = 4 if dt == "f32" else 8
    calls = []
    for name, kind, tree, units in ops_of(synth):
        nbytes = units * sz * N
        if kind == "eval":
            if name == "axpy":
                fn = (lambda tree=tree: coot.eval(tree, [X, Yw], Yw, unfused=unfused))
            else:
                fn = (lambda tree=tree: coot.eval(tree, [X, Y], Z, unfused=unfused))
        else:
            ops = [X, Y] if kind == "dot" else [X]
            out = torch.empty(1, dtype=torch.int64 if kind == "index_max" else (torch.float32 if dt == "f32" else torch.float64),
                              device="cuda")
            fn = (lambda tree=tree, kind=kind, ops=ops, out=out: coot.reduce(kind, tree, ops, out=out, unfused=unfused))
        calls.append((f"{name}_{dt}", nbytes, fn))
    return calls


def cpu_baseline(oracle, synth, np, min_s: float = 10.0, max_passes: int = 64):
    """The oracle on a bounded sample of the same workload (1 host thread):
    whole passes of the ten calls on 2^22-element inputs, repeated until at
    least `min_s` seconds of oracle time; input generation is not timed."""
    n = 1 << 22
    trees = synth.cfg2_trees()
    inputs = []
    for dt in ("f32", "f64"):
        d = synth.cfg2_inputs(dt, n=n, n_ties=64)
        inputs.append(([d["x"], d["y"]], 4 if dt == "f32" else 8))
    total_bytes = 0.0
    el = 0.0
    reps = 0
    while el < min_s and reps < max_passes:
        t0 = time.perf_counter()
        for mats, sz in inputs:
            oracle.evaluate(trees["axpy"].postfix(), mats, "exact")
            oracle.evaluate(trees["z"].postfix(), mats, "exact")
            oracle.reduce("dot", trees["dot"].postfix(), mats)
            oracle.reduce("norm2", [synth.Node("leaf", 0)], mats[:1])
            oracle.reduce("index_max", [synth.Node("leaf", 0)], mats[:1])
            total_bytes += (3 + 3 + 2 + 1 + 1) * sz * n
        el += time.perf_counter() - t0
        reps += 1
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": round(total_bytes / el / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} pass(es) of the 10 FP32+FP64 calls on 2^22-element vectors "
                      f"(inputs generated beforehand, untimed), {el:.1f} s",
            "host_cpus": os.cpu_count(), "host_cpus_usable": len(os.sched_getaffinity(0)), "cpu_model": model}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--unfused-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="scale workload: skip the precision, batched and small figures added to the line")
    ap.add_argument("--workload", default="scale",
                    choices=["scale", "costmodel", "batched", "precision", "tiled", "small", "stats"],
                    help="scale (default): the 2^28-element FP32/FP64 calls; costmodel: learned launch "
                         "configuration over 6,000 random trees; batched: 10,000 matrices in one launch; "
                         "precision: 16384^2 BF16/FP16 sums and dots; tiled: transposed reads (64x64 and "
                         "shape-adaptive tiles); small: the 1000x1000 FP32 calls, warm and cold; stats: mean, "
                         "var, stddev, count / all / any of relational trees")
    ap.add_argument("--out-dir", default=os.path.join(ROOT, "bench_out"),
                    help="where the cost-model workload writes its corpus table and weights")
    ap.add_argument("--trees", type=int, default=6000)
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter files and exit")
    ap.add_argument("--no-baselines", action="store_true",
                    help="batched workload: time only the one-launch plan (for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run the library's plain 1 GiB copy kernel 3 times (counter calibration)")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(args.traffic_from[0], args.traffic_from[1], os.path.join(ROOT, "profiles", "traffic.json"))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2308_03120_amd import coot

    torch.cuda.set_device(0)
    coot.init(0)
    if args.calibrate_copy:
        src = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            coot.copy(dst, src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "costmodel":
        return costmodel_workload(args, np, torch, synth, coot)
    if args.workload == "batched":
        return batched_workload(args, np, torch, synth, coot)
    if args.workload == "precision":
        return precision_workload(args, np, torch, synth, coot)
    if args.workload == "tiled":
        return tiled_workload(args, np, torch, synth, coot)
    if args.workload == "small":
        return small_workload(args, np, torch, synth, coot)
    if args.workload == "stats":
        return stats_workload(args, np, torch, synth, coot)
    steps = []
    bufs = []
    for dt in ("f32", "f64"):
        log(f"generating {dt} inputs")
        d = synth.cfg2_inputs(dt, n=N)
        X = torch.from_numpy(d["x"]).cuda()
        Y = torch.from_numpy(d["y"]).cuda()
        Yw = Y.clone()
        Z = torch.empty_like(X)
        bufs.append((dt, X, Y, Yw, Z))
        steps += build_step(coot, synth, torch, dt, X, Y, Yw, Z)
        del d
    step_bytes = sum(b for _, b, _ in steps)

    # warm-up: compiles / loads kernels, then a breakdown pass with HIP events
    # between the calls (on the stream the kernels are launched on)
    for _, _, fn in steps:
        fn()
    torch.cuda.synchronize()
    W = max(1, args.warmup)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(steps) + 1)] for _ in range(W)]
    for k in range(W):
        ev[k][0].record()
        for i, (_, _, fn) in enumerate(steps):
            fn()
            ev[k][i + 1].record()
    torch.cuda.synchronize()
    per = {}
    for i, (name, nbytes, _) in enumerate(steps):
        ts = [ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(W)]
        avg = sum(ts) / len(ts)
        per[name] = {"us": round(avg * 1e3, 2), "GBps": round(nbytes / (avg * 1e-3) / 1e9, 1)}
    dom = max(per, key=lambda k: per[k]["us"])
    dom_i = [n for n, _, _ in steps].index(dom)

    # timed region: K steps; events bracket only the dominant kernel
    K = args.steps
    evd = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        for i, (_, _, fn) in enumerate(steps):
            if i == dom_i:
                evd[k][0].record()
                fn()
                evd[k][1].record()
            else:
                fn()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dom_us = sum(a.elapsed_time(b) for a, b in evd) / K * 1e3
    ms_step = wall / K * 1e3
    value = step_bytes * K / wall / 1e9

    # unfused baseline: the same step, one kernel per node with temporaries
    un_steps = []
    for dt, X, Y, Yw, Z in bufs:
        un_steps += build_step(coot, synth, torch, dt, X, Y, Yw, Z, unfused=True)
    for _, _, fn in un_steps:
        fn()
    torch.cuda.synchronize()
    Ku = max(1, args.unfused_steps)
    t1 = time.perf_counter()
    for _ in range(Ku):
        for _, _, fn in un_steps:
            fn()
    torch.cuda.synchronize()
    ms_unfused = (time.perf_counter() - t1) / Ku * 1e3

    del bufs
    torch.cuda.empty_cache()
    # streaming ceilings of each read/write mix (the library's probes, 1 GiB
    # per stream): element-wise calls (two reads per write) against the 2:1
    # probe, reductions against the read-only probe
    log("streaming ceilings")
    ceil = ceilings(torch, coot)
    for name, v in per.items():
        mix = "mix_2to1" if name.split("_")[0] in ("axpy", "z") else "read_only"
        v["ceiling"] = mix
        v["frac_of_ceiling"] = round(v["GBps"] / ceil[mix]["GBps"], 4)

    # roofline of the dominant kernel (largest share of the step)
    dom_bytes = dict((n, b) for n, b, _ in steps)[dom]
    achieved = dom_bytes / (dom_us * 1e-6) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            tj = json.load(f)
        entry = tj.get("calls", {}).get(dom)
        # the counters count only while the kernel they were taken on is unchanged
        if entry and entry.get("kernel") == kernel_names(coot, synth).get(dom):
            traffic = entry.get("bytes")

    extra = {}
    if not args.headline_only:
        # the other workloads' headline figures, measured in the same run
        log("precision: 16384^2 BF16/FP16 column sums, accu, dot")
        extra["precision_16384sq_bf16_f16"] = precision_calls(np, torch, synth, coot)
        log("batched: 10,000 matrices")
        extra["batched_10000_matrices"] = batched_calls(np, torch, synth, coot)
        log("small: 1000x1000 FP32, warm and cold")
        extra["small_1000sq_f32"] = small_calls(np, torch, synth, coot)

    cpu = None
    if not args.no_cpu:
        import oracle

        log("timing the oracle on a CPU sample")
        cpu = cpu_baseline(oracle, synth, np)

    out = {
        "metric": "fused elementwise+reduction effective GB/s vs HBM peak; speedup over unfused",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic: seeded N(0,1) vectors, 64 injected tied maxima",
        "config": {"workload": "plain method at scale: axpy, z, dot, norm, index_max on 2^28-element "
                               "FP32 and FP64 vectors (fused, one kernel per call)",
                   "n": N, "calls_per_step": len(steps)},
        "frac_of_peak": round(value / PEAK_GBS, 4),
        "unfused_ms_per_step": round(ms_unfused, 3),
        "speedup_vs_unfused": round(ms_unfused / ms_step, 3),
        "per_call": per,
        "roofline": {"bound": "hbm", "kernel": dom, "kernel_us": round(dom_us, 2), "achieved": round(achieved, 1),
                     "peak": PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_GBS, 4), "traffic": traffic},
        "cpu_baseline": cpu,
        "ceilings": ceil,
        **extra,
    }
    print(json.dumps(out), flush=True)


def costmodel_workload(args, np, torch, synth, coot):
    """Learned launch configuration: exhaustive autotuning of the random-tree
    corpus, training of the MLP on the GPU, regret on the held-out trees."""
    from paper_2308_03120_amd import costmodel as cm

    os.makedirs(args.out_dir, exist_ok=True)
    trees = synth.cfg5_trees(args.trees)
    tr_idx, te_idx = synth.cfg5_split(len(trees), int(round(len(trees) * 5 / 6)))
    t0 = time.perf_counter()
    n = cm.precompile_corpus(trees, per_module=64, workers=16)
    t_compile = time.perf_counter() - t0
    log(f"compiled {n} kernels in {t_compile:.0f} s")
    t0 = time.perf_counter()
    times, feats, default = cm.time_corpus(trees, reps=3, log=log)
    t_tune = time.perf_counter() - t0
    np.savez_compressed(os.path.join(args.out_dir, "costmodel_corpus.npz"), times=times, feats=feats,
                        default=default, train=tr_idx, test=te_idx)
    t0 = time.perf_counter()
    params, mean, std, hist = cm.train(feats[tr_idx], cm.targets(times[tr_idx]), log=log)
    t_train = time.perf_counter() - t0
    cm.save_model(os.path.join(args.out_dir, "costmodel_weights.bin"), params, mean, std)
    pred = cm.predict(params, mean, std, feats[te_idx])
    picks = pred.argmin(axis=1)
    held = cm.summarize(times[te_idx], default[te_idx], picks)
    fit = cm.summarize(times[tr_idx], default[tr_idx], cm.predict(params, mean, std, feats[tr_idx]).argmin(axis=1))
    # the model inside the library (GPU inference at plan time) against fused default and unfused
    coot.model_set(params, mean, std)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    sample = te_idx
    t_def = t_mod = t_unf = 0.0
    agree = 0
    for i in sample:
        rt = trees[i]
        red, dim, ops, out = cm.allocate(rt, torch, gen)
        agree += int(coot.model_choose(red, dim, rt.expr, ops, out) == picks[list(te_idx).index(i)])

        def run(cfg=None, unfused=False):
            if red is None:
                coot.eval(rt.expr, ops, out, cfg=cfg, unfused=unfused)
            else:
                coot.reduce(red, rt.expr, ops, out=out, dim=dim, cfg=cfg, unfused=unfused)

        def med(fn, reps=3):
            fn()
            ts = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                fn()
                b.record()
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b))
            return sorted(ts)[reps // 2]

        coot.set_tuning(coot.TUNE_DEFAULT)
        t_def += med(lambda: run())
        coot.set_tuning(coot.TUNE_MODEL)
        t_mod += med(lambda: run())
        coot.set_tuning(coot.TUNE_DEFAULT)
        t_unf += med(lambda: run(unfused=True))
        del ops, out
    out = {
        "metric": "learned launch configuration: regret vs exhaustive autotune on held-out trees",
        "value": round(held["regret_model_mean"], 5), "unit": "mean regret (t_pick/t_best - 1)",
        "higher_is_better": False, "n_gpus": 1, "data": "synthetic: 6,000 seeded random expression trees",
        "config": {"workload": "random trees, depth 1-6, 2^10-2^26 elements, F64/F32/F16/BF16; MLP 32-64-64",
                   "trees": len(trees), "train": int(len(tr_idx)), "held_out": int(len(te_idx)),
                   "configs": 64},
        "held_out": held, "train_fit": fit, "loss_history": hist,
        "end_to_end_held_out": {"trees": int(len(sample)), "model_picks_match_library_inference": agree,
                              "ms_default": round(t_def, 3), "ms_model": round(t_mod, 3), "ms_unfused": round(t_unf, 3),
                              "model_speedup_over_default": round(t_def / t_mod, 4),
                              "model_speedup_over_unfused": round(t_unf / t_mod, 4)},
        "seconds": {"compile": round(t_compile, 1), "autotune": round(t_tune, 1), "train": round(t_train, 2)},
    }
    print(json.dumps(out), flush=True)


def batched_calls(np, torch, synth, coot, reps=20, baselines=True):
    """10,000 matrices: one graph-replayed launch (through a plan and through
    the one-call entry) vs per-matrix fused launches vs unfused per-node
    launches."""
    d = synth.cfg4_inputs()
    shapes, offs = d["shapes"], d["offsets"]
    dA, dB = torch.from_numpy(d["A"]).cuda(), torch.from_numpy(d["Bp"]).cuda()
    dY = torch.zeros(d["total"], device="cuda")
    red = torch.zeros(len(shapes), device="cuda")
    es = 4
    ptrs = [[dA.data_ptr() + int(o) * es, dB.data_ptr() + int(o) * es] for o in offs]
    outs = [dY.data_ptr() + int(o) * es for o in offs]
    yshape = [[int(c), int(r)] for r, c in shapes]
    elems = int((shapes[:, 0] * shapes[:, 1]).sum())
    nbytes = 12 * elems
    Ytree, Rtree = synth.cfg4_tree(), synth.leaf(0) % synth.leaf(0)

    def plan(flags):
        return coot.BatchPlan(Ytree, [coot.F32, coot.F32], ptrs, yshape, out_ptrs=outs, red_tree=Rtree,
                              red_op="accu", red_out=red, flags=flags)

    def timed(run, reps):
        run()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record()
        for _ in range(reps):
            run()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps, (time.perf_counter() - t0) / reps * 1e3

    one = plan(0)
    t_one, w_one = timed(one.run, max(10, reps))
    us_one = event_stats(torch, one.run)[0]
    desc = coot.BatchDescriptor(Ytree, [coot.F32, coot.F32], ptrs, yshape, out_ptrs=outs, red_tree=Rtree,
                                red_op="accu", red_out=red)
    t_call, w_call = timed(lambda: coot.eval_batched(desc), max(10, reps))
    nog = plan(coot.BATCH_NO_GRAPH)
    t_nog, _ = timed(nog.run, max(10, reps))
    per = unf = None
    t_per = t_unf = float("nan")
    if baselines:
        per = plan(coot.BATCH_PER_ITEM)
        t_per, w_per = timed(per.run, 3)
        unf = plan(coot.BATCH_UNFUSED)
        t_unf, w_unf = timed(unf.run, 1)
    for p in (one, nog, per, unf):
        if p is not None:
            p.close()
    return {
        "elements": elems, "algorithmic_bytes": nbytes,
        "us_one_replay": round(us_one, 2),
        "GBps_one_replay": round(nbytes / (us_one * 1e-6) / 1e9, 1),
        "ms_one_launch_graph": round(t_one, 4), "ms_one_launch_direct": round(t_nog, 4),
        "ms_eval_batched_call": round(t_call, 4), "ms_eval_batched_wall": round(w_call, 4),
        "ms_per_matrix_launches": None if per is None else round(t_per, 3),
        "ms_unfused_per_node": None if unf is None else round(t_unf, 3),
        "speedup_vs_per_matrix": None if per is None else round(t_per / t_one, 2),
        "speedup_vs_unfused": None if unf is None else round(t_unf / t_one, 2),
        "frac_of_peak": round(nbytes / (us_one * 1e-6) / 1e9 / PEAK_GBS, 4),
    }


def batched_workload(args, np, torch, synth, coot):
    """10,000 matrices: one graph-replayed launch vs per-matrix fused launches vs unfused per-node launches."""
    r = batched_calls(np, torch, synth, coot, reps=args.steps, baselines=not args.no_baselines)
    out = {
        "metric": "batched fused evaluation effective GB/s (one graph-replayed launch)",
        "value": r["GBps_one_replay"], "unit": "GB/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic: seeded U[-1,1], 10,000 matrices, rows/cols log-uniform in [8, 512]",
        "config": {"workload": "Y_i = trans(A_i) + 0.5*B_i', r_i = accu(Y_i % Y_i) for 10,000 matrices",
                   "elements": r["elements"], "algorithmic_bytes": r["algorithmic_bytes"]},
        **{k: v for k, v in r.items() if k not in ("elements", "algorithmic_bytes")},
    }
    print(json.dumps(out), flush=True)


def cfg3_device_inputs(torch, dt, tdt, n_rows=16384, n_cols=16384, seed=2308_3120_3):
    """The precision workload's two matrices drawn on the device with a seeded
    torch generator: |x| = exp(3 z), z ~ N(0,1) clipped to +-ln(1e4)/3, random
    signs, stored (round to nearest even) in the 16-bit type; column-major.
    The same distribution as the host recipe the parity tests use, drawn in
    milliseconds instead of a minute (timing only: HBM-bound calls whose cost
    does not depend on the values)."""
    import math

    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    clip = math.log(1e4) / 3.0
    mats = []
    for _ in range(2):
        z = torch.randn(n_cols, n_rows, generator=g, device="cuda").clamp_(-clip, clip)
        sign = torch.randint(0, 2, (n_cols, n_rows), generator=g, device="cuda").float().mul_(2.0).sub_(1.0)
        mats.append((sign * torch.exp(3.0 * z)).to(tdt).t())
        del z, sign
    return mats


def precision_calls(np, torch, synth, coot, host_inputs=False):
    """16384 x 16384 BF16/FP16: column sums, accu, dot, plain vs compensated
    FP32 accumulation; median single-call device times."""
    res = {}
    for dt, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        if host_inputs:
            d = synth.cfg3_inputs(dt)
            A = torch.from_numpy(np.ascontiguousarray(d["A"].data.T).view(np.int16)).view(tdt).cuda().t()
            B = torch.from_numpy(np.ascontiguousarray(d["B"].data.T).view(np.int16)).view(tdt).cuda().t()
            del d
        else:
            A, B = cfg3_device_inputs(torch, dt, tdt)
        x, y = synth.leaves(2)
        calls = (("colsum", lambda pw: coot.reduce("sum", x, [A], dim=0, pairwise=pw), 2),
                 ("accu", lambda pw: coot.reduce("accu", x, [A], pairwise=pw), 2),
                 ("dot", lambda pw: coot.reduce("dot", x % y, [A, B], pairwise=pw), 4))
        for name, fn, nb in calls:  # compile and load every kernel before timing any
            for pw in (False, True):
                fn(pw)
        torch.cuda.synchronize()
        for name, fn, nb in calls:
            for pw in (False, True):
                us = event_stats(torch, lambda: fn(pw))[0]
                res[f"{name}_{dt}_{'pairwise' if pw else 'kahan'}"] = {
                    "us": round(us, 2), "GBps": round(nb * A.numel() / (us * 1e-6) / 1e9, 1)}
        del A, B
        torch.cuda.empty_cache()
    return res


def precision_workload(args, np, torch, synth, coot):
    """16384 x 16384 BF16/FP16: column sums, accu, dot, plain vs compensated FP32 accumulation."""
    res = precision_calls(np, torch, synth, coot, host_inputs=True)
    gb = [v["GBps"] for k, v in res.items() if "kahan" in k]
    out = {"metric": "compensated FP32 reductions of 16-bit storage, effective GB/s", "value": min(gb),
           "unit": "GB/s (slowest compensated call)", "n_gpus": 1, "higher_is_better": True, "dtype": "bf16,f16",
           "data": "synthetic: |x| = exp(3z), z~N(0,1) clipped to [1e-4, 1e4], random signs, 16384^2",
           "per_call": res}
    print(json.dumps(out), flush=True)


def ceilings(torch, coot, nbytes=1 << 30):
    """Median device time and GB/s of the library's streaming probes over
    `nbytes` per stream: read only, write only, 1:1 copy, 2 reads : 1 write,
    each the fastest of four launch shapes (threads x vectors per thread:
    256x4, 64x1, 256x1, 128x2); plus the 2:1 ceiling derived from the
    read-only and write-only rates (time of 2 read streams at the read rate
    plus 1 write stream at the write rate)."""
    src = torch.zeros(2 * nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    res = {}
    shapes = ("256x4", "64x1", "256x1", "128x2")
    for name, kind, moved in (("read_only", coot.PROBE_READ, nbytes), ("write_only", coot.PROBE_WRITE, nbytes),
                              ("copy_1to1", coot.PROBE_COPY, 2 * nbytes),
                              ("mix_2to1", coot.PROBE_READ2_WRITE1, 3 * nbytes)):
        per = [event_stats(torch, lambda: coot.bandwidth_probe(kind | (sh << 8), dst, src, nbytes))[0]
               for sh in range(4)]
        b = min(range(4), key=lambda i: per[i])
        res[name] = {"us": round(per[b], 2), "GBps": round(moved / (per[b] * 1e-6) / 1e9, 1), "shape": shapes[b],
                     "GBps_by_shape": {shapes[i]: round(moved / (per[i] * 1e-6) / 1e9, 1) for i in range(4)}}
    r, w = res["read_only"]["GBps"], res["write_only"]["GBps"]
    res["mix_2to1_derived"] = {"GBps": round(3.0 / (2.0 / r + 1.0 / w), 1)}
    res["bytes_per_stream"] = nbytes
    del src, dst
    torch.cuda.empty_cache()
    return res


def event_stats(torch, fn, reps=21, between=None):
    """median, min and p90 in microseconds of single-call HIP-event timings.  A
    spin on the GPU (no memory traffic, about 0.4 ms) is queued before the start
    event, so the host's preparation of the call -- a dozen launches for the
    unfused per-node forms -- overlaps it and the interval is the device's time
    for the call."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        if between is not None:
            between()
        torch.cuda._sleep(1000000)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) * 1e3)
    ts.sort()
    return ts[len(ts) // 2], ts[0], ts[int(0.9 * (len(ts) - 1))]


def tiled_workload(args, np, torch, synth, coot):
    """Transposed reads: Y = trans(A) + 0.5*B and accu(trans(A) % B) on square and thin values;
    generator and view calls (A + eye, a scaled submatrix, trace)."""
    x, y = synth.leaves(2)
    res = {}
    cases = (("square_16384x16384_f32", 16384, 16384, torch.float32),
             ("square_16384x8192_f64", 16384, 8192, torch.float64),
             ("square_16384x16384_bf16", 16384, 16384, torch.bfloat16),
             ("thin_2x67108864_f32", 2, 1 << 26, torch.float32),
             ("thin_8388608x12_f32", 1 << 23, 12, torch.float32))
    for name, r, c, tdt in cases:
        # Y is r x c; A is c x r (read transposed), B is r x c
        A = torch.rand(r, c, dtype=tdt, device="cuda").t()   # column-major c x r
        B = torch.rand(c, r, dtype=tdt, device="cuda").t()   # column-major r x c
        Y = torch.empty(c, r, dtype=tdt, device="cuda").t()
        es = A.element_size()
        for call, fn, bpe in (("add", lambda: coot.eval(synth.trans(x) + 0.5 * y, [A, B], Y), 3),
                              ("accu", lambda: coot.reduce("accu", synth.trans(x) % y, [A, B]), 2)):
            med, mn, p90 = event_stats(torch, fn)
            gbs = bpe * es * r * c / (med * 1e-6) / 1e9
            res[f"{call}_{name}"] = {"us_median": round(med, 1), "us_min": round(mn, 1), "us_p90": round(p90, 1),
                                     "GBps": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_GBS, 4)}
        del A, B, Y
        torch.cuda.empty_cache()
    # generator and view calls on a 16384^2 FP32 matrix: A + eye (reads A only,
    # tiled: eye needs rows and columns), a submatrix view (rows 1..16383,
    # columns 1..16383: a strided operand) scaled into a second view, and trace
    # (16384 strided elements, one per cache line: latency, not bandwidth)
    n = 16384
    A = torch.rand(n, n, device="cuda").t()
    B2 = torch.rand(n, n, device="cuda").t()
    Y = torch.empty(n, n, device="cuda").t()
    X0 = synth.leaf(0)
    for call, fn, nbytes in (("add_eye_16384x16384_f32", lambda: coot.eval(X0 + synth.leaf(1), [A, coot.eye(n, n)], Y),
                              8 * n * n),
                             ("scale_submat_16383x16383_f32",
                              lambda: coot.eval(X0 * 2.0, [coot.submat(A, 1, 1, n - 1, n - 1)],
                                                coot.submat(Y, 0, 0, n - 2, n - 2)), 8 * (n - 1) * (n - 1)),
                             # both views one element off their lines (the tile grid follows the output)
                             ("scale_submat_offset_out_16383x16383_f32",
                              lambda: coot.eval(X0 * 2.0, [coot.submat(A, 1, 1, n - 1, n - 1)],
                                                coot.submat(Y, 1, 1, n - 1, n - 1)), 8 * (n - 1) * (n - 1)),
                             # a transposed read and a straight read one element off their
                             # lines, into an aligned view (64 x 64 tiles)
                             ("add_trans_submat_offset_in_16383x16383_f32",
                              lambda: coot.eval(synth.trans(X0) + 0.5 * synth.leaf(1),
                                                [coot.submat(A, 1, 1, n - 1, n - 1), coot.submat(B2, 1, 1, n - 1, n - 1)],
                                                coot.submat(Y, 0, 0, n - 2, n - 2)), 12 * (n - 1) * (n - 1)),
                             ("trace_16384x16384_f32", lambda: coot.trace(A), 4 * n)):
        med, mn, p90 = event_stats(torch, fn)
        gbs = nbytes / (med * 1e-6) / 1e9
        res[call] = {"us_median": round(med, 1), "us_min": round(mn, 1), "us_p90": round(p90, 1),
                     "GBps": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_GBS, 4)}
    del A, B2, Y
    torch.cuda.empty_cache()
    # the tiled kernels' access pattern without their arithmetic: 16384-row
    # FP32 streams of 1 GiB moved in tiles of 64..4096 rows (a wave access is
    # 64 rows of one column; the run down a column is the tile's height)
    nbytes = 1 << 30
    src = torch.zeros(2 * nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    ceil = {}
    for name, kind, moved in (("copy", coot.PROBE_TILED_COPY, 2 * nbytes),
                              ("mix_2to1", coot.PROBE_TILED_READ2_WRITE1, 3 * nbytes)):
        for sh, rows in enumerate((64, 256, 1024, 4096)):
            med = event_stats(torch, lambda: coot.bandwidth_probe(kind | (sh << 8), dst, src, nbytes))[0]
            ceil[f"{name}_{rows}_row_runs"] = {"us": round(med, 1), "GBps": round(moved / (med * 1e-6) / 1e9, 1)}
    del src, dst
    torch.cuda.empty_cache()
    gb = [v["GBps"] for k, v in res.items() if not k.startswith("trace")]
    print(json.dumps({"metric": "transposed-read kernels, effective GB/s", "value": min(gb),
                      "unit": "GB/s (slowest case)", "n_gpus": 1, "higher_is_better": True, "dtype": "f32,f64",
                      "data": "synthetic: torch.rand on the device", "per_call": res,
                      "tiled_ceilings_16384_rows_f32": ceil}), flush=True)


def small_calls(np, torch, synth, coot):
    """The 1000 x 1000 FP32 calls: device time (events; warm = inputs in the 256 MB
    last-level cache, cold = a 512 MiB write between calls) and the paper-style host
    wall clock around call + synchronise (the host's preparation included); fused
    and unfused."""
    mats = synth.cfg1_inputs()
    names = "ABCD"
    dev = [torch.from_numpy(np.ascontiguousarray(mats[k].data.T)).cuda().t() for k in names]
    t = synth.cfg1_trees()
    Y = torch.empty(1000, 1000, device="cuda").t()
    scratch = torch.empty(1 << 27, device="cuda")

    def flush():
        scratch.fill_(1.0)

    calls = (("Y", lambda u: coot.eval(t["Y"], dev, Y, unfused=u), 20),
             ("accu_AB", lambda u: coot.reduce("accu", t["accu_AB"], dev, unfused=u), 8),
             ("sum_A_dim0", lambda u: coot.reduce("sum", t["sumA"], dev, dim=0, unfused=u), 4),
             ("index_max_absB", lambda u: coot.reduce("index_max", t["absB"], dev, unfused=u), 4))
    res = {}
    for name, fn, bpe in calls:
        for u in (False, True):
            warm = event_stats(torch, lambda: fn(u))
            cold = event_stats(torch, lambda: fn(u), between=flush)
            fn(u)
            torch.cuda.synchronize()
            walls = []
            for _ in range(21):
                t0 = time.perf_counter()
                fn(u)
                torch.cuda.synchronize()
                walls.append((time.perf_counter() - t0) * 1e6)
            walls.sort()
            res[f"{name}_{'unfused' if u else 'fused'}"] = {
                "us_warm_median": round(warm[0], 1), "us_cold_median": round(cold[0], 1),
                "us_wall_median": round(walls[10], 1), "GBps_warm": round(bpe * 1e6 / (warm[0] * 1e-6) / 1e9, 1)}
    del scratch
    torch.cuda.empty_cache()
    return res


def small_workload(args, np, torch, synth, coot):
    res = small_calls(np, torch, synth, coot)
    tot_f = sum(v["us_wall_median"] for k, v in res.items() if k.endswith("_fused"))
    tot_u = sum(v["us_wall_median"] for k, v in res.items() if k.endswith("_unfused"))
    print(json.dumps({"metric": "1000x1000 FP32 calls, host wall clock per call set (call + synchronise)",
                      "value": round(tot_f, 1), "unit": "us", "higher_is_better": False, "n_gpus": 1, "dtype": "f32",
                      "data": "synthetic: seeded U[-1,1] (D: U[-4,4]), 1000x1000",
                      "speedup_vs_unfused": round(tot_u / tot_f, 3), "per_call": res}), flush=True)


def stats_workload(args, np, torch, synth, coot):
    """Statistics and predicate reductions on the 2^28-element FP32 and FP64
    vectors of the scale workload and per column of a 16384^2 FP32 matrix,
    against the plain sum of the same data; count(x > 0.3) also unfused
    (predicate materialised, then summed); and element-wise trees of Table 7
    functions (sin, cos, pow, floor), fused and unfused."""
    x = synth.leaf(0)
    res = {}
    for dt, tdt in (("f32", torch.float32), ("f64", torch.float64)):
        d = synth.cfg2_inputs(dt, n=N)
        X = torch.from_numpy(d["x"]).cuda()
        Yv = torch.from_numpy(d["y"]).cuda()
        del d
        Z = torch.empty_like(X)
        es = X.element_size()
        y = synth.leaf(1)
        # Table 7 functions: algorithmic bytes = operands read + output written
        for name, fn, nbytes in (
                ("sin_x_schur_cos_y", lambda: coot.eval(synth.sin(x) % synth.cos(y), [X, Yv], Z), 3 * es * N),
                ("sin_x_schur_cos_y_unfused",
                 lambda: coot.eval(synth.sin(x) % synth.cos(y), [X, Yv], Z, unfused=True), 3 * es * N),
                ("pow_x_2.5", lambda: coot.eval(synth.pow_(synth.abs_(x), 2.5), [X], Z), 2 * es * N),
                ("floor_4x", lambda: coot.eval(synth.floor(x * 4.0), [X], Z), 2 * es * N)):
            med, mn, p90 = event_stats(torch, fn)
            res[f"{name}_{dt}"] = {"us_median": round(med, 1), "us_min": round(mn, 1), "us_p90": round(p90, 1),
                                   "GBps": round(nbytes / (med * 1e-6) / 1e9, 1)}
        del Yv, Z
        nb = X.element_size() * N
        calls = (("accu", lambda: coot.reduce("accu", x, [X])),
                 ("mean", lambda: coot.reduce("mean", x, [X])),
                 ("var", lambda: coot.reduce("var", x, [X])),
                 ("stddev", lambda: coot.reduce("stddev", x, [X])),
                 ("count_gt", lambda: coot.reduce("count", x > 0.3, [X])),
                 ("all_gt", lambda: coot.reduce("all", x > -10.0, [X])),
                 ("any_gt", lambda: coot.reduce("any", x > 7.9, [X])),
                 ("count_gt_unfused", lambda: coot.reduce("count", x > 0.3, [X], unfused=True)))
        for name, fn in calls:
            med, mn, p90 = event_stats(torch, fn)
            res[f"{name}_{dt}"] = {"us_median": round(med, 1), "us_min": round(mn, 1), "us_p90": round(p90, 1),
                                   "GBps": round(nb / (med * 1e-6) / 1e9, 1)}
        del X
        torch.cuda.empty_cache()
    A = torch.rand(16384, 16384, device="cuda").t()
    nb = 4 * A.numel()
    for name, fn in (("colsum", lambda: coot.reduce("sum", x, [A], dim=0)),
                     ("colmean", lambda: coot.reduce("mean", x, [A], dim=0)),
                     ("colvar", lambda: coot.reduce("var", x, [A], dim=0)),
                     ("rowvar", lambda: coot.reduce("var", x, [A], dim=1)),
                     ("colcount_gt", lambda: coot.reduce("count", x > 0.5, [A], dim=0))):
        med, mn, p90 = event_stats(torch, fn)
        res[f"{name}_16384x16384_f32"] = {"us_median": round(med, 1), "us_min": round(mn, 1),
                                          "us_p90": round(p90, 1), "GBps": round(nb / (med * 1e-6) / 1e9, 1)}
    del A
    fused = [v["GBps"] for k, v in res.items() if "unfused" not in k]
    print(json.dumps({"metric": "statistics, predicate reductions and Table 7 functions, effective GB/s",
                      "value": min(fused),
                      "unit": "GB/s (slowest fused call)", "n_gpus": 1, "higher_is_better": True,
                      "dtype": "f32,f64", "data": "synthetic: seeded N(0,1) vectors; torch.rand matrix",
                      "per_call": res}), flush=True)


def kernel_names(coot, synth):
    """Generated kernel behind every benchmark call (the name hashes the kernel
    text).  Host only: operand descriptors without memory, 256-byte aligned
    like the device buffers."""
    G = 1 << 40
    names = {}
    for dt in ("f32", "f64"):
        X = coot.fake_operand(N, 1, dt, ptr=G)
        Y = coot.fake_operand(N, 1, dt, ptr=2 * G)
        Z = coot.fake_operand(N, 1, dt, ptr=3 * G)
        for nm, kind, tree, _ in ops_of(synth):
            if kind == "eval":
                ops, out, red = ([X, Y], Y, None) if nm == "axpy" else ([X, Y], Z, None)
            else:
                ops = [X, Y] if kind == "dot" else [X]
                out = coot.fake_operand(1, 1, "u64" if kind == "index_max" else dt, ptr=4 * G)
                red = kind
            src = coot.kernel_source(red, -1, tree, ops, out)
            m = re.search(r'extern "C" __global__ void __launch_bounds__\(\d+\) (coot_[a-z]+_[0-9a-f]{16})\(', src)
            names[f"{nm}_{dt}"] = m.group(1) if m else None
    return names


def traffic_from(fetch_csv, write_csv, out_path):
    """HBM bytes per launch of every benchmark kernel from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the
    same counter reads for the library's plain copy of a known size."""
    import csv
    from collections import defaultdict

    import synth
    from paper_2308_03120_amd import coot

    def load(p, counter):
        agg = defaultdict(list)
        for r in csv.DictReader(open(p)):
            if r["Counter_Name"] == counter:
                agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return agg

    f, w = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    copy = [k for k in f if "coot_copy16" in k]
    assert copy, "the counter runs need --calibrate-copy"
    copy_kib = (1 << 30) / 1024.0   # 1 GiB read and 1 GiB written per copy
    f_scale = copy_kib / (sum(f[copy[0]]) / len(f[copy[0]]))
    w_scale = copy_kib / (sum(w[copy[0]]) / len(w[copy[0]]))
    names = kernel_names(coot, synth)
    calls = {}
    for call, kname in names.items():
        if kname in f and kname in w:
            fk = sum(f[kname]) / len(f[kname]) * f_scale
            wk = sum(w[kname]) / len(w[kname]) * w_scale
            calls[call] = {"kernel": kname, "fetch_bytes": round(fk * 1024), "write_bytes": round(wk * 1024),
                           "bytes": round((fk + wk) * 1024)}
    out = {"fetch_scale": f_scale, "write_scale": w_scale, "calls": calls,
           "source": [os.path.basename(fetch_csv), os.path.basename(write_csv)]}
    with open(out_path, "w") as fo:
        json.dump(out, fo, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
