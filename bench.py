"""Benchmark: literal-gradient evaluations per second on one MI355X.

Workload: the mixed hybrid instance n = 2000 (8000 OR clauses of length
3..7, 500 XOR of length 3..20, 200 at-least-t of length 10..100), 1024
restarts, FP32, seeded synthetic data.  One step is one pass of the whole
per-batch hot path: objective and gradient of every constraint at every
restart (with the deterministic reduction into the gradient), the projected
step, the exact round-and-check, and the adaptive-weight update.

value = nnz * B / (seconds per step): one "literal-gradient evaluation" is
one (literal occurrence, restart) pair whose gradient contribution and the
objective are produced.

The JSON line carries `roofline` for the kernel that takes the most time
(timed live with HIP events on the stream it runs on) and `cpu_baseline`,
the FP64 oracle timed on the host cores on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "literal-gradient evals/s at 1 GPU (vs FP64 oracle); time-to-solve learned vs random"
UNIT = "literal-gradient evals/s"
HBM_PEAK_GBS = 8000.0
# FP32 vector FMA without packed math (disabled for all device code here) and
# FP64 vector FMA: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
VALU_PEAK_PACKED_TFLOPS = 157.3


WORKLOADS = {
    "mixed2000": {"gen": "config2", "seed": 2000, "B": 1024,
                  "desc": "mixed hybrid SAT n=2000: 8000 OR (len 3-7), 500 XOR (len 3-20), "
                          "200 at-least-t (len 10-100), {B} restarts, FP32"},
    "large": {"gen": "config3", "seed": 3000, "B": 256,
              "desc": "large hybrid SAT n=100000: 420000 3-SAT, 10000 XOR (len 8-64), 2000 at-least-t "
                      "(len 128-512; FP64 beyond 256), {B} restarts, FP32"},
    "uf50": {"gen": "config1", "seed": 1000, "B": 1,
             "desc": "random 3-SAT n=50, m=213 (latency: one restart), {B} restart(s), FP32"},
    "large3sat": {"gen": "config3a", "seed": 3000, "B": 256,
                  "desc": "random 3-SAT n=100000, m=420000 (the 3-SAT part of the large instance), "
                          "{B} restarts, FP32"},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--seed", type=int, default=2000)
    ap.add_argument("--restarts", type=int, default=0, help="restarts (0: the workload's own, 1024 for the default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tts", action="store_true",
                    help="skip the time-to-solve comparison (learned vs uniform initialisation)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--eta", type=float, default=0.05)
    ap.add_argument("--workload", default="mixed2000", choices=sorted(WORKLOADS),
                    help="instance family (the default is the headline configuration)")
    ap.add_argument("--chunk", type=int, default=20,
                    help="iterations per graph replay in the headline loop")
    ap.add_argument("--mode", default="auto", choices=["auto", "per_bin", "group_all", "group_dft"],
                    help="launch structure of the evaluation (auto: chosen by the autotuner)")
    ap.add_argument("--serial", action="store_true",
                    help="launch every bin on the caller's stream (no concurrent bins)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of tuned tile shapes (read if present, written after tuning)")
    ap.add_argument("--rq1", action="store_true",
                    help="instead of the step benchmark: the paper's RQ1 gradient timing (seven formulas, "
                         "10000 random points, time per point in FP32 and FP64, the FP64 oracle beside it)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def measured_traffic(roof):
    """HBM bytes per launch of the grouped evaluation kernel from the committed
    rocprofv3 counter summary, if the kernel sources are unchanged since the
    counters were taken (else None)."""
    if not roof.get("kernel", "").startswith("grouped evaluation launch"):
        return None
    from paper_2308_15020_amd.profsum import kernel_source_hash
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        "eval_group_mixed2000_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash() or "traffic_bytes_per_launch" not in kv:
        return None
    return float(kv["traffic_bytes_per_launch"])


def time_to_solve():
    """The second half of the metric: learned initialisation against uniform
    restarts on planted instances of the mixed n = 2000 shape with 200 XOR
    constraints (50 training instances, 100 test instances, 256 restarts, 60
    rounds of 40 steps); the harness's log goes to stderr."""
    import contextlib
    from paper_2308_15020_amd import tts
    argv = ["--train", "50", "--test", "100", "--planted", "--n-xor", "200", "--rounds", "60", "--T", "40",
            "--eta", "0.3"]
    t0 = time.perf_counter()
    with contextlib.redirect_stdout(sys.stderr):
        s = tts.main(argv)
    return {"instances": s["instances"], "family": "planted, mixed n=2000 shape, 200 XOR", "B": s["B"],
            "solve_rate": s["solve_rate"], "both_solved": s["both_solved"],
            "median_ms": {k: (None if v is None else v * 1e3) for k, v in s["median_s"].items()},
            "mean_ms": {k: (None if v is None else v * 1e3) for k, v in s["mean_s"].items()},
            "median_rounds": s["median_rounds"],
            "cactus_at_lower_solve_rate": {
                (k[:-2] + "_ms" if k.endswith("_s") else k): (v * 1e3 if k.endswith("_s") and v is not None else v)
                for k, v in s["cactus_at_lower_solve_rate"].items()},
            "learned_vs_polarity_median_ms": [None if v is None else v * 1e3
                                              for v in s["learned_vs_polarity_median_s"]],
            "harness_seconds": time.perf_counter() - t0}


def cpu_baseline(inst, x_np, budget_s=12.0):
    """FP64 oracle on the host: the same instance and points (all restarts
    when one pass takes under a third of the budget, else a leading subset),
    passes repeated until about `budget_s` of work; median pass time."""
    import numpy as np

    import oracle
    n, B = x_np.shape
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    Bp = max(1, min(B, threads))
    probe = np.ascontiguousarray(x_np[:, :Bp].astype(np.float64))
    t0 = time.perf_counter()
    oracle.eval_batch(inst, probe, want_g=True, nthreads=threads)
    t_probe = max(time.perf_counter() - t0, 1e-6)
    Bs = min(B, Bp * max(1, int(budget_s / 3.0 / t_probe)))
    sub = np.ascontiguousarray(x_np[:, :Bs].astype(np.float64))
    times = []
    used = 1
    t_start = time.perf_counter()
    while len(times) < 3 or (time.perf_counter() - t_start < budget_s and len(times) < 1000):
        t0 = time.perf_counter()
        r = oracle.eval_batch(inst, sub, want_g=True, nthreads=threads)
        times.append(time.perf_counter() - t0)
        used = r["threads"]
    t = float(np.median(times))
    return {"value": inst.nnz * Bs / t, "unit": UNIT, "cores": int(used), "kind": "oracle",
            "sample": f"{Bs} of {B} restarts of the same instance and points, F and gradient in FP64 "
                      f"(count-lattice recursion for at-least-t, closed forms for OR/XOR); median of "
                      f"{len(times)} passes, {sum(times):.1f} s in total"}


def rq1(args, dev, points=10000, reps=20):
    """Average time of one objective + gradient evaluation per random point
    for the paper's seven RQ1 formulas (its Benchmark Details lists their
    counts and lengths; n = 1000 and t = len/2 are not given there): all
    points as restarts of one batch, FP32 and FP64 evaluation, HIP events over
    `reps` evaluations; the FP64 oracle on the host beside it (a subset of the
    points, all threads and one thread)."""
    import numpy as np
    import torch

    import oracle
    import workloads
    from paper_2308_15020_amd import Plan, Problem
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rows = []
    for name in workloads.RQ1_SHAPES:
        inst = workloads.rq1(name)
        x_np = workloads.points(inst.n_vars, points, workloads.point_seed(6000))
        prob = Problem(inst, device=0)
        plan = Plan(prob, points, autotune=not args.no_autotune, tune_cache=args.tune_cache)
        row = {"formula": name, "n": inst.n_vars, "m": inst.m, "nnz": inst.nnz, "points": points}
        for dt, key in ((torch.float32, "gpu_f32_us_per_point"), (torch.float64, "gpu_f64_us_per_point")):
            x = torch.from_numpy(x_np).to(dev, dt)
            out = plan.eval(x)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                plan.eval(x, out=out)
            e1.record()
            torch.cuda.synchronize()
            row[key] = e0.elapsed_time(e1) * 1e3 / reps / points
        sub = np.ascontiguousarray(x_np[:, :256].astype(np.float64))
        for nt, key in ((threads, "oracle_us_per_point"), (1, "oracle_1thread_us_per_point")):
            times = []
            for _ in range(3):
                t0 = time.perf_counter()
                oracle.eval_batch(inst, sub, want_g=True, nthreads=nt)
                times.append(time.perf_counter() - t0)
            row[key] = float(np.median(times)) * 1e6 / sub.shape[1]
        row["oracle_threads"] = threads
        rows.append(row)
        plan.close()
        prob.close()
    print(json.dumps({"metric": "RQ1 gradient computation time per random point", "unit": "us",
                      "data": "synthetic", "rows": rows}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU path "
                                   "(sharding over restarts) is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import workloads
    from paper_2308_15020_amd import Plan, Problem

    dev = torch.device("cuda:0")
    if args.rq1:
        return rq1(args, dev)
    wl = WORKLOADS[args.workload]
    seed = args.seed if args.workload == "mixed2000" else wl["seed"]
    inst = getattr(workloads, wl["gen"])(seed)
    B = args.restarts if args.restarts else wl["B"]
    x_np = workloads.points(inst.n_vars, B, workloads.point_seed(seed))
    prob = Problem(inst, device=0)
    plan = Plan(prob, B, autotune=not args.no_autotune, tune_cache=args.tune_cache, side_streams=not args.serial,
                mode=args.mode)
    x0 = torch.from_numpy(x_np).to(dev)
    x = x0.clone()
    out = {"F": torch.empty(B, device=dev), "grad": torch.empty(inst.n_vars, B, device=dev)}
    U = torch.empty(inst.m, dtype=torch.int32, device=dev)
    n_sat = torch.empty(B, dtype=torch.int32, device=dev)

    import ctypes as C
    from paper_2308_15020_amd._lib import check, lib
    L = lib()
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    ph = plan.handle
    p = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    eta = C.c_float(args.eta)

    def step():
        # objective, gradient, exact check of x_t and the projected step to
        # x_{t+1} in one pass, then the adaptive weights from the check
        check(L.ffsat_eval_step(ph, p(x), eta, p(out["F"]), p(n_sat), p(U), stream))
        check(L.ffsat_erwa_update(ph, p(U), C.c_float(0.4), stream))

    if args.copy_mib > 0:
        # a plain elementwise kernel of known size: reads and writes copy_mib MiB
        src = torch.ones(args.copy_mib * 262144, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    x.copy_(x0)
    prob.set_weights(inst.weights_or_ones())
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_read(reset=True)
    plan.profile(False)
    # the same iterations without timing events, for the headline number:
    # replayed from a captured graph (ffsat_run_iters), chunk steps at a time
    x.copy_(x0)
    prob.set_weights(inst.weights_or_ones())
    chunk = max(1, min(args.chunk, args.steps))
    while args.steps % chunk:                                # one graph for the whole loop
        chunk -= 1
    outs = {"F": out["F"], "n_sat": n_sat, "U": U}
    plan.run_iters(x, chunk, args.eta, 0.4, out=outs)          # capture outside the timed region
    x.copy_(x0)
    prob.set_weights(inst.weights_or_ones())
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    done = 0
    while done < args.steps:
        c = min(chunk, args.steps - done)
        plan.run_iters(x, c, args.eta, 0.4, out=outs)
        done += c
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ms_per_step = (t3 - t2) * 1e3 / args.steps
    value = inst.nnz * B / (ms_per_step / 1e3)

    desc = plan.describe()
    bins = desc["bins"]["f32"]
    kern = [k for k in prof["kernels"] if k["io"] == "f32"]
    dom = max(kern, key=lambda k: k["total_ms"])
    avg_s = dom["avg_ms"] / 1e3
    if dom["bin"] == -2:
        # the grouped launch: every bin in the group; bound by whichever
        # peak its algorithmic work needs longer on
        grp = [b for b in bins if b["in_group"]]
        flops = sum(b["flops_per_restart"] for b in grp) * B
        nbytes = sum(b["bytes_per_restart"] for b in grp) * B
        alu_bound = flops / (VALU_PEAK_TFLOPS * 1e12) >= nbytes / (HBM_PEAK_GBS * 1e9)
        n_dft = sum(1 for b in grp if b["class"] == "dft")
        label = (f"grouped evaluation launch ({len(grp)} bins, {n_dft} root-of-unity, "
                 f"{sum(b['count'] for b in grp)} constraints)")
        if alu_bound:
            achieved = flops / avg_s / 1e12
            roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / VALU_PEAK_TFLOPS, "traffic": None, "kernel": label,
                    "avg_launch_ms": dom["avg_ms"], "flops_per_launch": flops, "bytes_per_launch": nbytes,
                    "frac_of_packed_fp32_peak": achieved / VALU_PEAK_PACKED_TFLOPS}
        else:
            achieved = nbytes / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": label,
                    "avg_launch_ms": dom["avg_ms"], "flops_per_launch": flops, "bytes_per_launch": nbytes}
    elif dom["bin"] >= 0:
        bd = bins[dom["bin"]]
        if bd["class"] == "dft":
            achieved = bd["flops_per_restart"] * B / avg_s / 1e12
            roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / VALU_PEAK_TFLOPS, "traffic": None,
                    "kernel": f"eval bin {dom['bin']} ({bd['class']}, {bd['ct']}, seg {bd['seg']}, "
                              f"L {bd['L']}, {bd['count']} constraints, len <= {bd['maxk']})",
                    "avg_launch_ms": dom["avg_ms"],
                    "frac_of_packed_fp32_peak": achieved / VALU_PEAK_PACKED_TFLOPS}
        else:
            achieved = bd["bytes_per_restart"] * B / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "kernel": f"eval bin {dom['bin']} ({bd['class']}, len <= {bd['maxk']})",
                    "avg_launch_ms": dom["avg_ms"]}
    else:
        # the gradient reduction: 4 B per literal slot read + 4 B per point read and written
        nbytes = (4.0 * inst.nnz + 8.0 * inst.n_vars) * B
        achieved = nbytes / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "gradient reduction + step",
                "avg_launch_ms": dom["avg_ms"], "bytes_per_launch": nbytes}
    roof["traffic"] = measured_traffic(roof)
    kernels = []
    for k in sorted(kern, key=lambda k: -k["total_ms"]):
        name = "reduce" if k["bin"] == -1 else "grouped eval" if k["bin"] == -2 else (
            f"bin{k['bin']}:{bins[k['bin']]['class']}/{bins[k['bin']]['ct']}/L{bins[k['bin']]['L']}"
            f"/k<={bins[k['bin']]['maxk']}")
        ent = {"kernel": name, "avg_ms": round(k["avg_ms"], 5),
               "share": round(k["total_ms"] / sum(q["total_ms"] for q in kern), 4)}
        if k["bin"] >= 0:
            # algorithmic rates of one bin (launched beside others: shares the chip)
            bd = bins[k["bin"]]
            sec = k["avg_ms"] / 1e3
            ent["alg_GBps"] = round(bd["bytes_per_restart"] * B / sec / 1e9, 1)
            ent["alg_TFLOPps"] = round(bd["flops_per_restart"] * B / sec / 1e12, 2)
            ent["constraints"] = bd["count"]
        kernels.append(ent)

    res = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["desc"].format(B=B),
                   "n_vars": inst.n_vars, "n_cons": inst.m, "nnz": inst.nnz, "restarts": B,
                   "step": "objective + gradient + exact round-and-check of x_t (one pass), ERWA weight "
                           "update, projected step",
                   "iterations_per_graph_replay": chunk,
                   "eager_events_ms_per_step": (t1 - t0) * 1e3 / args.steps},
        "roofline": roof,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(inst, x_np)
    if not args.no_tts and args.workload == "mixed2000":
        res["time_to_solve"] = time_to_solve()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
