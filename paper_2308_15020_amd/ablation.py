"""Basis ablation on the device: the paper's unit-circle form against the
bounded basis, per constraint length, point distribution and precision.

    python -m paper_2308_15020_amd.ablation [--B 256] [--per-k 8] [--out table.json]

For each length k, `per-k` at-least-k/4 constraints over k distinct
variables are evaluated at B restarts with both bases, in FP32 and FP64.
The reference is the bounded basis in FP64, which agrees with the exact
count-lattice values to ~1e-13 at every length (its parity tests); the
table reports max |WE - WE_ref| over all constraints and restarts, the
fraction of non-finite values, and the evaluation time of each variant.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from . import FLAG_UNIT_CIRCLE, Plan, Problem

KS = (8, 16, 32, 48, 64, 96, 128, 192, 256)


def instance(k: int, count: int, seed: int):
    import workloads
    rng = np.random.default_rng(seed)
    n = max(2 * k, 64)
    rows = [(rng.choice(n, size=k, replace=False) + 1).astype(np.int32) for _ in range(count)]
    return workloads.assemble(n, [(2, [max(1, k // 4)] * count, rows)])


def points(n: int, B: int, dist: str, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, (n, B))
    return np.where(rng.random((n, B)) < 0.5, -0.99, 0.99)


def run(args) -> list:
    rows = []
    for k in KS:
        inst = instance(k, args.per_k, 1000 + k)
        probs = {"uc": Problem(inst, device=0, flags=FLAG_UNIT_CIRCLE), "pb": Problem(inst, device=0)}
        plans = {b: Plan(p, args.B) for b, p in probs.items()}
        for dist in ("uniform", "near_corner"):
            x64 = torch.from_numpy(points(inst.n_vars, args.B, dist, k)).to("cuda:0")
            ref = plans["pb"].eval(x64, want_con=True)["con_val"].double()
            for basis in ("uc", "pb"):
                for dt in (torch.float32, torch.float64):
                    x = x64.to(dt)
                    out = plans[basis].eval(x, want_con=True)
                    torch.cuda.synchronize()
                    cv = out["con_val"].double()
                    fin = torch.isfinite(cv)
                    err = (cv - ref).abs()
                    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    ev0.record()
                    for _ in range(args.reps):
                        plans[basis].eval(x)
                    ev1.record()
                    torch.cuda.synchronize()
                    rows.append({"k": k, "dist": dist, "basis": basis, "dtype": str(dt).split(".")[-1],
                                 "max_err": float(err[fin].max()) if bool(fin.any()) else None,
                                 "nonfinite": float(1.0 - fin.double().mean()),
                                 "ms_per_eval": ev0.elapsed_time(ev1) / args.reps})
                    print(json.dumps(rows[-1]), flush=True)
        for p in plans.values():
            p.close()
        for p in probs.values():
            p.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--B", type=int, default=256)
    ap.add_argument("--per-k", type=int, default=8)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("the basis ablation runs on the GPU")
    rows = run(args)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rows, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
