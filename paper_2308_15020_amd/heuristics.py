"""Restart heuristics on random 3-SAT: the analogue of the paper's Table 2
(search with and without the weighting and rephasing heuristics, and the
portfolio of the two), on seeded synthetic instances.

    python -m paper_2308_15020_amd.heuristics [--n 50 100 150 200 250]
        [--instances 100] [--B 1024] [--rounds 1000] [--T 50] [--eta 0.1] [--out table.json]

Instances: satisfiable random 3-SAT at clause ratio 4.26 from the 2-hidden
generator (`workloads.hidden2_ksat`, seeds 1000 n + i), standing in for the
uniform random 3-SAT benchmark sets the paper draws from (all satisfiable,
not available here).

An iteration is one round of Alg. 1: a local search of T projected-gradient
steps from every restart's current point, then the exact check of the
rounded points.  Arms, within a budget of `rounds` iterations:
  w/o heuristics  B restarts, fixed unit weights, every failed round restarts
                  at random ((R)^inf);
  w/ heuristics   B restarts, adaptive weights (ERWA, alpha = 0.4) and
                  rephasing (ROF)^inf; the step size is divided by the mean
                  weight (--no-step-norm keeps it fixed);
  portfolio       both strategies on one GPU with B/2 restarts each (the same
                  total work as one arm);
  two-device portfolio: both full arms as if on two GPUs (the paper's
                  set-up: solved by either, at the smaller iteration count),
                  derived from the two runs.
Reported per n: instances solved and the average iterations with PAR-2
(an unsolved instance counts 2 x rounds), the paper's two measures.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import Problem
from .solver import Arm, solve, solve_portfolio


def instance(n: int, i: int):
    import workloads
    return workloads.hidden2_ksat(n, 1000 * n + i, ratio=4.26)[0]


def run(args) -> dict:
    table = {}
    for n in args.n:
        rows = []
        for i in range(args.instances):
            inst = instance(n, i)
            prob = Problem(inst, device=0)
            res = {}
            r = solve(prob, B=args.B, rounds=args.rounds, T=args.T, eta=args.eta, weighting=False, policy="R", seed=i)
            res["plain"] = (r.solved, r.rounds, r.seconds)
            sn = not getattr(args, "no_step_norm", False)
            r = solve(prob, B=args.B, rounds=args.rounds, T=args.T, eta=args.eta, weighting=True, policy="ROF",
                      seed=i, step_norm=sn)
            res["heuristic"] = (r.solved, r.rounds, r.seconds)
            half = args.B // 2
            probs = [prob, Problem(inst, device=0)]
            r = solve_portfolio(inst, [Arm(half, weighting=False, policy="R", eta=args.eta),
                                       Arm(args.B - half, weighting=True, policy="ROF", eta=args.eta, step_norm=sn)],
                                rounds=args.rounds, T=args.T, seed=i, problems=probs)
            res["portfolio"] = (r.solved, r.rounds, r.seconds)
            probs[1].close()
            pl, he = res["plain"], res["heuristic"]
            both = [v for v in (pl, he) if v[0]]
            res["two_device"] = (bool(both), min(v[1] for v in both) if both else args.rounds,
                                 min(v[2] for v in both) if both else max(pl[2], he[2]))
            prob.close()
            rows.append(res)
            print(json.dumps({"n": n, "i": i, **{k: v[:2] for k, v in res.items()}}), flush=True)
        summ = {"instances": len(rows), "solved_by_any": sum(1 for r in rows if any(v[0] for v in r.values()))}
        for arm in ("plain", "heuristic", "portfolio", "two_device"):
            par2 = [r[arm][1] if r[arm][0] else 2 * args.rounds for r in rows]
            sol = [r[arm] for r in rows if r[arm][0]]
            summ[arm] = {"solved": len(sol), "par2_iters": float(np.mean(par2)),
                         "mean_iters_solved": float(np.mean([v[1] for v in sol])) if sol else None,
                         "mean_ms_solved": float(1e3 * np.mean([v[2] for v in sol])) if sol else None}
        table[n] = summ
        print(json.dumps({"n": n, "summary": summ}), flush=True)
    return table


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[50, 100, 150, 200, 250])
    ap.add_argument("--instances", type=int, default=100)
    ap.add_argument("--B", type=int, default=1024)
    ap.add_argument("--rounds", type=int, default=1000)
    ap.add_argument("--T", type=int, default=50)
    ap.add_argument("--eta", type=float, default=0.1)
    ap.add_argument("--no-step-norm", action="store_true",
                    help="weighting arms keep the fixed step size (default: divided by the mean weight)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    table = run(args)
    out = {"args": vars(args), "table": {str(k): v for k, v in table.items()}}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
