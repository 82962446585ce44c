"""Time-to-solve: learned initialisation against uniform restarts.

    python -m paper_2308_15020_amd.tts [--train 50] [--test 100] [--B 256]
        [--rounds 30] [--T 40] [--family planted|hidden2|random] [--out result.json]

Instances have the shape of the mixed n = 2000 workload (8000 OR of length
3-7, 500 XOR of length 3-20, 200 at-least-t of length 10-100; --n-xor sets
the XOR count of the generated families, since the XOR constraints decide
how hard an instance is for the continuous search).  Families:
  planted  drawn around a hidden assignment (OR signs redrawn until it
           satisfies them, at-least-t signs aligned with it): satisfiable,
           but literal counts lean towards the hidden assignment;
  hidden2  satisfiable with no such lean: OR clauses hold under the hidden
           assignment and its complement, XOR parities come from it,
           at-least-t signs are drawn independently of it;
  random   the unplanted generator (satisfiability not guaranteed).
Training instances use seeds 10000.., test instances seeds 20000..
(disjoint).  The network is trained on the mean signs of the best end
points of uniform-init searches (1024 restarts per training instance).

Arms, on the same plan, step size, weighting and rephasing policy:
uniform U[-1, 1] restarts; learned (the network's lean, a quarter of the
restarts kept uniform, every random phase after a failed round drawn as a
fresh proposal unless --no-reuse-proposal); learned_once (the proposal in
the first round only, random phases uniform); polarity (the same proposal
from a non-learned lean towards each variable's majority sign, to separate
what the network learns from plain occurrence counts).  The arms share one
iterate buffer, whose step graph is captured before any arm is timed, and
take turns at going first.  Per test instance and arm the clock runs from
the start of initialisation (network inference and proposal included) to
the round in which a restart's rounded point passes the exact checker,
within `rounds` rounds of T projected-gradient steps.
Reported: solve rate per arm, median / mean time over the instances both
learned and uniform solve, median rounds, and the time each arm needs to
solve as many instances as the lower of the two solve rates allows (a point
of the cactus curve).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import Plan, Problem
from .mpnn import Mpnn, fit, targets_from_solves
from .solver import solve


def instance(seed: int, family: str, n_xor: int = 500):
    import workloads
    if family == "planted":
        inst, _ = workloads.planted_hybrid(2000, seed, n_or=8000, or_len=(3, 7), n_xor=n_xor, xor_len=(3, 20),
                                           n_card=200, card_len=(10, 100))
        return inst
    if family == "hidden2":
        inst, _ = workloads.hidden2_hybrid(2000, seed, n_or=8000, or_len=(3, 7), n_xor=n_xor, xor_len=(3, 20),
                                           n_card=200, card_len=(10, 100))
        return inst
    return workloads.config2(seed)


def polarity_mu(inst, device) -> torch.Tensor:
    """The non-learned baseline: lean each variable towards the polarity it
    occurs in more often (x < 0 is True, so mu = -(P - N)/(P + N + 1))."""
    lits = inst.lits.astype(np.int64)
    v = np.abs(lits) - 1
    P = np.bincount(v[lits > 0], minlength=inst.n_vars).astype(np.float64)
    N = np.bincount(v[lits < 0], minlength=inst.n_vars).astype(np.float64)
    return torch.from_numpy((-(P - N) / (P + N + 1.0)).astype(np.float32)).to(device)


def run_arm(prob: Problem, plan: Plan, net, args, seed: int, x_buf, mu_fixed=None, reuse=None) -> dict:
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0 = None
    again = None
    reuse = args.reuse_proposal if reuse is None else reuse
    if net is not None:
        mu = net.forward(prob) if mu_fixed is None else mu_fixed
        x0 = net.propose(plan, mu, frac_learned=args.frac, sigma=args.sigma, seed=seed)
        if reuse:
            # the random phase draws a fresh proposal from the same lean
            def again(r):
                return net.propose(plan, mu, frac_learned=args.frac, sigma=args.sigma, seed=seed * 1009 + r + 1)
    res = solve(prob, B=args.B, rounds=args.rounds, T=args.T, eta=args.eta, policy=args.policy, x0=x0,
                seed=seed, plan=plan, random_phase=again, x_buf=x_buf)
    torch.cuda.synchronize()
    return {"solved": bool(res.solved), "seconds": time.perf_counter() - t0, "rounds": res.rounds,
            "best_sat": res.best_sat}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=50)
    ap.add_argument("--test", type=int, default=100)
    ap.add_argument("--B", type=int, default=256)
    ap.add_argument("--rounds", type=int, default=30)
    ap.add_argument("--T", type=int, default=40)
    ap.add_argument("--eta", type=float, default=0.1)
    ap.add_argument("--policy", default="ROF")
    ap.add_argument("--frac", type=float, default=0.75)
    ap.add_argument("--sigma", type=float, default=0.3)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--family", default="random", choices=["planted", "hidden2", "random"])
    ap.add_argument("--planted", action="store_true", help="same as --family planted")
    ap.add_argument("--n-xor", type=int, default=500, help="XOR constraints of a planted instance")
    ap.add_argument("--no-reuse-proposal", dest="reuse_proposal", action="store_false",
                    help="learned and polarity arms: the random phase after a failed round draws U[-1, 1] "
                         "(default: a fresh proposal from the same lean)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.planted:
        args.family = "planted"

    def log(msg):
        print(msg, flush=True)

    # training data
    t_tr = time.perf_counter()
    train_p, train_t = [], []
    for i in range(args.train):
        p = Problem(instance(10000 + i, args.family, args.n_xor), device=0)
        train_p.append(p)
        train_t.append(targets_from_solves(p, B=1024, seed=10000 + i))
        if (i + 1) % 10 == 0:
            log(f"targets {i + 1}/{args.train}")
    net = Mpnn(64, 3, device=0, seed=1)
    hist = fit(net, train_p, train_t, epochs=args.epochs, lr=args.lr)
    log(f"trained: loss {hist[0]:.4f} -> {hist[-1]:.4f} in {time.perf_counter() - t_tr:.1f} s")
    del train_p, train_t

    rows = []
    for i in range(args.test):
        seed = 20000 + i
        inst = instance(seed, args.family, args.n_xor)
        prob = Problem(inst, device=0)
        plan = Plan(prob, args.B)
        x_buf = torch.empty(prob.n, args.B, dtype=torch.float32, device=prob.device)
        # capture the step graph of this (plan, buffer) before any arm is timed
        plan.rephase(x_buf, 2, seed=seed)
        plan.run_steps(x_buf, args.T, args.eta)
        torch.cuda.synchronize()
        pol = polarity_mu(inst, prob.device)   # host-side counts, outside the clock
        arms = {
            "uniform": lambda: run_arm(prob, plan, None, args, seed, x_buf),
            "learned": lambda: run_arm(prob, plan, net, args, seed, x_buf),
            "learned_once": lambda: run_arm(prob, plan, net, args, seed, x_buf, reuse=False),
            "polarity": lambda: run_arm(prob, plan, net, args, seed, x_buf, mu_fixed=pol),
        }
        names = list(arms)
        order = names[i % len(names):] + names[:i % len(names)]
        row = {"seed": seed}
        for a in order:
            row[a] = arms[a]()
        rows.append(row)
        log(f"test {seed}: " + " | ".join(f"{a} {row[a]['solved']} {row[a]['seconds']:.3f}s r{row[a]['rounds']}"
                                         for a in names))
        plan.close()
        prob.close()

    su = [r["uniform"]["solved"] for r in rows]
    sl = [r["learned"]["solved"] for r in rows]
    sp = [r["polarity"]["solved"] for r in rows]
    bl = [r for r in rows if r["polarity"]["solved"] and r["learned"]["solved"]]
    both = [r for r in rows if r["uniform"]["solved"] and r["learned"]["solved"]]
    tu = np.array([r["uniform"]["seconds"] for r in both])
    tl = np.array([r["learned"]["seconds"] for r in both])
    # cactus measure: the time by which each arm has solved as many instances
    # as the lower of the two solve rates allows (its k-th fastest solve)
    k_low = int(min(sum(su), sum(sl)))
    cactus = {"instances": k_low}
    for arm in ("uniform", "learned"):
        ts = sorted(r[arm]["seconds"] for r in rows if r[arm]["solved"])
        cactus[arm + "_s"] = float(ts[k_low - 1]) if k_low > 0 else None
    lo = [r for r in rows if r["learned_once"]["solved"] and r["uniform"]["solved"]]
    summary = {
        "instances": args.test, "family": args.family, "n_xor": args.n_xor if args.family != "random" else 500,
        "reuse_proposal": bool(args.reuse_proposal),
        "B": args.B, "rounds": args.rounds, "T": args.T,
        "eta": args.eta, "policy": args.policy, "frac_learned": args.frac, "sigma": args.sigma,
        "train_instances": args.train, "train_loss": [hist[0], hist[-1]],
        "solve_rate": {"uniform": float(np.mean(su)), "learned": float(np.mean(sl)),
                       "polarity": float(np.mean(sp))},
        "learned_vs_polarity_both_solved": len(bl),
        "learned_vs_polarity_median_s": [float(np.median([r["learned"]["seconds"] for r in bl])) if bl else None,
                                         float(np.median([r["polarity"]["seconds"] for r in bl])) if bl else None],
        "both_solved": len(both),
        "median_s": {"uniform": float(np.median(tu)) if len(both) else None,
                     "learned": float(np.median(tl)) if len(both) else None},
        "mean_s": {"uniform": float(np.mean(tu)) if len(both) else None,
                   "learned": float(np.mean(tl)) if len(both) else None},
        "median_rounds": {"uniform": float(np.median([r["uniform"]["rounds"] for r in both])) if both else None,
                          "learned": float(np.median([r["learned"]["rounds"] for r in both])) if both else None},
        "cactus_at_lower_solve_rate": cactus,
        "learned_once_solve_rate": float(np.mean([r["learned_once"]["solved"] for r in rows])),
        "learned_once_median_s": float(np.median([r["learned_once"]["seconds"] for r in lo])) if lo else None,
        "learned_once_uniform_both_solved": len(lo),
        "median_rounds_all": {a: float(np.median([r[a]["rounds"] for r in rows]))
                              for a in ("uniform", "learned", "learned_once", "polarity")},
    }
    log(json.dumps(summary))
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": summary, "rows": rows}, f, indent=1)
    return summary


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
