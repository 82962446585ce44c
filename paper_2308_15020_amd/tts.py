"""Time-to-solve: learned initialisation against uniform restarts.

    python -m paper_2308_15020_amd.tts [--train 50] [--test 100] [--B 256]
        [--rounds 30] [--T 40] [--planted] [--out result.json]

Instances are mixed hybrid formulas with the shape of the n = 2000 workload
(8000 OR of length 3-7, 500 XOR of length 3-20, 200 at-least-t of length
10-100); with --planted, each is drawn around a hidden assignment so that it
is satisfiable (--n-xor sets its XOR count: the XOR constraints decide how
hard an instance is for the continuous search).  Training instances use seeds 10000.., test instances seeds
20000.. (disjoint).  The network is trained on the mean signs of the best end
points of uniform-init searches (1024 restarts per training instance).

The learned and polarity arms also draw every random phase after a failed
round from their own lean (a fresh proposal), unless --no-reuse-proposal.
Per test instance and arm, the clock runs from the start of initialisation
(network inference and proposal included for the learned arm) to the round in
which a restart's rounded point passes the exact checker, within a budget of
`rounds` rounds of T projected-gradient steps.  Both arms use the same plan,
step size, weighting and rephasing policy; the learned arm keeps a quarter of
its restarts uniform.  A third arm proposes the same way from a non-learned
polarity lean (each variable towards the sign it occurs in more often), to
separate what the network learns from the plain occurrence counts.
Reported: solve rate per arm, median / mean time over the instances both
arms solve, and the time each arm needs to solve as many instances as the
lower of the two solve rates allows (a point of the cactus curve).
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


def instance(seed: int, planted: bool, n_xor: int = 500):
    import workloads
    if planted:
        inst, _ = workloads.planted_hybrid(2000, seed, n_or=8000, or_len=(3, 7), n_xor=n_xor, xor_len=(3, 20),
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


def run_arm(prob: Problem, plan: Plan, net, args, seed: int, mu_fixed=None) -> dict:
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0 = None
    again = None
    if net is not None:
        mu = net.forward(prob) if mu_fixed is None else mu_fixed
        x0 = net.propose(plan, mu, frac_learned=args.frac, sigma=args.sigma, seed=seed)
        if args.reuse_proposal:
            # the random phase draws a fresh proposal from the same lean
            def again(r):
                return net.propose(plan, mu, frac_learned=args.frac, sigma=args.sigma, seed=seed * 1009 + r + 1)
    res = solve(prob, B=args.B, rounds=args.rounds, T=args.T, eta=args.eta, policy=args.policy, x0=x0,
                seed=seed, plan=plan, random_phase=again)
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
    ap.add_argument("--planted", action="store_true")
    ap.add_argument("--n-xor", type=int, default=500, help="XOR constraints of a planted instance")
    ap.add_argument("--no-reuse-proposal", dest="reuse_proposal", action="store_false",
                    help="learned and polarity arms: the random phase after a failed round draws U[-1, 1] "
                         "(default: a fresh proposal from the same lean)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    # training data
    t_tr = time.perf_counter()
    train_p, train_t = [], []
    for i in range(args.train):
        p = Problem(instance(10000 + i, args.planted, args.n_xor), device=0)
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
        inst = instance(seed, args.planted, args.n_xor)
        prob = Problem(inst, device=0)
        plan = Plan(prob, args.B)
        r_u = run_arm(prob, plan, None, args, seed)
        r_l = run_arm(prob, plan, net, args, seed)
        # host-side polarity counts happen before the clock in run_arm starts
        r_p = run_arm(prob, plan, net, args, seed, mu_fixed=polarity_mu(inst, prob.device))
        rows.append({"seed": seed, "uniform": r_u, "learned": r_l, "polarity": r_p})
        log(f"test {seed}: uniform {r_u['solved']} {r_u['seconds']:.3f}s r{r_u['rounds']} | "
            f"learned {r_l['solved']} {r_l['seconds']:.3f}s r{r_l['rounds']} | "
            f"polarity {r_p['solved']} {r_p['seconds']:.3f}s r{r_p['rounds']}")
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
    summary = {
        "instances": args.test, "planted": args.planted, "n_xor": args.n_xor if args.planted else 500,
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
    }
    log(json.dumps(summary))
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": summary, "rows": rows}, f, indent=1)
    return summary


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
