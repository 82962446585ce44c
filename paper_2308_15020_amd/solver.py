"""Continuous local search over the library (Alg. 1 with the restart
heuristics of the appendix): a batch of B restarts runs T projected-gradient
steps (Alg. 5 with a fixed step size), the rounded points are checked
exactly, and on failure the constraint weights are adapted (ERWA, Prop. 3)
and the restarts are rephased (original / flipped / random phase).

Every arithmetic step runs in libffsat; the loop itself, one host
synchronisation per round (the best satisfied count), lives here.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from .api import Plan, Problem

PHASE_MODE = {"O": 0, "F": 1, "R": 2}


@dataclass
class SolveResult:
    solved: bool
    restart: int                      # index of a satisfying restart (-1 if none)
    assignment: Optional[np.ndarray]  # bool [n], True = variable True (x_v < 0)
    rounds: int
    steps: int
    seconds: float
    best_sat: int
    history: list = field(default_factory=list)
    best_weight: Optional[float] = None     # optimisation mode: best satisfied weight


def _assignment(x: torch.Tensor, b: int) -> np.ndarray:
    return (x[:, b] < 0).cpu().numpy()


def solve(problem: Problem, B: int = 256, rounds: int = 100, T: int = 50, eta: float = 0.05,
          alpha: float = 0.4, weighting: bool = True, policy: str = "ROF",
          x0: Optional[torch.Tensor] = None, seed: int = 0, time_limit: Optional[float] = None,
          plan: Optional[Plan] = None, log: bool = False, optimizer: str = "pgd",
          max_ls: int = 15, maximize: Optional[np.ndarray] = None) -> SolveResult:
    """Alg. 1: returns at the first round in which some restart's rounded point
    satisfies every constraint (decided by the exact checker).

    policy: the rephasing sequence applied to all restarts after each failed
    round, cycled ('ROF' = random, original, flipped; 'RF'; 'O' = continue;
    'R' = plain random restarts).  weighting=False keeps w fixed.
    x0: initial points [n][B] (device, float32); default U[-1, 1] drawn by the
    library's random phase.
    optimizer: 'pgd' (T projected steps of size eta, captured as one graph) or
    'fista' (T accelerated iterations with backtracking from step eta, Alg. 5's
    line search; the state restarts after every rephasing).
    maximize: optimisation mode (weighted MaxSAT, e.g. Max-Cut as weighted
    2-XOR): the score of a restart is the sum of these weights over the
    constraints its rounded point satisfies; the run keeps the best scoring
    assignment over all rounds and stops early only if every constraint holds.
    The search itself still uses the problem's (adaptive) weights.
    """
    if optimizer not in ("pgd", "fista"):
        raise ValueError("optimizer must be 'pgd' or 'fista'")
    t_start = time.perf_counter()
    dev = problem.device
    plan = plan or Plan(problem, B)
    m = problem.m
    problem.set_weights(np.ones(m, dtype=np.float32))
    if x0 is None:
        x = torch.empty(problem.n, B, dtype=torch.float32, device=dev)
        plan.rephase(x, PHASE_MODE["R"], seed=seed)
    else:
        x = x0.detach().to(dev, torch.float32).contiguous().clone()
    history = []
    best = -1
    steps = 0
    state = plan.fista_state(x, eta) if optimizer == "fista" else None
    w_score = None if maximize is None else torch.as_tensor(np.asarray(maximize, np.float32), device=dev)
    best_w, best_assign = None, None
    for r in range(rounds):
        if state is None:
            plan.run_steps(x, T, eta)
        else:
            plan.fista(x, state, T, max_ls=max_ls)
        steps += T
        chk = plan.round_check(x, want=("n_sat", "U") if w_score is None else ("n_sat", "U", "unsat_bits"))
        n_sat = chk["n_sat"]
        b = int(torch.argmax(n_sat).item())
        cur = int(n_sat[b].item())
        best = max(best, cur)
        history.append(cur)
        if w_score is not None:
            score = plan.sat_weight(chk["unsat_bits"], w_score)
            bw = int(torch.argmax(score).item())
            sw = float(score[bw].item())
            if best_w is None or sw > best_w:
                best_w, best_assign = sw, _assignment(x, bw)
        if log:
            print(f"round {r}: best satisfied {cur}/{m}")
        if cur == m:
            return SolveResult(True, b, _assignment(x, b), r + 1, steps, time.perf_counter() - t_start, m, history,
                               best_weight=best_w if w_score is None else float(w_score.sum().item()))
        if time_limit is not None and time.perf_counter() - t_start > time_limit:
            break
        if weighting:
            plan.erwa_update(chk["U"], alpha)
        phase = policy[r % len(policy)]
        plan.rephase(x, PHASE_MODE[phase], seed=seed * 1000003 + r + 1)
        if state is not None:
            state = plan.fista_state(x, eta)
    return SolveResult(False, -1, best_assign, len(history), steps, time.perf_counter() - t_start, best, history,
                       best_weight=best_w)
