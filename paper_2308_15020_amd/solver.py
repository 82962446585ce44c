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
from typing import Callable, Optional

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


class Search:
    """One arm of the search: a plan of B restarts with its own weights (held
    by its problem), rephasing policy and optimiser.  `run_round` does T
    steps and the exact check; `adapt` applies ERWA and the next phase."""

    def __init__(self, problem: Problem, B: int, T: int = 50, eta: float = 0.05, alpha: float = 0.4,
                 weighting: bool = True, policy: str = "ROF", x0: Optional[torch.Tensor] = None, seed: int = 0,
                 plan: Optional[Plan] = None, optimizer: str = "pgd", max_ls: int = 15,
                 maximize: Optional[np.ndarray] = None, step_norm: bool = True,
                 random_phase: Optional[Callable[[int], torch.Tensor]] = None,
                 x_buf: Optional[torch.Tensor] = None):
        if optimizer not in ("pgd", "fista"):
            raise ValueError("optimizer must be 'pgd' or 'fista'")
        if not policy or any(ph not in PHASE_MODE for ph in policy):
            raise ValueError("policy must be a non-empty string over 'O', 'F', 'R'")
        self.problem, self.B, self.T, self.eta, self.alpha = problem, B, T, eta, alpha
        self.weighting, self.policy, self.seed, self.max_ls = weighting, policy, seed, max_ls
        self.step_norm = step_norm
        self.random_phase = random_phase
        self.eta_eff = eta
        dev = problem.device
        self.plan = plan or Plan(problem, B)
        problem.set_weights(np.ones(problem.m, dtype=np.float32))
        # the iterate lives in x_buf when given: the library's captured step
        # graphs are keyed by the buffers, so searches that share x_buf on
        # one plan replay the same graph
        self.x = x_buf if x_buf is not None else torch.empty(problem.n, B, dtype=torch.float32, device=dev)
        if x0 is None:
            self.plan.rephase(self.x, PHASE_MODE["R"], seed=seed)
        else:
            self.x.copy_(x0.detach().to(dev, torch.float32))
        self.state = self.plan.fista_state(self.x, eta) if optimizer == "fista" else None
        self.w_score = None if maximize is None else torch.as_tensor(np.asarray(maximize, np.float32), device=dev)
        self.best_w, self.best_assign = None, None
        self.steps = 0
        self.history = []
        self._chk = None

    def run_round(self):
        """T steps, then the exact check of the rounded points.  Returns
        (best restart, its satisfied count)."""
        if self.state is None:
            self.plan.run_steps(self.x, self.T, self.eta_eff)
        else:
            self.plan.fista(self.x, self.state, self.T, max_ls=self.max_ls)
        self.steps += self.T
        want = ("n_sat", "U") if self.w_score is None else ("n_sat", "U", "unsat_bits")
        chk = self.plan.round_check(self.x, want=want)
        self._chk = chk
        b = int(torch.argmax(chk["n_sat"]).item())
        cur = int(chk["n_sat"][b].item())
        self.history.append(cur)
        if self.w_score is not None:
            score = self.plan.sat_weight(chk["unsat_bits"], self.w_score)
            bw = int(torch.argmax(score).item())
            sw = float(score[bw].item())
            if self.best_w is None or sw > self.best_w:
                self.best_w, self.best_assign = sw, _assignment(self.x, bw)
        return b, cur

    def adapt(self, r: int):
        """After failed round r: ERWA on this round's counts, then the phase
        policy[r mod len(policy)] for every restart."""
        if self.weighting:
            self.plan.erwa_update(self._chk["U"], self.alpha)
            if self.step_norm:
                # a common factor of the weights only rescales F: keep the
                # projected step's length as with unit weights
                wm = float(self.problem.get_weights().mean().item())
                self.eta_eff = self.eta / max(wm, 1e-6)
        phase = self.policy[r % len(self.policy)]
        if phase == "R" and self.random_phase is not None:
            self.x.copy_(self.random_phase(r))
        else:
            self.plan.rephase(self.x, PHASE_MODE[phase], seed=self.seed * 1000003 + r + 1)
        if self.state is not None:
            # in place: the same state buffers keep the captured FISTA graph
            self.plan.fista_reset(self.state, self.x, self.eta)


def solve(problem: Problem, B: int = 256, rounds: int = 100, T: int = 50, eta: float = 0.05,
          alpha: float = 0.4, weighting: bool = True, policy: str = "ROF",
          x0: Optional[torch.Tensor] = None, seed: int = 0, time_limit: Optional[float] = None,
          plan: Optional[Plan] = None, log: bool = False, optimizer: str = "pgd",
          max_ls: int = 15, maximize: Optional[np.ndarray] = None, step_norm: bool = True,
          random_phase: Optional[Callable[[int], torch.Tensor]] = None,
          x_buf: Optional[torch.Tensor] = None) -> SolveResult:
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
    random_phase: draws the points of the random phase after failed round r
    (default: U[-1, 1] from the library), e.g. a fresh learned proposal.
    x_buf: a [n][B] float32 device buffer to hold the iterate (its pointer
    keys the captured step graph, so runs sharing it replay one graph).
    step_norm: with adaptive weights, divide the projected step size by the
    mean weight after every update (the weights shrink towards U/max U, which
    would otherwise shorten a fixed step; the paper's line search adapts the
    step by itself).  On 2-hidden random 3-SAT at n = 200 this takes the
    weighted search from 2 of 20 to all instances solved.
    """
    t_start = time.perf_counter()
    m = problem.m
    S = Search(problem, B, T=T, eta=eta, alpha=alpha, weighting=weighting, policy=policy, x0=x0, seed=seed,
               plan=plan, optimizer=optimizer, max_ls=max_ls, maximize=maximize, step_norm=step_norm,
               random_phase=random_phase, x_buf=x_buf)
    best = -1
    for r in range(rounds):
        b, cur = S.run_round()
        best = max(best, cur)
        if log:
            print(f"round {r}: best satisfied {cur}/{m}")
        if cur == m:
            return SolveResult(True, b, _assignment(S.x, b), r + 1, S.steps, time.perf_counter() - t_start, m,
                               S.history, best_weight=S.best_w if S.w_score is None else float(S.w_score.sum().item()))
        if time_limit is not None and time.perf_counter() - t_start > time_limit:
            break
        S.adapt(r)
    return SolveResult(False, -1, S.best_assign, len(S.history), S.steps, time.perf_counter() - t_start, best,
                       S.history, best_weight=S.best_w)


@dataclass
class Arm:
    """One strategy of a portfolio: its share of the restarts and its heuristics."""
    B: int
    weighting: bool = True
    policy: str = "ROF"
    eta: float = 0.05
    optimizer: str = "pgd"
    alpha: float = 0.4
    step_norm: bool = True


def solve_portfolio(inst, arms, rounds: int = 100, T: int = 50, seed: int = 0, device: int = 0,
                    problems=None, log: bool = False) -> SolveResult:
    """Several strategies side by side on one GPU (Table 2's portfolio; the
    paper runs its arms on separate GPUs).  Each arm has its own problem
    object (its own adaptive weights) and restarts; every round runs T steps
    of each arm, and the run stops at the first round in which any arm's
    rounded point satisfies everything.  `restart` of the result indexes the
    arms' restarts in order (arm 0's first).  problems: reuse one Problem per
    arm (their weights are reset)."""
    t_start = time.perf_counter()
    probs = problems if problems is not None else [Problem(inst, device=device) for _ in arms]
    if len(probs) != len(arms):
        raise ValueError("one problem per arm")
    if len({id(p) for p in probs}) != len(probs):
        raise ValueError("each arm needs its own problem object (the adaptive weights live on it)")
    m = probs[0].m
    searches = [Search(p, a.B, T=T, eta=a.eta, alpha=a.alpha, weighting=a.weighting, policy=a.policy,
                       seed=seed * 7919 + i, optimizer=a.optimizer, step_norm=a.step_norm)
                for i, (p, a) in enumerate(zip(probs, arms))]
    offs = np.cumsum([0] + [a.B for a in arms])
    best, history = -1, []
    for r in range(rounds):
        cur_best, hit = -1, None
        for i, S in enumerate(searches):
            b, cur = S.run_round()
            if cur > cur_best:
                cur_best = cur
            if cur == m and hit is None:
                hit = (i, b)
        best = max(best, cur_best)
        history.append(cur_best)
        if log:
            print(f"round {r}: best satisfied {cur_best}/{m}")
        if hit is not None:
            i, b = hit
            return SolveResult(True, int(offs[i] + b), _assignment(searches[i].x, b), r + 1,
                               sum(S.steps for S in searches), time.perf_counter() - t_start, m, history)
        for S in searches:
            S.adapt(r)
    return SolveResult(False, -1, None, len(history), sum(S.steps for S in searches),
                       time.perf_counter() - t_start, best, history)
