"""Learned initialiser: a message-passing network over the clause-variable
incidence graph proposes restart points (ffsat_mpnn_* in the C ABI).

The paper observes that the starting point of the continuous search matters
(restart heuristics of its appendix) but gives no network; this one, its
features, targets and training loop are additions.  Every forward, backward
and optimiser step runs in libffsat's HIP kernels; this module marshals
arguments and drives the training loop.

Targets: for each training instance, the sign pattern of the best end points
of uniform-init solves, averaged (``targets_from_solves``), in [-1, 1] with
-1 = True as everywhere in the library.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check, lib
from .api import Plan, Problem, _need, _ptr, _stream


class Mpnn:
    """Network parameters and optimiser state on one device."""

    def __init__(self, hidden: int = 64, rounds: int = 3, device: int = 0, seed: int = 0):
        self.hidden, self.rounds = int(hidden), int(rounds)
        self.device = torch.device("cuda", device)
        d = _lib.MpnnDesc(self.hidden, self.rounds, int(device), 0, int(seed) & (2 ** 64 - 1))
        h = C.c_void_p()
        check(lib().ffsat_mpnn_create(C.byref(d), C.byref(h)))
        self._h = h
        n = C.c_int64()
        check(lib().ffsat_mpnn_num_params(self._h, C.byref(n)))
        self.num_params = int(n.value)

    def _io(self, which: int, to_net: bool, buf: np.ndarray) -> None:
        check(lib().ffsat_mpnn_params(self._h, C.c_void_p(buf.ctypes.data), which, int(to_net), 0,
                                      _stream(self.device)))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params, np.float32)
        self._io(0, False, out)
        return out

    def set_params(self, flat) -> None:
        a = np.ascontiguousarray(np.asarray(flat, dtype=np.float32))
        if a.shape != (self.num_params,):
            raise ValueError(f"expected {self.num_params} parameters, got {a.shape}")
        self._io(0, True, a)

    def grads(self) -> np.ndarray:
        out = np.empty(self.num_params, np.float32)
        self._io(1, False, out)
        return out

    def forward(self, problem: Problem, mu: Optional[torch.Tensor] = None) -> torch.Tensor:
        if mu is None:
            mu = torch.empty(problem.n, dtype=torch.float32, device=self.device)
        _need(mu, (problem.n,), torch.float32, self.device, "mu")
        check(lib().ffsat_mpnn_forward(self._h, problem.handle, _ptr(mu), _stream(self.device)))
        return mu

    def backward(self, problem: Problem, target: torch.Tensor) -> torch.Tensor:
        """Forward + loss + parameter gradients; returns the loss (device scalar)."""
        _need(target, (problem.n,), torch.float32, self.device, "target")
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        check(lib().ffsat_mpnn_backward(self._h, problem.handle, _ptr(target), _ptr(loss), _stream(self.device)))
        return loss

    def adam(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        check(lib().ffsat_mpnn_adam(self._h, float(lr), float(beta1), float(beta2), float(eps),
                                    _stream(self.device)))

    def propose(self, plan: Plan, mu: torch.Tensor, frac_learned: float = 0.75, sigma: float = 0.3,
                seed: int = 0, x: Optional[torch.Tensor] = None) -> torch.Tensor:
        """x[n][B]: the first round(frac_learned*B) restarts near mu, the rest uniform."""
        if x is None:
            x = torch.empty(plan.n, plan.B, dtype=torch.float32, device=self.device)
        _need(x, (plan.n, plan.B), torch.float32, self.device, "x")
        _need(mu, (plan.n,), torch.float32, self.device, "mu")
        check(lib().ffsat_mpnn_propose(plan.handle, _ptr(mu), _ptr(x), float(frac_learned), float(sigma),
                                       int(seed) & (2 ** 64 - 1), _stream(self.device)))
        return x

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().ffsat_mpnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def targets_from_solves(problem: Problem, B: int = 1024, rounds: int = 4, T: int = 40, eta: float = 0.1,
                        alpha: float = 0.4, top_frac: float = 0.1, seed: int = 0) -> torch.Tensor:
    """Mean sign of the rounded end points of the best restarts (by satisfied
    count) after a short uniform-init search with adaptive weights; the
    problem's weights are reset to one afterwards."""
    plan = Plan(problem, B)
    problem.set_weights(np.ones(problem.m, dtype=np.float32))
    x = torch.empty(problem.n, B, dtype=torch.float32, device=problem.device)
    plan.rephase(x, 2, seed=seed)
    for r in range(rounds):
        plan.run_steps(x, T, eta)
        chk = plan.round_check(x, want=("n_sat", "U"))
        if r + 1 < rounds:
            plan.erwa_update(chk["U"], alpha)
    q = max(1, int(round(top_frac * B)))
    best = torch.topk(chk["n_sat"].to(torch.float32), q).indices
    t = torch.where(x[:, best] < 0, -1.0, 1.0).mean(dim=1).contiguous()
    problem.set_weights(np.ones(problem.m, dtype=np.float32))
    plan.close()
    return t


def fit(net: Mpnn, problems: Sequence[Problem], targets: Sequence[torch.Tensor], epochs: int = 30,
        lr: float = 2e-3, log: bool = False) -> list:
    """Plain Adam over the training instances, one instance per step."""
    hist = []
    for ep in range(epochs):
        tot = torch.zeros(1, dtype=torch.float32, device=net.device)
        for p, t in zip(problems, targets):
            tot += net.backward(p, t)
            net.adam(lr)
        v = float(tot.item()) / max(1, len(problems))
        hist.append(v)
        if log:
            print(f"epoch {ep}: loss {v:.5f}")
    return hist
