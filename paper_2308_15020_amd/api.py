"""Python classes over the C ABI: a constraint set on the device (Problem)
and a batch size with its workspace (Plan).

Torch tensors only carry device memory and the current stream; every step
runs in libffsat's HIP kernels.  Points are ``x[n][B]`` (restarts
contiguous) as in the C ABI.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import FFSatError, check, lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t: torch.Tensor, shape, dtype, device, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)} on {device}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


class Problem:
    """A validated constraint set copied to the device (ffsat_problem_create)."""

    def __init__(self, inst, device: int = 0, fp64_min_len: int = 0, flags: int = 0):
        L = lib()
        self.n = int(inst.n_vars)
        self.m = int(inst.m)
        self.device = torch.device("cuda", device)
        self._keep = dict(
            con_ptr=np.ascontiguousarray(inst.con_ptr, np.int64),
            lits=np.ascontiguousarray(inst.lits, np.int32),
            kinds=np.ascontiguousarray(inst.kinds, np.int32),
            params=np.ascontiguousarray(inst.params, np.int32),
            weights=None if inst.weights is None else np.ascontiguousarray(inst.weights, np.float32),
        )
        k = self._keep
        d = _lib.ProblemDesc(
            self.n, self.m, k["con_ptr"].ctypes.data, k["lits"].ctypes.data, k["kinds"].ctypes.data,
            k["params"].ctypes.data, None if k["weights"] is None else k["weights"].ctypes.data,
            int(device), int(fp64_min_len), int(flags))
        h = C.c_void_p()
        if torch.cuda.is_available() and 0 <= device < torch.cuda.device_count():
            torch.cuda.set_device(device)
        check(L.ffsat_problem_create(C.byref(d), C.byref(h)))
        self._h = h
        self._keep = None   # host arrays were copied by the library
        self.nnz = int(inst.nnz)

    @property
    def handle(self):
        if self._h is None:
            raise FFSatError(-1, "problem was closed")
        return self._h

    def info(self) -> dict:
        inf = _lib.ProblemInfo()
        check(lib().ffsat_problem_info_get(self.handle, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def set_weights(self, w) -> None:
        if isinstance(w, torch.Tensor) and w.is_cuda:
            _need(w, (self.m,), torch.float32, self.device, "w")
            check(lib().ffsat_set_weights(self.handle, _ptr(w), 1, _stream(self.device)))
        else:
            a = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
            assert a.shape == (self.m,)
            check(lib().ffsat_set_weights(self.handle, C.c_void_p(a.ctypes.data), 0, _stream(self.device)))

    def get_weights(self) -> torch.Tensor:
        out = torch.empty(self.m, dtype=torch.float32, device=self.device)
        check(lib().ffsat_get_weights(self.handle, _ptr(out), 1, _stream(self.device)))
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().ffsat_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A batch size B bound to a problem, with its device workspace."""

    def __init__(self, problem: Problem, B: int, autotune: bool = False, use_graphs: bool = True,
                 tune_cache: Optional[str] = None, side_streams: bool = True, mode: str = "auto",
                 pull: str = "auto", pull_vc: int = 0, persistent: bool = False):
        self.problem = problem
        self.B = int(B)
        self.device = problem.device
        o = _lib.PlanOpts()
        o.autotune = 1 if autotune else 0
        o.use_graphs = 1 if use_graphs else 0
        o.tune_cache = tune_cache.encode() if tune_cache else None
        o.reserved[0] = 0 if side_streams else 1
        modes = {"auto": 0, "per_bin": 1, "group_all": 2, "group_dft": 3}
        if mode not in modes:
            raise ValueError(f"mode must be one of {sorted(modes)}")
        o.reserved[1] = modes[mode]
        # gradient of the short transform-free constraints gathered per variable
        # ("le3": length <= 3, "le7": <= 7) instead of through slots ("off");
        # "auto": chosen by the autotuner (off without it)
        pulls = {"auto": 0, "off": 1, "le7": 2, "le3": 3}
        if pull not in pulls:
            raise ValueError(f"pull must be one of {sorted(pulls)}")
        o.reserved[2] = pulls[pull]
        o.reserved[3] = int(pull_vc)
        # run_steps as one persistent launch for small problems of short
        # transform-free constraints (falls back to the usual steps otherwise)
        o.reserved[4] = 1 if persistent else 0
        h = C.c_void_p()
        check(lib().ffsat_plan_create(problem.handle, self.B, C.byref(o), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise FFSatError(-1, "plan was closed")
        return self._h

    @property
    def n(self):
        return self.problem.n

    @property
    def m(self):
        return self.problem.m

    def _x(self, x, dtype=torch.float32):
        _need(x, (self.n, self.B), dtype, self.device, "x")

    def eval(self, x: torch.Tensor, want_F=True, want_grad=True, want_con=False, want_check=False,
             out=None) -> dict:
        """Objective F[B], gradient [n][B], per-constraint values [m][B] at x[n][B];
        with want_check also the exact check of the same point (n_sat, unsat_bits, U)
        from the same kernels (FP32 only)."""
        dt = x.dtype
        if dt not in (torch.float32, torch.float64):
            raise TypeError("x must be float32 or float64")
        self._x(x, dt)
        out = dict(out or {})
        dev = self.device
        if want_F and "F" not in out:
            out["F"] = torch.empty(self.B, dtype=dt, device=dev)
        if want_grad and "grad" not in out:
            out["grad"] = torch.empty(self.n, self.B, dtype=dt, device=dev)
        if want_con and "con_val" not in out:
            out["con_val"] = torch.empty(self.m, self.B, dtype=dt, device=dev)
        F, g, cv = out.get("F"), out.get("grad"), out.get("con_val")
        if want_check:
            if dt != torch.float32:
                raise TypeError("the fused check is FP32; use round_check for FP64 points")
            out.setdefault("n_sat", torch.empty(self.B, dtype=torch.int32, device=dev))
            out.setdefault("unsat_bits", torch.empty(self.B, (self.m + 31) // 32, dtype=torch.int32, device=dev))
            out.setdefault("U", torch.empty(self.m, dtype=torch.int32, device=dev))
            check(lib().ffsat_eval_check(self.handle, _ptr(x), _ptr(F), _ptr(g), _ptr(cv), _ptr(out["n_sat"]),
                                         _ptr(out["unsat_bits"]), _ptr(out["U"]), _stream(dev)))
            return out
        fn = lib().ffsat_eval if dt == torch.float32 else lib().ffsat_eval_f64
        check(fn(self.handle, _ptr(x), _ptr(F), _ptr(g), _ptr(cv), _stream(dev)))
        return out

    def step(self, x: torch.Tensor, grad: torch.Tensor, eta: float, eta_b: Optional[torch.Tensor] = None):
        """In place: x <- clip(x - eta * grad, -1, 1)."""
        dt = x.dtype
        self._x(x, dt)
        _need(grad, (self.n, self.B), dt, self.device, "grad")
        if eta_b is not None:
            _need(eta_b, (self.B,), dt, self.device, "eta_b")
        fn = lib().ffsat_step if dt == torch.float32 else lib().ffsat_step_f64
        check(fn(self.handle, _ptr(x), _ptr(grad), _ptr(eta_b), float(eta), _stream(self.device)))
        return x

    def eval_step(self, x: torch.Tensor, eta: float, want_F=True, want_check=True) -> dict:
        """One fused iteration: F, n_sat and U at x_t, then x <- clip(x - eta grad, -1, 1)."""
        self._x(x)
        dev = self.device
        out = {}
        if want_F:
            out["F"] = torch.empty(self.B, dtype=torch.float32, device=dev)
        if want_check:
            out["n_sat"] = torch.empty(self.B, dtype=torch.int32, device=dev)
            out["U"] = torch.empty(self.m, dtype=torch.int32, device=dev)
        check(lib().ffsat_eval_step(self.handle, _ptr(x), float(eta), _ptr(out.get("F")), _ptr(out.get("n_sat")),
                                    _ptr(out.get("U")), _stream(dev)))
        return out

    def run_steps(self, x: torch.Tensor, T: int, eta: float, F_last: Optional[torch.Tensor] = None):
        """T fused (gradient, projected step) iterations on x in place."""
        self._x(x)
        if F_last is not None:
            _need(F_last, (self.B,), torch.float32, self.device, "F_last")
        check(lib().ffsat_run_steps(self.handle, _ptr(x), int(T), float(eta), _ptr(F_last),
                                    _stream(self.device)))
        return x

    def round_check(self, x: torch.Tensor, want=("assign_bits", "n_sat", "unsat_bits", "U")) -> dict:
        dt = x.dtype
        self._x(x, dt)
        dev = self.device
        out = {}
        if "assign_bits" in want:
            out["assign_bits"] = torch.empty(self.B, (self.n + 31) // 32, dtype=torch.int32, device=dev)
        if "n_sat" in want:
            out["n_sat"] = torch.empty(self.B, dtype=torch.int32, device=dev)
        if "unsat_bits" in want:
            out["unsat_bits"] = torch.empty(self.B, (self.m + 31) // 32, dtype=torch.int32, device=dev)
        if "U" in want:
            out["U"] = torch.empty(self.m, dtype=torch.int32, device=dev)
        fn = lib().ffsat_round_check if dt == torch.float32 else lib().ffsat_round_check_f64
        check(fn(self.handle, _ptr(x), _ptr(out.get("assign_bits")), _ptr(out.get("n_sat")),
                 _ptr(out.get("unsat_bits")), _ptr(out.get("U")), _stream(dev)))
        return out

    def sat_weight(self, unsat_bits: torch.Tensor, w: Optional[torch.Tensor] = None) -> torch.Tensor:
        """score[b] = sum of w_c over the constraints restart b satisfies (FP64)."""
        _need(unsat_bits, (self.B, (self.m + 31) // 32), torch.int32, self.device, "unsat_bits")
        if w is not None:
            _need(w, (self.m,), torch.float32, self.device, "w")
        score = torch.empty(self.B, dtype=torch.float64, device=self.device)
        check(lib().ffsat_sat_weight(self.handle, _ptr(unsat_bits), _ptr(w), _ptr(score), _stream(self.device)))
        return score

    def erwa_update(self, U: torch.Tensor, alpha: float = 0.4) -> None:
        _need(U, (self.m,), torch.int32, self.device, "U")
        check(lib().ffsat_erwa_update(self.handle, _ptr(U), float(alpha), _stream(self.device)))

    def weight_grad(self, con_val: torch.Tensor, gF: torch.Tensor) -> torch.Tensor:
        _need(con_val, (self.m, self.B), torch.float32, self.device, "con_val")
        _need(gF, (self.B,), torch.float32, self.device, "gF")
        gw = torch.empty(self.m, dtype=torch.float32, device=self.device)
        check(lib().ffsat_weight_grad(self.handle, _ptr(con_val), _ptr(gF), _ptr(gw), _stream(self.device)))
        return gw

    def vjp(self, gF: torch.Tensor, grad: Optional[torch.Tensor] = None,
            con_val: Optional[torch.Tensor] = None) -> tuple:
        """(gx, gw) for an upstream gradient gF[B] of F (either may be None)."""
        dev = self.device
        _need(gF, (self.B,), torch.float32, dev, "gF")
        gx = torch.empty(self.n, self.B, dtype=torch.float32, device=dev) if grad is not None else None
        gw = torch.empty(self.m, dtype=torch.float32, device=dev) if con_val is not None else None
        check(lib().ffsat_vjp(self.handle, _ptr(grad), _ptr(con_val), _ptr(gF), _ptr(gx), _ptr(gw), _stream(dev)))
        return gx, gw

    def rephase(self, x: torch.Tensor, mode: int, seed: int = 0, mask: Optional[torch.Tensor] = None) -> None:
        """0: keep, 1: flip, 2: redraw uniformly (restarts with mask[b] != 0, or all)."""
        self._x(x)
        if mask is not None:
            _need(mask, (self.B,), torch.int32, self.device, "mask")
        check(lib().ffsat_rephase(self.handle, _ptr(x), int(mode), int(seed) & ((1 << 64) - 1), _ptr(mask),
                                  _stream(self.device)))

    def run_iters(self, x: torch.Tensor, T: int, eta: float, alpha: float = 0.0, out: Optional[dict] = None) -> dict:
        """T fused iterations (objective, exact check, projected step, then the
        adaptive weights when alpha > 0), replayed from a captured graph."""
        self._x(x)
        dev = self.device
        out = dict(out or {})
        out.setdefault("F", torch.empty(self.B, dtype=torch.float32, device=dev))
        out.setdefault("n_sat", torch.empty(self.B, dtype=torch.int32, device=dev))
        out.setdefault("U", torch.empty(self.m, dtype=torch.int32, device=dev))
        check(lib().ffsat_run_iters(self.handle, _ptr(x), int(T), float(eta), float(alpha), _ptr(out["F"]),
                                    _ptr(out["n_sat"]), _ptr(out["U"]), _stream(dev)))
        return out

    def fista_state(self, x: torch.Tensor, eta0: float) -> dict:
        """Fresh FISTA state for the points x: y = x, eta = eta0, t = 1."""
        self._x(x)
        return {"y": x.clone(), "eta": torch.full((self.B,), float(eta0), dtype=torch.float32, device=self.device),
                "t": torch.ones(self.B, dtype=torch.float32, device=self.device)}

    def fista_reset(self, state: dict, x: torch.Tensor, eta0: float) -> dict:
        """Restarts a FISTA state in place for the points x (same buffers)."""
        self._x(x)
        state["y"].copy_(x)
        state["eta"].fill_(float(eta0))
        state["t"].fill_(1.0)
        return state

    def fista(self, x: torch.Tensor, state: dict, T: int, max_ls: int = 15,
              F: Optional[torch.Tensor] = None) -> None:
        """T FISTA iterations with backtracking (ffsat_fista), in place on x and state."""
        self._x(x)
        self._x(state["y"])
        _need(state["eta"], (self.B,), torch.float32, self.device, "eta")
        _need(state["t"], (self.B,), torch.float32, self.device, "t")
        if F is not None:
            _need(F, (self.B,), torch.float32, self.device, "F")
        check(lib().ffsat_fista(self.handle, _ptr(x), _ptr(state["y"]), _ptr(state["eta"]), _ptr(state["t"]),
                                int(T), int(max_ls), _ptr(F), _stream(self.device)))

    def tune(self) -> None:
        check(lib().ffsat_plan_tune(self.handle, _stream(self.device)))

    def describe(self) -> dict:
        import json
        buf = C.create_string_buffer(1 << 16)
        check(lib().ffsat_plan_describe(self.handle, buf, len(buf)))
        return json.loads(buf.value.decode())

    def profile(self, on: bool = True) -> None:
        check(lib().ffsat_plan_profile(self.handle, 1 if on else 0))

    def profile_read(self, reset: bool = False) -> dict:
        import json
        buf = C.create_string_buffer(1 << 16)
        check(lib().ffsat_plan_profile_read(self.handle, 1 if reset else 0, buf, len(buf)))
        return json.loads(buf.value.decode())

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().ffsat_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def coefficients(kind: int, k: int, param: int) -> np.ndarray:
    """Host-only: conjugated coefficients h[a], a = 0..floor((k+1)/2) (complex)."""
    na = (k + 1) // 2 + 1
    buf = np.zeros(2 * na, dtype=np.float64)
    check(lib().ffsat_coefficients(int(kind), int(k), int(param), C.c_void_p(buf.ctypes.data)))
    return buf[0::2] + 1j * buf[1::2]


def walsh_coefficients(kind: int, k: int, param: int) -> np.ndarray:
    """Host-only: Walsh coefficients f^_j of e_j, j = 0..k (exact, rounded once)."""
    buf = np.zeros(k + 1, dtype=np.float64)
    check(lib().ffsat_walsh_coefficients(int(kind), int(k), int(param), C.c_void_p(buf.ctypes.data)))
    return buf


def unit_circle_coefficients(kind: int, k: int, param: int) -> np.ndarray:
    """Host-only: conjugated Walsh coefficients f~[a] of the unit-circle form, a = 0..k (complex)."""
    buf = np.zeros(2 * (k + 1), dtype=np.float64)
    check(lib().ffsat_unit_circle_coefficients(int(kind), int(k), int(param), C.c_void_p(buf.ctypes.data)))
    return buf[0::2] + 1j * buf[1::2]
