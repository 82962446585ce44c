"""CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It never imports the HIP
library and the HIP library never imports it.

``oracle.c`` is the FP64 C implementation (count-lattice recursion, ESP
recurrence with exact Walsh coefficients, closed forms, checker, projected
step, adaptive weights, weight gradient, finite differences); ``exact.py``
holds exact rational versions for tiny inputs.  This module compiles
``oracle.c`` with gcc and wraps it with ctypes and numpy.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ROUTE_AUTH, ROUTE_DP, ROUTE_ESP, ROUTE_CLOSED = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, -O2, OpenMP)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
           "-ffp-contract=off", SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        d, i, u, p = C.c_double, C.c_int, C.c_uint32, C.c_void_p
        L.orc_truth.restype = d
        L.orc_truth.argtypes = [i, i, i, i]
        L.orc_we_dp.restype = d
        L.orc_we_dp.argtypes = [i, p, p, p]
        L.orc_prob_at_least.restype = d
        L.orc_prob_at_least.argtypes = [i, p, i]
        L.orc_walsh_coeffs.restype = i
        L.orc_walsh_coeffs.argtypes = [i, p, p]
        L.orc_esp.restype = None
        L.orc_esp.argtypes = [i, p, p]
        L.orc_we_esp.restype = d
        L.orc_we_esp.argtypes = [i, p, p, p]
        L.orc_we_closed.restype = i
        L.orc_we_closed.argtypes = [i, i, i, p, p, p]
        L.orc_constraint.restype = d
        L.orc_constraint.argtypes = [i, i, i, p, p, i]
        L.orc_eval.restype = i
        L.orc_eval.argtypes = [i, i, p, p, p, p, p, i, p, p, p, p, p, i, i]
        L.orc_fd_grad.restype = None
        L.orc_fd_grad.argtypes = [i, p, p, p, p, p, p, p, i, p, i, p, p, d, p]
        L.orc_check.restype = None
        L.orc_check.argtypes = [i, i, p, p, p, p, i, p, p, p, p, p]
        L.orc_step_f32.restype = None
        L.orc_step_f32.argtypes = [i, i, p, p, p, C.c_float]
        L.orc_step_f64.restype = None
        L.orc_step_f64.argtypes = [i, i, p, p, p, d]
        L.orc_erwa.restype = None
        L.orc_erwa.argtypes = [i, p, p, d]
        L.orc_wgrad.restype = None
        L.orc_wgrad.argtypes = [i, i, p, p, p]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- single constraint

def truth_table(kind: int, param: int, k: int) -> np.ndarray:
    L = lib()
    return np.array([L.orc_truth(kind, param, k, c) for c in range(k + 1)])


def we_dp(l, fv, grad=True):
    l, fv = _f64(l), _f64(fv)
    k = l.shape[0]
    dl = np.zeros(k) if grad else None
    we = lib().orc_we_dp(k, _p(l), _p(fv), _p(dl))
    return (we, dl) if grad else we


def prob_at_least(l, t):
    l = _f64(l)
    return lib().orc_prob_at_least(l.shape[0], _p(l), int(t))


def walsh_coeffs(fv):
    fv = _f64(fv)
    k = fv.shape[0] - 1
    out = np.zeros(k + 1)
    if lib().orc_walsh_coeffs(k, _p(fv), _p(out)) != 0:
        raise ValueError("exact Walsh coefficients need k <= 62")
    return out


def esp(l):
    l = _f64(l)
    e = np.zeros(l.shape[0] + 1)
    lib().orc_esp(l.shape[0], _p(l), _p(e))
    return e


def we_esp(l, fhat, grad=True):
    l, fhat = _f64(l), _f64(fhat)
    k = l.shape[0]
    dl = np.zeros(k) if grad else None
    we = lib().orc_we_esp(k, _p(l), _p(fhat), _p(dl))
    return (we, dl) if grad else we


def we_closed(kind, param, l, grad=True):
    l = _f64(l)
    k = l.shape[0]
    out = np.zeros(1)
    dl = np.zeros(k) if grad else None
    if lib().orc_we_closed(kind, param, k, _p(l), _p(out), _p(dl)) != 0:
        return None
    return (out[0], dl) if grad else out[0]


def constraint(kind, param, l, route=ROUTE_AUTH, grad=True):
    l = _f64(l)
    k = l.shape[0]
    dl = np.zeros(k) if grad else None
    we = lib().orc_constraint(kind, param, k, _p(l), _p(dl), route)
    return (we, dl) if grad else we


# ---------------------------------------------------------------- whole formula

def _inst_arrays(inst):
    return (np.ascontiguousarray(inst.con_ptr, np.int64), np.ascontiguousarray(inst.lits, np.int32),
            np.ascontiguousarray(inst.kinds, np.int32), np.ascontiguousarray(inst.params, np.int32))


def eval_batch(inst, x, w=None, *, route=ROUTE_AUTH, want_g=True, want_con=False,
               want_lit=False, nthreads=0):
    """Returns dict with F[B], g[n][B], con_val[m][B], lit_grad[nnz][B] (as asked)
    and the thread count used."""
    cp, lits, kinds, params = _inst_arrays(inst)
    x = _f64(x)
    n, B = x.shape
    assert n == inst.n_vars
    if w is None:
        w = inst.weights
    wd = None if w is None else _f64(w)
    F = np.zeros(B)
    g = np.zeros((n, B)) if want_g else None
    cv = np.zeros((inst.m, B)) if want_con else None
    lg = np.zeros((inst.nnz, B)) if want_lit else None
    used = lib().orc_eval(n, inst.m, _p(cp), _p(lits), _p(kinds), _p(params), _p(wd), B, _p(x),
                          _p(F), _p(g), _p(cv), _p(lg), route, nthreads)
    return {"F": F, "g": g, "con_val": cv, "lit_grad": lg, "threads": used}


def var_incidence(inst):
    """variable -> constraints CSR (0-based), in constraint order."""
    lens = np.diff(inst.con_ptr)
    con_of_slot = np.repeat(np.arange(inst.m, dtype=np.int32), lens)
    var_of_slot = np.abs(inst.lits).astype(np.int64) - 1
    order = np.argsort(var_of_slot, kind="stable")
    counts = np.bincount(var_of_slot, minlength=inst.n_vars)
    ptr = np.zeros(inst.n_vars + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return ptr, np.ascontiguousarray(con_of_slot[order], np.int32)


def fd_grad(inst, x, sample_var, sample_b, w=None, h=1e-6):
    cp, lits, kinds, params = _inst_arrays(inst)
    x = _f64(x)
    n, B = x.shape
    vp, vc = var_incidence(inst)
    if w is None:
        w = inst.weights
    wd = None if w is None else _f64(w)
    sv = np.ascontiguousarray(sample_var, np.int32)
    sb = np.ascontiguousarray(sample_b, np.int32)
    out = np.zeros(sv.shape[0])
    lib().orc_fd_grad(n, _p(cp), _p(lits), _p(kinds), _p(params), _p(wd), _p(vp), _p(vc), B,
                      _p(x), sv.shape[0], _p(sv), _p(sb), float(h), _p(out))
    return out


def check(inst, x):
    """Integer checker on the rounded point (x_v < 0 means True)."""
    cp, lits, kinds, params = _inst_arrays(inst)
    x = _f64(x)
    n, B = x.shape
    wn, wm = (n + 31) // 32, (inst.m + 31) // 32
    ab = np.zeros((B, wn), np.uint32)
    ns = np.zeros(B, np.int32)
    ub = np.zeros((B, wm), np.uint32)
    U = np.zeros(inst.m, np.int32)
    lib().orc_check(n, inst.m, _p(cp), _p(lits), _p(kinds), _p(params), B, _p(x), _p(ab), _p(ns),
                    _p(ub), _p(U))
    return {"assign_bits": ab, "n_sat": ns, "unsat_bits": ub, "U": U}


def step_f32(x, g, eta, eta_b=None):
    x = np.array(x, dtype=np.float32, order="C", copy=True)
    g = np.ascontiguousarray(g, np.float32)
    eb = None if eta_b is None else np.ascontiguousarray(eta_b, np.float32)
    n, B = x.shape
    lib().orc_step_f32(n, B, _p(x), _p(g), _p(eb), float(eta))
    return x


def step_f64(x, g, eta, eta_b=None):
    x = np.array(x, dtype=np.float64, order="C", copy=True)
    g = _f64(g)
    eb = None if eta_b is None else _f64(eta_b)
    n, B = x.shape
    lib().orc_step_f64(n, B, _p(x), _p(g), _p(eb), float(eta))
    return x


def erwa(U, w, alpha=0.4):
    U = np.ascontiguousarray(U, np.int32)
    w = np.array(w, dtype=np.float64, copy=True)
    lib().orc_erwa(U.shape[0], _p(U), _p(w), float(alpha))
    return w


def wgrad(con_val, gF):
    cv = _f64(con_val)
    gF = _f64(gF)
    m, B = cv.shape
    gw = np.zeros(m)
    lib().orc_wgrad(m, B, _p(cv), _p(gF), _p(gw))
    return gw
