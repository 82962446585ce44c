"""The C-ABI library: exports, validation and host-only helpers (no GPU)."""
import ctypes as C

import numpy as np
import pytest

from paper_2308_15020_amd import _lib
from workloads import assemble, random_hybrid


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    names = _lib.header_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    # and the binding declares a signature for each
    assert set(names) == set(_lib._SIGS)


def test_status_strings(L):
    for code in _lib.STATUS:
        s = L.ffsat_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.ffsat_status_string(12345).decode() == "unknown status"


def _create(L, inst, device=0, weights=None, fp64_min_len=0, flags=0):
    cp = np.ascontiguousarray(inst.con_ptr, np.int64)
    li = np.ascontiguousarray(inst.lits, np.int32)
    ki = np.ascontiguousarray(inst.kinds, np.int32)
    pa = np.ascontiguousarray(inst.params, np.int32)
    w = None if weights is None else np.ascontiguousarray(weights, np.float32)
    d = _lib.ProblemDesc(inst.n_vars, inst.m, cp.ctypes.data, li.ctypes.data, ki.ctypes.data,
                         pa.ctypes.data, None if w is None else w.ctypes.data, device,
                         fp64_min_len, flags)
    h = C.c_void_p()
    st = L.ffsat_problem_create(C.byref(d), C.byref(h))
    return st, h


def _one(lits, kind=0, param=0, n=5):
    return assemble(n, [(kind, [param], [np.array(lits, np.int32)])])


@pytest.mark.parametrize("lits,code", [
    ([1, 6], "E_VAR_RANGE"),
    ([0, 1], "E_VAR_RANGE"),
    ([-6], "E_VAR_RANGE"),
    ([2, -2], "E_DUP_VAR"),
    ([3, 1, 3], "E_DUP_VAR"),
])
def test_validation_errors(L, lits, code):
    st, h = _create(L, _one(lits))
    assert _lib.STATUS[st] == code
    assert h.value is None                       # *out untouched on failure
    assert L.ffsat_last_error().decode()


def test_empty_constraint_and_bad_kind(L):
    inst = _one([1, 2])
    inst.con_ptr = np.array([0, 0, 2], np.int64)
    inst.kinds = np.array([0, 0], np.int32)
    inst.params = np.array([0, 0], np.int32)
    st, _ = _create(L, inst)
    assert _lib.STATUS[st] == "E_EMPTY_CONSTRAINT"
    st, _ = _create(L, _one([1, 2], kind=7))
    assert _lib.STATUS[st] == "E_BAD_KIND"


def test_too_long_constraint(L):
    inst = random_hybrid(600, 1, n_or=1, or_len=(513, 513))
    st, _ = _create(L, inst)
    assert _lib.STATUS[st] == "E_UNSUPPORTED"


def test_bad_sizes_and_nulls(L):
    inst = _one([1, 2])
    inst.n_vars = 0
    st, _ = _create(L, inst)
    assert _lib.STATUS[st] == "E_INVALID_ARG"
    h = C.c_void_p()
    assert _lib.STATUS[L.ffsat_problem_create(None, C.byref(h))] == "E_INVALID_ARG"
    st, _ = _create(L, _one([1, 2]), weights=np.array([np.nan], np.float32))
    assert _lib.STATUS[st] == "E_INVALID_ARG"
    # every call rejects NULL handles without touching a device
    assert _lib.STATUS[L.ffsat_plan_create(None, 4, None, C.byref(h))] == "E_INVALID_ARG"
    assert _lib.STATUS[L.ffsat_eval(None, None, None, None, None, None)] == "E_INVALID_ARG"
    assert _lib.STATUS[L.ffsat_eval_f64(None, None, None, None, None, None)] == "E_INVALID_ARG"
    assert _lib.STATUS[L.ffsat_step(None, None, None, None, 0.1, None)] == "E_INVALID_ARG"
    assert _lib.STATUS[L.ffsat_run_steps(None, None, 1, 0.1, None, None)] == "E_INVALID_ARG"
    assert _lib.STATUS[L.ffsat_round_check(None, None, None, None, None, None, None)] == "E_INVALID_ARG"
    assert _lib.STATUS[L.ffsat_erwa_update(None, None, 0.4, None)] == "E_INVALID_ARG"
    assert _lib.STATUS[L.ffsat_weight_grad(None, None, None, None, None)] == "E_INVALID_ARG"
    assert L.ffsat_problem_destroy(None) == 0 and L.ffsat_plan_destroy(None) == 0


@pytest.mark.parametrize("k", [1, 2, 3, 4, 7, 8, 31, 100, 257, 512])
def test_coefficients_invert_to_truth_table(k, orc):
    """The host coefficient generator: the inverse transform of h (with the
    conjugate-symmetric half) gives back f(c) for c = 0..k."""
    from paper_2308_15020_amd.api import coefficients
    N = k + 1
    for kind, t in [(0, 0), (1, 0), (1, 1), (2, 1), (2, max(1, k // 2)), (2, k), (2, 0), (2, k + 1)]:
        h = coefficients(kind, k, t)
        c = np.arange(k + 1)
        rec = np.full(k + 1, h[0].real)
        for a in range(1, (N + 1) // 2):
            rec += 2 * (h[a] * np.exp(2j * np.pi * a * c / N)).real
        if N % 2 == 0:
            rec += (h[N // 2] * (-1.0) ** c).real
        want = orc.truth_table(kind, t, k)
        assert np.max(np.abs(rec - want)) < 1e-12, (kind, t)


def test_coefficients_worked_example_card(orc):
    """x1+..+x4 >= 2: h relates to the paper's Walsh coefficients through the
    count distribution; check the value -59/128 at (1/2,1/2,-1/2,-1/2) by
    evaluating prod_i ((1+l_i)/2 + (1-l_i)/2 z) at the roots of unity."""
    from paper_2308_15020_amd.api import coefficients
    k, N = 4, 5
    h = coefficients(2, k, 2)
    l = np.array([0.5, 0.5, -0.5, -0.5])
    we = h[0].real
    for a in range(1, 3):
        z = np.exp(2j * np.pi * a / N)
        G = np.prod((1 + l) / 2 + (1 - l) / 2 * z)
        we += 2 * (h[a] * G).real
    assert abs(we - (-59 / 128)) < 1e-15
