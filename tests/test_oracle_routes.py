"""Oracle routes pinned to the cube, closed forms, exact rationals and
invariants of the Walsh expansion (all CPU)."""
from fractions import Fraction
from itertools import product
from math import comb

import numpy as np
import pytest

from oracle import exact

KINDS = [(0, 0), (1, 0), (1, 1), (2, 1), (2, 2), (2, 3), (2, 0), (2, 99)]


def _constraints(k):
    out = [(0, 0), (1, 0), (1, 1)]
    out += [(2, t) for t in range(-1, k + 2)]
    return out


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_corners_equal_truth_table(orc, k):
    """Thm. 1: the expansion agrees with the constraint on every corner."""
    for kind, t in _constraints(k):
        for a in product((-1.0, 1.0), repeat=k):
            l = np.array(a)
            want = exact.f_on_point(kind, t, a)
            for route in (orc.ROUTE_AUTH, orc.ROUTE_DP, orc.ROUTE_ESP):
                we = orc.constraint(kind, t, l, route=route, grad=False)
                assert we == want, (kind, t, a, route)


@pytest.mark.parametrize("k", [1, 2, 4, 6, 9])
def test_dp_and_esp_against_exact_lagrange(orc, k):
    rng = np.random.default_rng(100 + k)
    for kind, t in _constraints(k):
        for _ in range(3):
            pt = [Fraction(int(v), 64) for v in rng.integers(-64, 65, size=k)]
            l = np.array([float(v) for v in pt])
            we_x = exact.we_lagrange(kind, t, pt)
            gr_x = exact.grad_lagrange(kind, t, pt)
            for route in (orc.ROUTE_DP, orc.ROUTE_ESP, orc.ROUTE_AUTH):
                we, dl = orc.constraint(kind, t, l, route=route)
                assert abs(we - float(we_x)) <= 1e-15, (kind, t, route)
                assert np.max(np.abs(dl - np.array([float(v) for v in gr_x]))) <= 1e-15


@pytest.mark.parametrize("k", [1, 3, 6])
def test_walsh_coeffs_against_thm1_sum(orc, k):
    for kind, t in _constraints(k):
        fv = orc.truth_table(kind, t, k)
        fh = orc.walsh_coeffs(fv)
        want = exact.walsh_coeffs_by_size(kind, t, k)
        assert np.array_equal(fh, np.array([float(v) for v in want]))


@pytest.mark.parametrize("k", [1, 7, 20, 40, 62])
def test_parseval(orc, k):
    """f^2 = 1 on the cube, so sum_S fhat(S)^2 = 1 (Parseval)."""
    for kind, t in [(0, 0), (1, 1), (2, 1), (2, k // 2), (2, k)]:
        fh = orc.walsh_coeffs(orc.truth_table(kind, t, k))
        s = sum(comb(k, j) * fh[j] ** 2 for j in range(k + 1))
        assert abs(s - 1.0) < 1e-12


def test_walsh_xor_is_single_top_term(orc):
    # XOR has only the highest-order term (App. Transform-free, Cor. 3)
    for k in (1, 5, 30):
        fh = orc.walsh_coeffs(orc.truth_table(1, 1, k))
        assert fh[k] == 1.0 and np.all(fh[:k] == 0)


@pytest.mark.parametrize("k", [2, 11, 64, 200, 512])
def test_dp_multilinearity(orc, k):
    """WE is affine in each literal: dWE/dl_i = (WE|l_i=1 - WE|l_i=-1)/2."""
    rng = np.random.default_rng(k)
    for kind, t in [(0, 0), (1, 1), (2, max(1, k // 3)), (2, max(1, k // 2))]:
        l = rng.uniform(-1, 1, size=k)
        _, dl = orc.constraint(kind, t, l, route=orc.ROUTE_DP)
        for i in rng.choice(k, size=min(k, 5), replace=False):
            hi, lo = l.copy(), l.copy()
            hi[i], lo[i] = 1.0, -1.0
            d = 0.5 * (orc.constraint(kind, t, hi, route=orc.ROUTE_DP, grad=False)
                       - orc.constraint(kind, t, lo, route=orc.ROUTE_DP, grad=False))
            assert abs(d - dl[i]) < 1e-13


@pytest.mark.parametrize("k", [1, 2, 16, 64, 128, 300])
def test_closed_forms_against_dp(orc, k):
    rng = np.random.default_rng(7 * k)
    for kind, t in [(0, 0), (1, 0), (1, 1), (2, 1), (2, k), (2, 0), (2, k + 1)]:
        for dist in ("uniform", "corner", "near"):
            if dist == "uniform":
                l = rng.uniform(-1, 1, size=k)
            elif dist == "corner":
                l = rng.choice([-1.0, 1.0], size=k)
            else:
                l = rng.choice([-0.99, 0.99], size=k)
            we_c, dl_c = orc.constraint(kind, t, l, route=orc.ROUTE_CLOSED)
            we_d, dl_d = orc.constraint(kind, t, l, route=orc.ROUTE_DP)
            assert abs(we_c - we_d) < 1e-13
            assert np.max(np.abs(dl_c - dl_d)) < 1e-13


@pytest.mark.parametrize("k", [10, 24, 40])
def test_esp_route_against_dp(orc, k):
    """R1 (ESP recurrence) and R2 agree where R1 is well conditioned."""
    rng = np.random.default_rng(11 * k)
    for kind, t in [(0, 0), (1, 1), (2, 1), (2, k // 4), (2, k // 2), (2, k)]:
        for dist in ("uniform", "near"):
            l = rng.uniform(-1, 1, size=k) if dist == "uniform" else rng.choice([-0.99, 0.99], size=k)
            we_e, dl_e = orc.constraint(kind, t, l, route=orc.ROUTE_ESP)
            we_d, dl_d = orc.constraint(kind, t, l, route=orc.ROUTE_DP)
            assert abs(we_e - we_d) < 1e-10
            assert np.max(np.abs(dl_e - dl_d)) < 1e-10


def test_value_at_origin(orc):
    """WE(0) = 2^-k sum_c C(k,c) f(c): the cube average of f."""
    for k in (1, 5, 33, 100):
        for kind, t in [(0, 0), (1, 1), (2, k // 2 + 1)]:
            fv = orc.truth_table(kind, t, k)
            want = sum(comb(k, c) * fv[c] for c in range(k + 1)) / 2.0 ** k
            we = orc.constraint(kind, t, np.zeros(k), route=orc.ROUTE_DP, grad=False)
            assert abs(we - want) < 1e-15


def test_range_on_the_box(orc):
    rng = np.random.default_rng(3)
    for k in (3, 50, 257):
        for kind, t in [(0, 0), (1, 0), (2, k // 3)]:
            for _ in range(5):
                we, dl = orc.constraint(kind, t, rng.uniform(-1, 1, size=k))
                assert -1.0 <= we <= 1.0
                assert np.all(np.abs(dl) <= 1.0)


def test_gradient_against_central_differences(orc):
    from workloads import random_hybrid, points
    inst = random_hybrid(60, 9, n_or=80, or_len=(2, 6), n_xor=20, xor_len=(2, 9),
                         n_card=15, card_len=(5, 30), weights="uniform")
    x = points(60, 4, 99, dtype=np.float64) * 0.9
    out = orc.eval_batch(inst, x)
    rng = np.random.default_rng(1)
    sv = rng.integers(0, 60, size=40)
    sb = rng.integers(0, 4, size=40)
    fd = orc.fd_grad(inst, x, sv, sb, h=1e-6)
    assert np.max(np.abs(fd - out["g"][sv, sb])) < 1e-8


def test_objective_is_weighted_sum(orc):
    """Def. 3 and the gradient bookkeeping: F = sum_c w_c WE_c and
    g_v = sum over slots of v of w_c s_i dWE_c/dl_i."""
    from workloads import random_hybrid, points
    inst = random_hybrid(40, 3, n_or=50, or_len=(1, 5), n_xor=10, xor_len=(1, 6),
                         n_card=10, card_len=(3, 12), weights="uniform")
    x = points(40, 3, 4, dtype=np.float64)
    out = orc.eval_batch(inst, x, want_con=True, want_lit=True)
    w = inst.weights.astype(np.float64)
    assert np.allclose(out["F"], (w[:, None] * out["con_val"]).sum(0), rtol=0, atol=1e-13)
    g = np.zeros_like(x)
    lens = np.diff(inst.con_ptr)
    con_of_slot = np.repeat(np.arange(inst.m), lens)
    for s, lit in enumerate(inst.lits):
        v = abs(lit) - 1
        g[v] += w[con_of_slot[s]] * np.sign(lit) * out["lit_grad"][s]
    assert np.allclose(out["g"], g, rtol=0, atol=1e-13)
