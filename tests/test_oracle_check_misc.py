"""Oracle checker, projected step, adaptive weights and weight gradient,
pinned to Thm. 1/Thm. 2, Prop. 3's definition and the linearity of Def. 3."""
import numpy as np
import pytest

from workloads import points, random_hybrid


def _small_inst(seed=0, n=30):
    return random_hybrid(n, seed, n_or=40, or_len=(1, 5), n_xor=15, xor_len=(1, 6),
                         n_card=12, card_len=(2, 9), card_t=(0, 10), weights="uniform")


def test_checker_matches_expansion_at_corners(orc):
    """At a corner, WE_c = -1 iff c is satisfied (Thm. 1), so the checker's
    verdicts must equal the signs of the oracle's per-constraint values."""
    inst = _small_inst(1)
    x = points(inst.n_vars, 64, 2, dist="corner", dtype=np.float64)
    out = orc.eval_batch(inst, x, want_con=True, want_g=False)
    chk = orc.check(inst, x)
    sat = out["con_val"] < 0
    assert np.all(np.abs(np.abs(out["con_val"]) - 1.0) < 1e-12)
    assert np.array_equal(chk["n_sat"], sat.sum(0).astype(np.int32))
    assert np.array_equal(chk["U"], (~sat).sum(1).astype(np.int32))
    m = inst.m
    bits = np.unpackbits(chk["unsat_bits"].view(np.uint8), axis=1, bitorder="little")[:, :m]
    assert np.array_equal(bits.T.astype(bool), ~sat)
    # certificate (Thm. 2): all satisfied iff F(sgn x) = -sum w
    w = inst.weights.astype(np.float64)
    F = (w[:, None] * out["con_val"]).sum(0)
    assert np.array_equal(np.isclose(F, -w.sum(), atol=1e-9), chk["n_sat"] == m)


def test_checker_rounds_variables_not_literals(orc):
    """x_v < 0 means True; +0 and -0 are False for the variable, so a
    negated literal of a zero variable is True."""
    from workloads import assemble
    inst = assemble(2, [(0, [0, 0], [np.array([-1], np.int32), np.array([2], np.int32)])])
    x = np.array([[0.0, -0.0, 1e-30, -1e-30], [0.0, -0.0, -1e-30, 1e-30]])
    chk = orc.check(inst, x)
    # clause 0 = NOT x1: true iff x1 >= 0 ; clause 1 = x2: true iff x2 < 0
    assert list(chk["n_sat"]) == [1, 1, 2, 0]
    bits = chk["assign_bits"][:, 0]
    assert list(bits) == [0, 0, 2, 1]


def test_checker_agrees_with_rounded_point(orc):
    """Checking x equals checking sgn(x) (with x < 0 -> -1)."""
    inst = _small_inst(4)
    x = points(inst.n_vars, 32, 5, dist="mixed_edge", dtype=np.float64)
    r = np.where(x < 0, -1.0, 1.0)
    a, b = orc.check(inst, x), orc.check(inst, r)
    for key in ("n_sat", "unsat_bits", "U", "assign_bits"):
        assert np.array_equal(a[key], b[key])


def test_step_f32_examples(orc):
    x = np.array([[0.9, -0.9, 0.0, 0.5]], np.float32)
    g = np.array([[-1.0, 1.0, 0.25, -0.5]], np.float32)
    out = orc.step_f32(x, g, 0.5)
    assert out.tolist() == [[1.0, -1.0, -0.125, 0.75]]
    eb = np.array([0.0, 0.1, 2.0, 4.0], np.float32)
    out = orc.step_f32(x, g, 99.0, eta_b=eb)
    assert out[0, 0] == np.float32(0.9) and out[0, 2] == -0.5 and out[0, 3] == 1.0


def test_step_f64_is_clip(orc):
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (5, 7))
    g = rng.normal(size=(5, 7))
    out = orc.step_f64(x, g, 0.3)
    assert np.allclose(out, np.clip(x - 0.3 * g, -1, 1), rtol=0, atol=1e-15)


def test_erwa_recurrence_equals_weighted_average(orc):
    """Prop. 3's recurrence reproduces the ERWA sum
    w(t) = (1-a)^t w(0) + sum_i a (1-a)^(t-i) r(i)."""
    rng = np.random.default_rng(8)
    m, T, a = 20, 6, 0.4
    w0 = rng.uniform(0.5, 1.5, m)
    Us = rng.integers(0, 9, size=(T, m)).astype(np.int32)
    Us[3] = 0                    # a round where every restart satisfied everything
    w = w0.copy()
    for t in range(T):
        w = orc.erwa(Us[t], w, a)
    rs = [U / U.max() if U.max() > 0 else np.zeros(m) for U in Us.astype(np.float64)]
    want = (1 - a) ** T * w0 + sum(a * (1 - a) ** (T - 1 - i) * rs[i] for i in range(T))
    assert np.allclose(w, want, rtol=0, atol=1e-14)


def test_erwa_zero_counts_decay(orc):
    w = orc.erwa(np.zeros(4, np.int32), np.ones(4), 0.4)
    assert np.allclose(w, 0.6)


def test_weight_gradient_is_derivative_in_w(orc):
    """F is linear in w (Def. 3): d(sum_b gF_b F_b)/dw_c by differences."""
    inst = _small_inst(6)
    x = points(inst.n_vars, 8, 7, dtype=np.float64)
    out = orc.eval_batch(inst, x, want_con=True, want_g=False)
    gF = np.random.default_rng(1).normal(size=8)
    gw = orc.wgrad(out["con_val"], gF)
    w = inst.weights.astype(np.float64)
    for c in (0, 5, inst.m - 1):
        e = np.zeros(inst.m)
        e[c] = 0.25
        Fp = orc.eval_batch(inst, x, w=w + e, want_g=False)["F"]
        Fm = orc.eval_batch(inst, x, w=w - e, want_g=False)["F"]
        assert abs(gF @ (Fp - Fm) / 0.5 - gw[c]) < 1e-12


def test_eval_thread_count_invariance(orc):
    inst = _small_inst(9)
    x = points(inst.n_vars, 16, 3, dtype=np.float64)
    a = orc.eval_batch(inst, x, nthreads=1)
    b = orc.eval_batch(inst, x, nthreads=4)
    assert np.array_equal(a["F"], b["F"]) and np.array_equal(a["g"], b["g"])
