"""Oracle pinned to the values the paper prints for its worked examples."""
from fractions import Fraction

import numpy as np
import pytest

from conftest import frac, load_golden
from oracle import exact

pytestmark = pytest.mark.filterwarnings("ignore")


def _lits_to_l(lits, x):
    return np.array([x[abs(v) - 1] if v > 0 else -x[abs(v) - 1] for v in lits], dtype=np.float64)


def test_card_example_walsh_coefficients(orc):
    g = load_golden("card4_t2_example.json")
    c = g["constraint"]
    k = len(c["lits"])
    fv = orc.truth_table(c["kind"], c["param"], k)
    fhat = orc.walsh_coeffs(fv)                         # e_0 .. e_k
    want = [float(frac(s)) for s in reversed(g["walsh_coeffs_e4_to_e0"])]
    assert np.array_equal(fhat, np.array(want))
    # the exact Thm. 1 sum over the cube agrees too
    assert [Fraction(v) for v in exact.walsh_coeffs_by_size(c["kind"], c["param"], k)] == \
        [frac(s) for s in reversed(g["walsh_coeffs_e4_to_e0"])]


@pytest.mark.parametrize("route", [0, 1, 2])
def test_card_example_value_and_gradient(orc, route):
    g = load_golden("card4_t2_example.json")
    c = g["constraint"]
    x = np.array([float(frac(s)) for s in g["point"]])
    l = _lits_to_l(c["lits"], x)
    we, dl = orc.constraint(c["kind"], c["param"], l, route=route)
    assert we == float(frac(g["we"]))
    assert np.array_equal(dl, np.array([float(frac(s)) for s in g["grad"]]))


def test_card_example_probabilities(orc):
    g = load_golden("card4_t2_example.json")
    c = g["constraint"]
    x = np.array([float(frac(s)) for s in g["point"]])
    l = _lits_to_l(c["lits"], x)
    p_true = orc.prob_at_least(l, c["param"])
    assert p_true == float(frac(g["p_true"]))
    assert 1.0 - p_true == float(frac(g["p_false"]))
    # the expansion is P(false) - P(true)
    assert float(frac(g["p_false"]) - frac(g["p_true"])) == float(frac(g["we"]))


def test_card_example_exact(orc):
    g = load_golden("card4_t2_example.json")
    c = g["constraint"]
    pt = [frac(s) for s in g["point"]]
    assert exact.we_lagrange(c["kind"], c["param"], pt) == frac(g["we"])
    assert exact.we_from_coeffs(c["kind"], c["param"], pt) == frac(g["we"])
    assert exact.grad_lagrange(c["kind"], c["param"], pt) == [frac(s) for s in g["grad"]]


def _poly_eval(poly, x1, x2):
    return (frac(poly["1"]) + frac(poly["x1"]) * x1 + frac(poly["x2"]) * x2
            + frac(poly["x1x2"]) * x1 * x2)


def _inst_from(constraints, n):
    from workloads import assemble
    groups = [(c["kind"], [c["param"]], [np.array(c["lits"], dtype=np.int32)]) for c in constraints]
    return assemble(n, groups)


def test_saddle_example(orc):
    g = load_golden("saddle_example.json")
    inst = _inst_from(g["constraints"], 2)
    rng = np.random.default_rng(5)
    # the oracle's objective is the printed polynomial (compare at random points)
    pts = rng.uniform(-1, 1, size=(2, 16))
    F = orc.eval_batch(inst, pts)["F"]
    want = [float(_poly_eval(g["F_poly"], Fraction(pts[0, b]), Fraction(pts[1, b]))) for b in range(16)]
    assert np.allclose(F, want, rtol=0, atol=1e-15)
    # the saddle point has zero gradient
    s = np.array([[float(frac(v))] for v in g["saddle"]])
    out = orc.eval_batch(inst, s)
    assert np.allclose(out["g"][:, 0], 0.0, atol=1e-15)
    # scores and adapted weights
    chk = orc.check(inst, s)
    U = chk["U"]
    assert list(U) == [int(frac(v)) for v in g["r"]]
    w1 = orc.erwa(U, [float(frac(v)) for v in g["w0"]], alpha=float(frac(g["alpha"])))
    assert np.allclose(w1, [float(frac(v)) for v in g["w1"]], rtol=0, atol=1e-15)
    # adapted objective equals the printed adapted polynomial; its gradient at
    # the saddle is what that polynomial gives (the printed gradient is not used)
    F1 = orc.eval_batch(inst, pts, w=w1)["F"]
    want1 = [float(_poly_eval(g["F1_poly"], Fraction(pts[0, b]), Fraction(pts[1, b]))) for b in range(16)]
    assert np.allclose(F1, want1, rtol=0, atol=1e-15)
    p = g["F1_poly"]
    x1, x2 = (frac(v) for v in g["saddle"])
    gx1 = frac(p["x1"]) + frac(p["x1x2"]) * x2
    gx2 = frac(p["x2"]) + frac(p["x1x2"]) * x1
    assert (gx1, gx2) == (Fraction(-2, 15), Fraction(2, 15))
    g1 = orc.eval_batch(inst, s, w=w1)["g"][:, 0]
    assert np.allclose(g1, [float(gx1), float(gx2)], rtol=0, atol=1e-15)


def test_local_optimum_example(orc):
    g = load_golden("local_optimum_example.json")
    inst = _inst_from(g["constraints"], 4)
    rng = np.random.default_rng(6)
    pts = rng.uniform(-1, 1, size=(4, 8))
    F = orc.eval_batch(inst, pts)["F"]
    want = [sum(float(frac(cf)) * pts[int(a[1]) - 1, b] * pts[int(bb[1]) - 1, b]
                for (a, bb), cf in g["F_poly_terms"]) for b in range(8)]
    assert np.allclose(F, want, rtol=0, atol=1e-15)
    x = np.array([[float(frac(v))] for v in g["point"]])
    U = orc.check(inst, x)["U"]
    assert list(U) == [int(frac(v)) for v in g["r"]]
    w1 = orc.erwa(U, [float(frac(v)) for v in g["w0"]], alpha=float(frac(g["alpha"])))
    assert np.allclose(w1, [float(frac(v)) for v in g["w1"]], rtol=0, atol=1e-15)
    g1 = orc.eval_batch(inst, x, w=w1)["g"][:, 0]
    assert np.allclose(g1, [float(frac(v)) for v in g["grad_F1"]], rtol=0, atol=1e-15)


def test_esp_is_the_convolution_of_pairs(orc):
    # Eq. convolution: esp = [l1,1] * ... * [lk,1] (highest degree first)
    rng = np.random.default_rng(7)
    for k in (1, 2, 5, 9):
        l = [Fraction(int(v), 16) for v in rng.integers(-16, 17, size=k)]
        conv = exact.esp_convolution(l)
        e = orc.esp(np.array([float(v) for v in l]))
        assert np.allclose(e, [float(v) for v in reversed(conv)], rtol=0, atol=1e-14)
