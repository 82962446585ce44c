"""Host tables of the unit-circle form (the paper's own basis, kept as an
ablation): the exact Walsh coefficients f^_j and the conjugated Walsh
coefficients f~ = f^ W^-1.  Pure host code in the library, no GPU."""
import json
import os
from fractions import Fraction
from math import comb

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def P():
    import paper_2308_15020_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


def _krawtchouk_walsh(fv, k):
    """f^_j = 2^-k sum_c f(c) C(k,c) K_j(c) / C(k,j) in Python integers
    (the Krawtchouk sum over counts, straight from the definition)."""
    out = []
    for j in range(k + 1):
        num = 0
        for c in range(k + 1):
            kj = sum((-1) ** q * comb(c, q) * comb(k - c, j - q) for q in range(j + 1))
            num += int(fv[c]) * comb(k, c) * kj
        out.append(float(Fraction(num, 2 ** k * comb(k, j))))
    return np.array(out)


def test_walsh_worked_example(P):
    """Example 1: x1+x2+x3+x4 >= 2 has f^ = (-3/8, 3/8, 1/8, -1/8, -3/8) for e_0..e_4."""
    with open(os.path.join(GOLD, "card4_t2_example.json")) as f:
        g = json.load(f)
    want = np.array([float(Fraction(v)) for v in g["walsh_coeffs_e4_to_e0"]])[::-1]
    got = P.walsh_coefficients(2, 4, 2)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 13, 24, 40, 62])
def test_walsh_matches_oracle_exact(P, orc, k):
    """Against the oracle's exact integer routine (k <= 62), every kind and
    thresholds inside and outside [1, k]."""
    for kind, t in [(0, 0), (1, 0), (1, 1), (2, 1), (2, 2), (2, max(1, k // 3)), (2, max(1, k // 2)),
                    (2, k), (2, 0), (2, k + 1)]:
        want = orc.walsh_coeffs(orc.truth_table(kind, t, k))
        got = P.walsh_coefficients(kind, k, t)
        rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-300)
        assert np.max(rel) <= 1e-15, (kind, k, t)


@pytest.mark.parametrize("k,t", [(64, 16), (100, 37), (127, 1), (130, 130)])
def test_walsh_long_matches_krawtchouk_sum(P, orc, k, t):
    """Past the oracle's integer range: the Krawtchouk sum in big integers."""
    want = _krawtchouk_walsh(orc.truth_table(2, t, k), k)
    got = P.walsh_coefficients(2, k, t)
    assert np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300)) <= 1e-15


def test_unit_circle_worked_example(P):
    """Example 3: the printed conjugated Walsh coefficient, column by column."""
    with open(os.path.join(GOLD, "card4_t2_unit_circle.json")) as f:
        g = json.load(f)
    k = g["k"]
    w = np.exp(-2j * np.pi / (k + 1))
    scale = float(Fraction(g["scale"]))
    want = np.array([scale * sum(cf * w ** e for e, cf in enumerate(row)) for row in g["rows_coeffs_omega0_to_omega4"]])
    got = P.unit_circle_coefficients(g["kind"], k, g["param"])
    assert np.max(np.abs(got - want)) < 1e-15


@pytest.mark.parametrize("k", [1, 4, 9, 32, 100, 257, 512])
def test_unit_circle_inverts_to_walsh(P, k):
    """f~ W = f^ (the ESP order e_k .. e_0): the forward DFT of the table
    gives back the Walsh coefficients; conjugate symmetry f~[N-a] = conj f~[a]."""
    N = k + 1
    for kind, t in [(0, 0), (1, 1), (1, 0), (2, max(1, k // 4)), (2, k)]:
        ft = P.unit_circle_coefficients(kind, k, t)
        fh = P.walsh_coefficients(kind, k, t)
        j = np.arange(N)
        w = np.exp(-2j * np.pi / N)
        back = np.array([np.sum(ft * w ** ((jj * np.arange(N)) % N)) for jj in j])
        assert np.max(np.abs(back.imag)) < 1e-12
        assert np.max(np.abs(back.real - fh[::-1])) < 1e-12 * max(1.0, np.abs(fh).max()), (kind, k, t)
        assert np.max(np.abs(ft[1:] - np.conj(ft[1:][::-1]))) < 1e-15


@pytest.mark.parametrize("k,t", [(4, 2), (7, 3), (16, 5), (33, 11)])
def test_unit_circle_value_and_gradient(P, orc, k, t):
    """WE = sum_a f~[a] prod_i (omega^a + l_i) and its leave-one-out gradient
    equal the count-lattice values (the oracle's authority) at interior points."""
    ft = P.unit_circle_coefficients(2, k, t)
    N = k + 1
    w = np.exp(-2j * np.pi * np.arange(N) / N)
    fv = orc.truth_table(2, t, k)
    rng = np.random.default_rng(k)
    for _ in range(5):
        l = rng.uniform(-1, 1, k)
        fac = w[:, None] + l[None, :]
        we = np.sum(ft * np.prod(fac, axis=1)).real
        g = np.array([np.sum(ft * np.prod(np.delete(fac, i, axis=1), axis=1)).real for i in range(k)])
        we_ref, g_ref = orc.we_dp(l, fv)
        assert abs(we - we_ref) < 1e-12 and np.max(np.abs(g - g_ref)) < 1e-12


def test_bad_arguments(P):
    from paper_2308_15020_amd import _lib
    L = P.lib()
    buf = np.zeros(2 * 600)
    import ctypes as C
    p = C.c_void_p(buf.ctypes.data)
    assert _lib.STATUS[L.ffsat_walsh_coefficients(2, 0, 1, p)] == "E_INVALID_ARG"
    assert _lib.STATUS[L.ffsat_walsh_coefficients(2, 513, 1, p)] == "E_INVALID_ARG"
    assert _lib.STATUS[L.ffsat_unit_circle_coefficients(3, 4, 1, p)] == "E_BAD_KIND"
    assert _lib.STATUS[L.ffsat_unit_circle_coefficients(2, 4, 1, None)] == "E_INVALID_ARG"
