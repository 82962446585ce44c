"""Exact rational oracle for tiny inputs (test infrastructure only).

Straight from the definitions, with Python Fractions and loops over the
whole cube, so that the FP64 routes in ``oracle.c`` are pinned to something
that shares none of their arithmetic:

* ``walsh_coeff_subset``: Thm. 1, fhat(S) = 2^-k sum_x f(x) prod_{i in S} x_i;
* ``we_lagrange``: the multilinear polynomial that agrees with f on the cube,
  in the Lagrange basis, sum_a f(a) prod_i (1 + a_i l_i)/2;
* ``we_from_coeffs``: Thm. 1's expansion sum_S fhat(S) prod_{i in S} l_i;
* ``esp_convolution``: Eq. convolution, the ESPs as the linear convolution of
  the k sequences [l_i, 1] (coefficients highest degree first).
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations, product


def truth(kind: int, param: int, ntrue: int) -> int:
    """-1 if satisfied with `ntrue` true literals, +1 otherwise."""
    if kind == 0:
        return -1 if ntrue >= 1 else 1
    if kind == 1:
        return -1 if ntrue % 2 == (param & 1) else 1
    if kind == 2:
        return -1 if ntrue >= param else 1
    raise ValueError(kind)


def f_on_point(kind, param, a):
    """a: tuple of +-1 literal values (-1 = True)."""
    return truth(kind, param, sum(1 for v in a if v == -1))


def walsh_coeff_subset(kind, param, k, S):
    tot = Fraction(0)
    for a in product((-1, 1), repeat=k):
        p = 1
        for i in S:
            p *= a[i]
        tot += f_on_point(kind, param, a) * p
    return tot / (2 ** k)


def walsh_coeffs_by_size(kind, param, k):
    """fhat_j for j = 0..k using the subset {0..j-1} (symmetric constraints)."""
    return [walsh_coeff_subset(kind, param, k, tuple(range(j))) for j in range(k + 1)]


def we_lagrange(kind, param, l):
    l = [Fraction(v) for v in l]
    k = len(l)
    tot = Fraction(0)
    for a in product((-1, 1), repeat=k):
        w = Fraction(1)
        for ai, li in zip(a, l):
            w *= (1 + ai * li) / 2
        tot += f_on_point(kind, param, a) * w
    return tot


def grad_lagrange(kind, param, l):
    """dWE/dl_i exactly: WE is affine in l_i, so the derivative is half the
    difference of the values at l_i = +1 and l_i = -1."""
    out = []
    for i in range(len(l)):
        hi = list(l)
        lo = list(l)
        hi[i] = 1
        lo[i] = -1
        out.append((we_lagrange(kind, param, hi) - we_lagrange(kind, param, lo)) / 2)
    return out


def we_from_coeffs(kind, param, l):
    l = [Fraction(v) for v in l]
    k = len(l)
    tot = Fraction(0)
    for j in range(k + 1):
        for S in combinations(range(k), j):
            p = Fraction(1)
            for i in S:
                p *= l[i]
            tot += walsh_coeff_subset(kind, param, k, S) * p
    return tot


def esp_convolution(l):
    """[e_k, ..., e_0] by convolving [l_i, 1] sequences."""
    seq = [Fraction(1)]
    for v in l:
        v = Fraction(v)
        nxt = [Fraction(0)] * (len(seq) + 1)
        for idx, s in enumerate(seq):
            nxt[idx] += v * s      # [l_i, 1] * seq: first element multiplies
            nxt[idx + 1] += s
        seq = nxt
    return seq
