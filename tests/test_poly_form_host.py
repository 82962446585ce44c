"""The FP64 polynomial form of the root-of-unity products, on the host (no
GPU): a float64 NumPy mirror of the kernel's loops (segment polynomials,
the Horner evaluation in -tau^2, the moments, the value term without c0,
the blocked gradient pass) against direct complex products.

This pins the algebra the FP64 kernels rely on, independently of them:
* P = init (A - i tau B) with A, B the even / odd parts at sigma = -tau^2
  equals init * prod_t (1 - i tau l_t);
* with W = c1 init T / P and c0 = i c1 / tau, Re(c0 T) = B Re(W) + A tau Im(W) / sigma;
* sum_m e^(-t)_m H_m over the moments H_m = sum_f Re(W_f z_f^m) equals the sum
  over frequencies of Re(W_f * the leave-one-out product of position t);
* the blocked gradient pass (suffix adjoints, per-block prefix polynomials)
  equals that sum for every segment length 1..32;
* the rounding stays within SEG eps 2^(SEG/2) of the largest term, also for
  tangents far above 1 (the form-2 frequencies run through form 1's code).
"""
import numpy as np
import pytest


def esp(v):
    s = len(v)
    e = [1.0] + [0.0] * s
    for t in range(s):
        for m in range(t + 1, 0, -1):
            e[m] = v[t] * e[m - 1] + e[m]
    return e


def horner_parts(e, sg):
    s = len(e) - 1
    ne, no = s // 2, (s - 1) // 2
    a = e[2 * ne]
    for n in range(ne - 1, -1, -1):
        a = a * sg + e[2 * n]
    b = e[2 * no + 1] if s >= 1 else 0.0
    for n in range(no - 1, -1, -1):
        b = b * sg + e[2 * n + 1]
    return a, b


def moments_update(H, cr, ci, sg):
    s = len(H)
    pw = 1.0
    for n in range(s):
        if 2 * n >= s:
            break
        H[2 * n] += pw * cr
        if 2 * n + 1 < s:
            H[2 * n + 1] += pw * ci
        if 2 * n + 2 < s:
            pw *= sg


def grad_pass(v, H, gb=8):
    """The kernel's gradient pass: blocks of gb positions, last first."""
    s = len(v)
    R = list(H)
    out = [None] * s
    nblk = (s + gb - 1) // gb
    for bi in range(nblk - 1, -1, -1):
        lo = bi * gb
        nb = min(gb, s - lo)
        hi = lo + nb
        P = esp(v[:lo])
        G = [sum(P[i] * R[a + i] for i in range(lo + 1)) for a in range(nb)]
        for tl in range(nb - 1, -1, -1):
            Q = esp(v[lo:lo + tl])
            out[lo + tl] = sum(Q[i] * G[i] for i in range(tl + 1))
            for i in range(tl):
                G[i] = G[i] + v[lo + tl] * G[i + 1]
        if bi > 0:
            for u in range(nb):
                ln = hi - u
                for q in range(ln - 1):
                    R[q] = R[q] + v[lo + u] * R[q + 1]
    return out


def leave_one_out(v, t, z):
    return np.prod([1.0 + z * x for u, x in enumerate(v) if u != t])


@pytest.mark.parametrize("s", [1, 2, 5, 8, 13, 16, 24, 31, 32])
def test_segment_product_and_value_term(s):
    rng = np.random.default_rng(100 + s)
    v = list(rng.uniform(-1, 1, s))
    e = esp(v)
    for tau in (0.01, 0.4, 1.0, 3.0, 300.0):
        init = 2.0 ** -3 * (tau ** -s if tau > 1 else 1.0)
        sg = -tau * tau
        a, b = horner_parts(e, sg)
        P = complex(init * a, -init * tau * b)
        direct = init * np.prod([1 - 1j * tau * x for x in v])
        assert abs(P - direct) <= 1e-12 * abs(direct)
        # value term: Re(c0 T) with c0 = i c1 / tau, T = P * (other lanes' product)
        c1 = complex(*rng.normal(size=2))
        other = complex(*rng.normal(size=2))
        T = P * other
        W = c1 * init * T / P
        cr, ci = W.real, tau * W.imag
        got = cr * b + ci * (1.0 / sg) * a
        want = (1j * c1 / tau * T).real
        assert abs(got - want) <= 1e-12 * (abs(c1 / tau * T) + 1e-300)


@pytest.mark.parametrize("s", list(range(1, 33)))
def test_moments_and_gradient_pass(s):
    rng = np.random.default_rng(7 * s)
    v = list(rng.uniform(-1, 1, s))
    if s > 3:
        v[-1] = 1.0        # a padding position
    H = [0.0] * s
    direct = np.zeros(s)
    for f in range(6):
        tau = rng.uniform(0.01, 1.0) if f < 4 else rng.uniform(1.0, 300.0)
        init = rng.uniform(0.5, 2.0) * (tau ** -s if tau > 1 else 1.0)
        W = complex(*rng.normal(size=2)) * init     # c1 init (T / P)
        sg = -tau * tau
        moments_update(H, W.real, tau * W.imag, sg)
        z = -1j * tau
        for t in range(s):
            direct[t] += (W * leave_one_out(v, t, z)).real
    # sum_m e^(-t)_m H_m, straight from the definition
    ref = [sum(esp(v[:t] + v[t + 1:])[m] * H[m] for m in range(s)) for t in range(s)]
    got = grad_pass(v, H)
    scale = np.abs(direct).max() + 1e-300
    assert np.max(np.abs(np.array(ref) - direct)) <= 1e-9 * scale * 2 ** (s / 2)
    assert np.max(np.abs(np.array(got) - np.array(ref))) <= 1e-12 * scale * 2 ** (s / 2)


def test_rounding_bound_at_the_corners():
    """All literals at +-1 and tau = 1: the sum of the terms' magnitudes is
    2^(s/2) times the product's modulus, the worst case of the bound."""
    for s in (16, 24, 32):
        v = [1.0 if t % 2 else -1.0 for t in range(s)]
        e = esp(v)
        a, b = horner_parts(e, -1.0)
        P = complex(a, -b)
        direct = np.prod([1 - 1j * x for x in v])
        assert abs(P - direct) <= s * 2.2e-16 * 2 ** (s / 2) * abs(direct)
