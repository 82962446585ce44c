"""Pins of the FP64 FISTA reference (oracle/fista.py) against cases worked
by hand: a linear objective (unit-length XOR constraints, so the gradient is
constant and every step is accepted), the bilinear objective of one
length-2 XOR constraint (the backtracking halves the step a known number of
times), stopped restarts and a fixed point."""
import math

import numpy as np
import pytest

import workloads
from oracle import fista


def _unit_xor(weights, parities):
    n = len(weights)
    rows = [np.array([v + 1], np.int32) for v in range(n)]
    inst = workloads.assemble(n, [(1, np.asarray(parities, np.int32), rows)])
    inst.weights = np.asarray(weights, np.float32)
    return inst


def test_linear_objective_trajectory_by_hand():
    # F(x) = sum_v w_v (2 p_v - 1) x_v: constant gradient c_v; the
    # sufficient-decrease test holds for every step size, so eta never moves
    w = np.array([1.0, 0.5, 2.0, 1.5])
    p = np.array([1, 0, 1, 0])
    c = w * (2 * p - 1)
    inst = _unit_xor(w, p)
    x0 = np.array([[0.3, -0.2], [0.9, 0.1], [-0.5, 0.0], [0.0, -0.95]])
    eta0 = 0.25
    T = 6
    # by hand: x1 = clip(x0 - eta c); t1 = (1 + sqrt 5)/2; y1 = x1 (t0 = 1);
    # x_{k+1} = clip(y_k - eta c); y_{k+1} = x_{k+1} + ((t_k - 1)/t_{k+1})(x_{k+1} - x_k)
    xs, ys, t = x0.copy(), x0.copy(), 1.0
    for _ in range(T):
        z = np.clip(ys - eta0 * c[:, None], -1, 1)
        tn = (1 + math.sqrt(1 + 4 * t * t)) / 2
        ys = z + ((t - 1) / tn) * (z - xs)
        xs, t = z, tn
    x, y, eta, tt = fista.run(inst, x0, eta0, T, w=w)
    assert np.allclose(x, xs, atol=1e-14) and np.allclose(y, ys, atol=1e-14)
    assert np.all(eta == eta0) and np.allclose(tt, t)


def test_bilinear_backtracking_by_hand():
    # one XOR of length 2 with odd parity: F = x1 x2 (-1 = True).  At
    # y = (1/2, 1/2), g = (1/2, 1/2); the test F(z) <= F(y) + <g, d> + |d|^2/(2 eta)
    # reads (eta/2)^2 - eta/2 <= -eta/4 (unclipped), i.e. eta <= 1; from eta = 4
    # the trials are eta = 4 (clipped to the corner, F = 1 > -11/16),
    # eta = 2 (F = 1/4 > -1/4), eta = 1 (F = 0 <= 0): accepted after 3 trials.
    inst = workloads.assemble(2, [(1, np.array([1], np.int32), [np.array([1, 2], np.int32)])])
    y = np.array([[0.5], [0.5]])
    xn, yn, eta, tn, Fy, Fx, trials, _ = fista.iterate(inst, y, y, np.array([4.0]), np.array([1.0]))
    assert trials[0] == 3 and eta[0] == 1.0
    assert np.allclose(xn[:, 0], [0.0, 0.0]) and np.allclose(yn[:, 0], [0.0, 0.0])
    assert Fy[0] == pytest.approx(0.25) and Fx[0] == pytest.approx(0.0)
    assert tn[0] == pytest.approx((1 + math.sqrt(5)) / 2)
    # from eta = 1 the first trial is accepted
    *_, trials1, _ = fista.iterate(inst, y, y, np.array([1.0]), np.array([1.0]))
    assert trials1[0] == 1
    # max_ls = 2 from eta = 4: both trials rejected, the second point taken, eta halved twice
    xn2, _, eta2, *_ = fista.iterate(inst, y, y, np.array([4.0]), np.array([1.0]), max_ls=2)
    assert eta2[0] == 1.0 and np.allclose(xn2[:, 0], [-0.5, -0.5])


def test_stopped_restarts_and_fixed_point():
    w = np.array([1.0, 1.0])
    inst = _unit_xor(w, [1, 1])           # F = x1 + x2, minimised at the corner (-1, -1)
    x = np.array([[-1.0, 0.2], [-1.0, 0.4]])
    y = x.copy()
    eta = np.array([0.5, 1e-13])          # restart 1 has stopped (eta < 1e-12)
    t = np.array([3.0, 2.0])
    xn, yn, en, tn, *_ = fista.iterate(inst, x, y, eta, t)
    assert np.array_equal(xn[:, 1], x[:, 1]) and np.array_equal(yn[:, 1], y[:, 1])
    assert en[1] == 1e-13 and tn[1] == 2.0
    # restart 0 sits at the minimiser: z = y, so x and y stay put
    assert np.array_equal(xn[:, 0], x[:, 0]) and np.array_equal(yn[:, 0], x[:, 0]) and en[0] == 0.5
