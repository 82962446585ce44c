"""The FP64 reference of the message-passing initialiser, pinned to central
finite differences of its own loss (CPU)."""
import numpy as np

import workloads
from oracle import mpnn_ref as M


def test_reference_gradients_match_finite_differences():
    inst = workloads.random_hybrid(30, 4, n_or=40, or_len=(2, 5), n_xor=8, xor_len=(2, 6),
                                   n_card=6, card_len=(3, 10))
    g = M.Graph(inst)
    H, R = 8, 2
    p = M.init_params(H, R, seed=1)
    for name in p:                       # non-zero biases so every term is exercised
        if name.startswith(("b", "e")):
            p[name] = np.random.default_rng(len(name)).normal(0, 0.1, p[name].shape)
    target = np.random.default_rng(2).uniform(-1, 1, inst.n_vars)
    L0, gr = M.backward(g, p, target, R=R)
    rng = np.random.default_rng(3)
    worst = 0.0
    for name, shp in M.param_shapes(H, R):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in shp)
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            h = 1e-6
            pp[name][idx] += h
            pm[name][idx] -= h
            fd = (M.loss(M.forward(g, pp, R), target) - M.loss(M.forward(g, pm, R), target)) / (2 * h)
            worst = max(worst, abs(fd - gr[name][idx]))
    assert worst < 1e-8, worst


def test_features_and_shapes():
    inst = workloads.assemble(3, [(0, [0], [np.array([1, -2], np.int32)]),
                                  (1, [1], [np.array([2, 3], np.int32)]),
                                  (2, [2], [np.array([-1, -3, 2], np.int32)])])
    fv, fc = M.features(inst)
    # variable 1: +1 in c0, -1 in c2 -> P=1, N=1
    assert np.allclose(fv[0], [1, 1 / 8, 1 / 8, 0, 0, 0, 0, 0])
    assert np.allclose(fc[2], [1, 0, 0, 1, 3 / 64, 2 / 3, 0, 0])
    assert np.allclose(fc[1], [1, 0, 1, 0, 2 / 64, 0, 1, 0])
    flat = M.flatten(M.init_params(16, 3), 16, 3)
    assert flat.size == sum(int(np.prod(s)) for _, s in M.param_shapes(16, 3))


def test_bf16_rounding():
    a = np.array([1.0, 1.00390625, 1.005859375, -3.14159], np.float32)
    r = M.bf16_round(a)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0078125
    assert abs(r[3] - (-3.140625)) < 1e-12
