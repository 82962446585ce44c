"""Generators of the optimisation-mode workloads (CPU)."""
import numpy as np

import workloads


def test_maxcut_planted_structure():
    inst = workloads.maxcut_planted(40, 3, p_in=0.2, p_out=0.5)
    part = inst.meta["part"]
    assert np.all(inst.kinds == 1) and np.all(inst.params == 1)       # XOR, odd parity
    assert np.all(np.diff(inst.con_ptr) == 2)
    u, v = np.abs(inst.lits[0::2]) - 1, np.abs(inst.lits[1::2]) - 1
    assert np.all(u < v)
    same = part[u] == part[v]
    assert np.all(inst.weights[same] == 1.0) and np.all(inst.weights[~same] == 2.0)
    # the planted cut (parts on opposite sides) cuts every cross edge
    assert (~same).sum() > same.sum()


def test_parity_learning_labels():
    inst = workloads.parity_learning(64, 9, m=4000, noise=0.25)
    s = inst.meta["secret"]
    agree = []
    for c in range(inst.m):
        v = np.abs(inst.lits[inst.con_ptr[c]:inst.con_ptr[c + 1]]) - 1
        agree.append(int(s[v].sum() % 2) == inst.params[c])
    frac_flipped = 1.0 - np.mean(agree)
    assert abs(frac_flipped - 0.25) < 0.03


def test_hidden2_ksat_is_satisfied_by_both_hidden_assignments():
    import oracle
    inst, sigma = workloads.hidden2_ksat(120, 5)
    assert inst.m == round(4.26 * 120) and np.all(np.diff(inst.con_ptr) == 3)
    for a in (sigma, ~sigma):
        x = np.where(a, -1.0, 1.0)[:, None]
        assert int(oracle.check(inst, x)["n_sat"][0]) == inst.m
    # no polarity bias: positive and negative occurrences balance overall
    pos = int((inst.lits > 0).sum())
    assert abs(pos - inst.nnz / 2) < 4 * np.sqrt(inst.nnz)
    # and the majority polarity of a variable does not reveal sigma
    v = np.abs(inst.lits) - 1
    net = np.bincount(v, weights=np.sign(inst.lits), minlength=inst.n_vars)
    lean_true = net < 0          # more negative occurrences: x < 0 is True
    agree = np.mean(lean_true[net != 0] == sigma[net != 0])
    assert 0.3 < agree < 0.7
