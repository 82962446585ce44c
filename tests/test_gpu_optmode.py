"""Optimisation-mode workloads on the GPU: weighted Max-Cut as weighted
2-XOR on planted-partition graphs and learning parity with noise, scored by
satisfied weight (ffsat_sat_weight) and checked against the optimum found by
brute force over all 2^n assignments (the definition of the optimum)."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ffs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_15020_amd as P
    P.lib()
    return P


def _all_assignments(n):
    a = np.arange(1 << n, dtype=np.int64)
    return ((a[:, None] >> np.arange(n)) & 1).astype(bool)        # [2^n][n], True = True


def _xor_sat_matrix(inst, A):
    """[2^n][m] bool: XOR constraint c holds under assignment row."""
    cp = inst.con_ptr
    out = np.empty((A.shape[0], inst.m), dtype=bool)
    for c in range(inst.m):
        lits = inst.lits[cp[c]:cp[c + 1]]
        v = np.abs(lits) - 1
        t = A[:, v] ^ (lits < 0)[None, :]
        out[:, c] = (t.sum(axis=1) % 2) == (inst.params[c] & 1)
    return out


def test_sat_weight_matches_bits(ffs):
    inst = workloads.random_hybrid(90, 4, n_or=200, or_len=(2, 5), n_xor=30, xor_len=(2, 7),
                                   n_card=10, card_len=(5, 20))
    B = 77
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, B)
    x = torch.from_numpy(workloads.points(inst.n_vars, B, 3)).to(DEV)
    chk = plan.round_check(x, want=("unsat_bits",))
    w = np.random.default_rng(1).uniform(0.1, 3.0, inst.m).astype(np.float32)
    got = plan.sat_weight(chk["unsat_bits"], torch.from_numpy(w).to(DEV)).cpu().numpy()
    got1 = plan.sat_weight(chk["unsat_bits"]).cpu().numpy()
    ref = oracle.check(inst, x.cpu().numpy().astype(np.float64))
    ub = ref["unsat_bits"]                                   # the oracle's own bits
    c = np.arange(inst.m)
    sat = ((ub[:, c >> 5] >> (c & 31).astype(np.uint32)) & 1) == 0     # [B][m]
    want = (sat * w.astype(np.float64)[None, :]).sum(axis=1)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-9)
    assert np.array_equal(got1, np.asarray(ref["n_sat"], np.float64))


def test_maxcut_reaches_brute_force_optimum(ffs):
    from paper_2308_15020_amd.solver import solve
    inst = workloads.maxcut_planted(16, 7, p_in=0.3, p_out=0.6)
    A = _all_assignments(16)
    S = _xor_sat_matrix(inst, A)
    opt = float((S * inst.weights.astype(np.float64)).sum(axis=1).max())
    prob = ffs.Problem(inst, device=0)
    res = solve(prob, B=256, rounds=20, T=30, eta=0.2, seed=2, maximize=inst.weights)
    assert res.best_weight == pytest.approx(opt)
    row = A[np.nonzero((A == res.assignment[None, :]).all(axis=1))[0][0]]
    assert float((_xor_sat_matrix(inst, row[None, :]) * inst.weights).sum()) == pytest.approx(opt)


def test_parity_learning_reaches_brute_force_optimum(ffs):
    from paper_2308_15020_amd.solver import solve
    inst = workloads.parity_learning(14, 5)
    A = _all_assignments(14)
    S = _xor_sat_matrix(inst, A)
    opt = int(S.sum(axis=1).max())
    prob = ffs.Problem(inst, device=0)
    res = solve(prob, B=512, rounds=40, T=30, eta=0.2, seed=4, maximize=np.ones(inst.m, np.float32))
    assert res.best_weight == pytest.approx(opt)
    assert res.best_sat <= opt
