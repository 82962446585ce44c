"""Autograd wrapper, restart kernels and the solve loop on the GPU.

* the weighted objective on the mixed n = 2000 instance with w ~ U[0.5, 1.5],
  x [2000][1024]: gradients with respect to x and w against the oracle's
  analytic gradients and FP64 central differences (h = 1e-6);
* rephasing (original / flipped / random with SplitMix64) bit-exact;
* Alg. 1 on planted satisfiable instances: the returned assignment passes
  the oracle's exact checker.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_cases import TOL32, var_scale

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


def test_autograd_weighted_objective(ffs):
    from paper_2308_15020_amd.autograd import objective
    inst = workloads.config4(workloads.instance_seed(4, 0))
    B = 1024
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, B)
    xn = workloads.points(inst.n_vars, B, workloads.point_seed(4000))
    x = torch.from_numpy(xn).to(DEV).requires_grad_(True)
    w = torch.from_numpy(inst.weights.copy()).to(DEV).requires_grad_(True)
    gF = torch.from_numpy(np.random.default_rng(3).normal(size=B).astype(np.float32)).to(DEV)
    F = objective(x, w, plan)
    (F * gF).sum().backward()
    gx = x.grad.cpu().numpy()
    gw = w.grad.cpu().numpy()
    gFn = gF.cpu().numpy().astype(np.float64)
    # analytic, on a restart subset (oracle cost)
    cols = np.array([0, 5, 511, 1023])
    sub = np.ascontiguousarray(xn[:, cols].astype(np.float64))
    ref = oracle.eval_batch(inst, sub, w=inst.weights.astype(np.float64), want_con=True)
    S = var_scale(inst)[:, None]
    err_x = np.max(np.abs(gx[:, cols] - ref["g"] * gFn[cols]) / (S * np.abs(gFn[cols])))
    assert err_x <= TOL32, err_x
    # gw needs all restarts: sum_b gF_b WE_c(x_b), natural scale sum_b |gF_b|
    full = oracle.eval_batch(inst, xn.astype(np.float64), w=inst.weights.astype(np.float64),
                             want_g=False, want_con=True)
    gw_ref = oracle.wgrad(full["con_val"], gFn)
    err_w = np.max(np.abs(gw - gw_ref)) / np.abs(gFn).sum()
    assert err_w <= TOL32, err_w
    # FP64 central differences: 64 variables x 16 restarts, 64 weights
    rng = np.random.default_rng(9)
    sv = rng.integers(0, inst.n_vars, 64)
    sb = rng.integers(0, B, 16)
    vv, bb = np.meshgrid(sv, sb, indexing="ij")
    fd = oracle.fd_grad(inst, xn.astype(np.float64), vv.ravel(), bb.ravel(),
                        w=inst.weights.astype(np.float64), h=1e-6)
    got = gx[vv.ravel(), bb.ravel()] / gFn[bb.ravel()]
    scale = var_scale(inst)[vv.ravel()]
    assert np.max(np.abs(got - fd) / scale) <= 1e-5
    # the GPU's own weight gradient over the first 64 restarts (gF zeroed
    # beyond them) against FP64 central differences of the oracle's F in w
    gF64 = gF.clone()
    gF64[64:] = 0.0
    x2 = torch.from_numpy(xn).to(DEV).requires_grad_(True)
    w2 = torch.from_numpy(inst.weights.copy()).to(DEV).requires_grad_(True)
    (objective(x2, w2, plan) * gF64).sum().backward()
    gw64_gpu = w2.grad.cpu().numpy()
    nat = np.abs(gFn[:64]).sum()
    cs = rng.integers(0, inst.m, 64)
    for c in cs:
        e = np.zeros(inst.m)
        e[c] = 1e-6
        Fp = oracle.eval_batch(inst, xn.astype(np.float64)[:, :64], w=inst.weights + e, want_g=False)["F"]
        Fm = oracle.eval_batch(inst, xn.astype(np.float64)[:, :64], w=inst.weights - e, want_g=False)["F"]
        fdw = gFn[:64] @ (Fp - Fm) / 2e-6
        assert abs(fdw - float(gw64_gpu[c])) <= TOL32 * nat, (c, fdw, gw64_gpu[c])


def _splitmix64(z):
    m = (1 << 64) - 1
    z &= m
    z = ((z ^ (z >> 30)) * 0xbf58476d1ce4e5b9) & m
    z = ((z ^ (z >> 27)) * 0x94d049bb133111eb) & m
    return z ^ (z >> 31)


def test_rephase_modes(ffs):
    inst = workloads.random_hybrid(37, 2, n_or=20, or_len=(2, 4))
    B = 67
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, B)
    x0 = workloads.points(37, B, 5)
    x = torch.from_numpy(x0).to(DEV)
    plan.rephase(x, 0)
    assert np.array_equal(x.cpu().numpy(), x0)
    plan.rephase(x, 1)
    assert np.array_equal(x.cpu().numpy(), -x0)
    mask = torch.zeros(B, dtype=torch.int32, device=DEV)
    mask[::3] = 1
    seed = 123456789
    plan.rephase(x, 2, seed=seed, mask=mask)
    got = x.cpu().numpy()
    idx = np.arange(37 * B).reshape(37, B)
    want = -x0.copy()
    for v in range(37):
        for b in range(0, B, 3):
            r = _splitmix64(seed + (int(idx[v, b]) + 1) * 0x9e3779b97f4a7c15)
            want[v, b] = np.float32((r >> 40) * (2.0 / 16777216.0) - 1.0)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("policy,weighting", [("ROF", True), ("O", True), ("R", False)])
def test_solver_planted(ffs, policy, weighting):
    from paper_2308_15020_amd.solver import solve
    inst, hidden = workloads.planted_hybrid(300, 11, n_or=1000, or_len=(3, 4), n_xor=10, xor_len=(2, 3),
                                            n_card=10, card_len=(5, 20))
    prob = ffs.Problem(inst, device=0)
    res = solve(prob, B=256, rounds=60, T=40, eta=0.1, policy=policy, weighting=weighting, seed=7)
    print(policy, weighting, res.solved, res.rounds, res.best_sat, inst.m, f"{res.seconds:.3f}s")
    if policy == "ROF":
        assert res.solved
    if res.solved:
        x = np.where(res.assignment, -1.0, 1.0)[:, None]
        assert int(oracle.check(inst, x)["n_sat"][0]) == inst.m


def test_time_to_solve_harness_runs(ffs):
    """The learned-vs-uniform harness end to end on a tiny planted budget."""
    from paper_2308_15020_amd import tts
    s = tts.main(["--train", "2", "--test", "2", "--B", "64", "--rounds", "4", "--T", "20", "--epochs", "3",
                  "--planted"])
    assert s["instances"] == 2
    assert 0.0 <= s["solve_rate"]["uniform"] <= 1.0 and 0.0 <= s["solve_rate"]["learned"] <= 1.0
    assert np.isfinite(s["train_loss"]).all()
    c = s["cactus_at_lower_solve_rate"]
    assert 0 <= c["instances"] <= 2 and (c["instances"] == 0 or c["learned_s"] > 0)


def test_learned_initialisation_needs_fewer_rounds(ffs):
    """What the trained network gains over the method without it, counted in
    rounds (deterministic: fixed seeds, deterministic kernels).  Leak-free
    family shaped like the mixed n = 2000 workload (OR clauses satisfied by
    the hidden assignment and its complement, XOR parities from it,
    at-least-t signs independent of it) with 400 XOR constraints; a short
    training run on 16 instances; 6 test instances (seeds disjoint from the
    training seeds).  An unsolved run counts as rounds + 1.  The learned arm
    must solve at least as many instances as uniform restarts and need fewer
    median rounds."""
    import argparse

    from paper_2308_15020_amd import tts
    from paper_2308_15020_amd.mpnn import Mpnn, fit, targets_from_solves
    train = [ffs.Problem(tts.instance(10000 + i, "hidden2", 400), device=0) for i in range(16)]
    targets = [targets_from_solves(p, B=1024, seed=10000 + i) for i, p in enumerate(train)]
    net = Mpnn(64, 3, device=0, seed=1)
    hist = fit(net, train, targets, epochs=20, lr=2e-3)
    assert hist[-1] < hist[0]
    args = argparse.Namespace(B=256, rounds=20, T=40, eta=0.3, policy="ROF", frac=0.75, sigma=0.3,
                              reuse_proposal=True)
    rounds = {"uniform": [], "learned": []}
    solved = {"uniform": 0, "learned": 0}
    for i in range(6):
        seed = 20000 + i
        prob = ffs.Problem(tts.instance(seed, "hidden2", 400), device=0)
        plan = ffs.Plan(prob, args.B)
        x_buf = torch.empty(prob.n, args.B, dtype=torch.float32, device=DEV)
        for arm, net_arm in (("uniform", None), ("learned", net)):
            r = tts.run_arm(prob, plan, net_arm, args, seed, x_buf)
            solved[arm] += int(r["solved"])
            rounds[arm].append(r["rounds"] if r["solved"] else args.rounds + 1)
        plan.close()
        prob.close()
    print(solved, rounds)
    assert solved["learned"] >= solved["uniform"]
    assert np.median(rounds["learned"]) < np.median(rounds["uniform"])


def test_portfolio_arms_keep_their_own_weights(ffs):
    """Two strategies side by side: the run stops when either arm satisfies
    everything (checked by the oracle), the weighting arm's problem has adapted
    weights and the fixed arm's problem keeps unit weights."""
    from paper_2308_15020_amd.solver import Arm, solve_portfolio
    inst, _ = workloads.planted_hybrid(300, 12, n_or=1150, or_len=(3, 3))
    probs = [ffs.Problem(inst, device=0), ffs.Problem(inst, device=0)]
    arms = [Arm(128, weighting=False, policy="R", eta=0.1), Arm(128, weighting=True, policy="ROF", eta=0.1)]
    res = solve_portfolio(inst, arms, rounds=60, T=40, seed=3, problems=probs)
    print(res.solved, res.rounds, res.restart, res.best_sat, inst.m)
    assert res.solved and 0 <= res.restart < 256
    x = np.where(res.assignment, -1.0, 1.0)[:, None]
    assert int(oracle.check(inst, x)["n_sat"][0]) == inst.m
    w0, w1 = probs[0].get_weights().cpu().numpy(), probs[1].get_weights().cpu().numpy()
    assert np.all(w0 == 1.0)
    if res.rounds > 1:
        assert not np.all(w1 == 1.0)


def test_table2_harness_runs(ffs):
    """The restart-heuristics table end to end on a tiny budget."""
    from paper_2308_15020_amd import heuristics
    import argparse
    t = heuristics.run(argparse.Namespace(n=[20], instances=2, B=64, rounds=3, T=20, eta=0.1))
    s = t[20]
    assert s["instances"] == 2
    for arm in ("plain", "heuristic", "portfolio", "two_device"):
        assert 0 <= s[arm]["solved"] <= 2 and 1 <= s[arm]["par2_iters"] <= 6
    assert s["two_device"]["solved"] >= max(s["plain"]["solved"], s["heuristic"]["solved"])
