"""Captured graphs: one graph per buffer set serves every step size and
weight-update rate (they are read from device memory), FISTA's fixed trial
sequence replays from a graph with the eager results, and the solver keeps
a single graph across its rounds."""
import numpy as np
import pytest

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


def _inst():
    return workloads.random_hybrid(150, 21, n_or=500, or_len=(2, 6), n_xor=40, xor_len=(2, 12),
                                   n_card=12, card_len=(8, 60))


def test_run_steps_one_graph_for_every_step_size(ffs):
    inst = _inst()
    B = 96
    prob = ffs.Problem(inst, device=0)
    pg = ffs.Plan(prob, B, use_graphs=True)
    pe = ffs.Plan(prob, B, use_graphs=False)
    x0 = torch.from_numpy(workloads.points(inst.n_vars, B, 5)).to(DEV)
    xg, xe = x0.clone(), x0.clone()
    for eta in (0.05, 0.2, 0.013, 0.05):
        pg.run_steps(xg, 7, eta)
        torch.cuda.synchronize()
        pe.run_steps(xe, 7, eta)          # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(xg, xe), eta
    d = pg.describe()
    assert d["graph_captures"] == 1 and d["graphs_cached"] == 1


def test_run_iters_one_graph_for_every_rate(ffs):
    inst = _inst()
    B = 64
    pg_prob, pe_prob = ffs.Problem(inst, device=0), ffs.Problem(inst, device=0)
    pg = ffs.Plan(pg_prob, B, use_graphs=True)
    pe = ffs.Plan(pe_prob, B, use_graphs=False)
    x0 = torch.from_numpy(workloads.points(inst.n_vars, B, 6)).to(DEV)
    xg, xe = x0.clone(), x0.clone()
    og, oe = {}, {}
    for eta, alpha in ((0.1, 0.4), (0.03, 0.2), (0.1, 0.7)):
        og = pg.run_iters(xg, 5, eta, alpha, out=og)
        torch.cuda.synchronize()
        oe = pe.run_iters(xe, 5, eta, alpha, out=oe)
        torch.cuda.synchronize()
        assert torch.equal(xg, xe)
        assert torch.equal(pg_prob.get_weights(), pe_prob.get_weights())
        for k in ("F", "n_sat", "U"):
            assert torch.equal(og[k], oe[k]), k
    # alpha = 0 has no weight update: a second graph
    pg.run_iters(xg, 5, 0.1, 0.0, out=og)
    assert pg.describe()["graph_captures"] == 2


def test_fista_graph_matches_eager_and_is_reused(ffs):
    inst = _inst()
    B = 80
    prob = ffs.Problem(inst, device=0)
    pg = ffs.Plan(prob, B, use_graphs=True)
    pe = ffs.Plan(prob, B, use_graphs=False)
    x0 = torch.from_numpy(workloads.points(inst.n_vars, B, 7)).to(DEV)
    xg, xe = x0.clone(), x0.clone()
    sg, se = pg.fista_state(xg, 2.0), pe.fista_state(xe, 2.0)   # a large step: several trials per iteration
    sg["eta"][::7] = 1e-13
    se["eta"][::7] = 1e-13
    Fg = torch.zeros(B, device=DEV)
    Fe = torch.zeros(B, device=DEV)
    for rep in range(3):
        pg.fista(xg, sg, 4, max_ls=6, F=Fg)
        torch.cuda.synchronize()
        pe.fista(xe, se, 4, max_ls=6, F=Fe)
        torch.cuda.synchronize()
        assert torch.equal(xg, xe) and torch.equal(sg["y"], se["y"]), rep
        assert torch.equal(sg["eta"], se["eta"]) and torch.equal(sg["t"], se["t"]) and torch.equal(Fg, Fe), rep
        if rep == 1:
            pg.fista_reset(sg, xg, 1.0)
            pe.fista_reset(se, xe, 1.0)
    assert pg.describe()["graph_captures"] == 1
    # the halving happened somewhere (the trials were exercised)
    assert float(se["eta"].min()) < 1.0


def test_solver_keeps_one_graph_across_rounds(ffs):
    """Adaptive weights with the step normalised by their mean change the
    step size every round; the captured step graph stays the same."""
    from paper_2308_15020_amd.solver import solve
    inst = workloads.config2(2000)
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, 64)
    res = solve(prob, B=64, rounds=5, T=5, eta=0.05, plan=plan, seed=1)
    assert not res.solved and res.rounds == 5
    w = prob.get_weights().cpu().numpy()
    assert not np.allclose(w, w.mean())          # the weights (and the step) moved
    d = plan.describe()
    assert d["graph_captures"] == 1, d
