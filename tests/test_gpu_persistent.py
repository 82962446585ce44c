"""The persistent fused-iteration loop for small problems of short
transform-free constraints (one workgroup runs all T iterations: gradient,
exact check, projected step, adaptive weights) against the oracle and
against the usual launch sequence (needs an MI355X).

* random 3-SAT n = 50, m = 213, one restart, 200 iterations: at every
  iteration the oracle evaluates the GPU's own iterate (F, the next point,
  n_sat and U bit-exact);
* random 3-SAT n = 100 with 4 restarts: T iterations with adaptive weights
  against the same iterations of a plan without the persistent loop;
* a problem with long constraints: the option falls back to the usual steps.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_cases import TOL32, every_bin_instance, var_scale

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


def test_persistent_3sat_trajectory(ffs):
    inst = workloads.config1(workloads.instance_seed(1, 0))
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, 1, persistent=True)
    assert plan.describe()["persistent_steps"]
    x = torch.from_numpy(workloads.points(50, 1, workloads.point_seed(1000))).to(DEV)
    eta = 0.05
    S = var_scale(inst)[:, None]
    wsum = float(inst.m)
    out = None
    for step in range(200):
        xt = x.cpu().numpy().astype(np.float64)
        out = plan.run_iters(x, 1, eta, 0.0, out=out)
        torch.cuda.synchronize()
        ref = oracle.eval_batch(inst, xt)
        assert abs(float(out["F"][0]) - ref["F"][0]) / wsum <= TOL32, step
        want = np.clip(xt - eta * ref["g"], -1.0, 1.0)
        assert np.max(np.abs(x.cpu().numpy() - want) / (eta * S)) <= TOL32 + 1e-6, step
        rc = oracle.check(inst, xt)
        assert int(out["n_sat"][0]) == int(rc["n_sat"][0]), step
        assert np.array_equal(out["U"].cpu().numpy(), rc["U"]), step


@pytest.mark.parametrize("T", [1, 7])
def test_persistent_matches_usual_iterations(ffs, T):
    inst = workloads.random_hybrid(100, 5, n_or=426, or_len=(3, 3))
    B, eta, alpha = 4, 0.05, 0.4
    x0 = torch.from_numpy(workloads.points(inst.n_vars, B, 6)).to(DEV)
    res = {}
    for persistent in (False, True):
        prob = ffs.Problem(inst, device=0)
        plan = ffs.Plan(prob, B, persistent=persistent, pull="off")
        assert plan.describe()["persistent_steps"] == persistent
        x = x0.clone()
        out = plan.run_iters(x, T, eta, alpha)
        torch.cuda.synchronize()
        res[persistent] = (x.cpu().numpy(), {k: v.cpu().numpy() for k, v in out.items()},
                           prob.get_weights().cpu().numpy())
    (xa, oa, wa), (xb, ob, wb) = res[False], res[True]
    assert np.max(np.abs(xa - xb)) <= 1e-5
    assert np.max(np.abs(wa - wb)) <= 1e-6
    assert np.max(np.abs(oa["F"] - ob["F"])) / inst.m <= 1e-6
    assert np.array_equal(oa["n_sat"], ob["n_sat"]) and np.array_equal(oa["U"], ob["U"])


def test_persistent_option_falls_back(ffs):
    inst = every_bin_instance()
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, 8, persistent=True)
    assert not plan.describe()["persistent_steps"]
    x = torch.from_numpy(workloads.points(inst.n_vars, 8, 3)).to(DEV)
    ref = x.clone()
    plan.run_steps(x, 2, 0.05)
    ffs.Plan(prob, 8).run_steps(ref, 2, 0.05)
    torch.cuda.synchronize()
    assert torch.equal(x, ref)
