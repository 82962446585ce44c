"""The measured configurations end to end on the GPU, against the oracle.

* random 3-SAT n=50, m=213, one restart, 200 projected steps: the oracle
  evaluates the GPU's own iterate at every step (FP32 and FP64 paths);
* mixed n=2000 (8000 OR, 500 XOR, 200 at-least-t), 1024 restarts: sampled
  restarts against the oracle, in the launch shapes the benchmark uses, and
  one fused iteration through the benchmark's own graph-replayed path;
* large mixed n=100000 (420000 3-SAT, 10000 XOR, 2000 at-least-t of length
  128..512), 256 restarts: sampled restarts against the oracle, and one fused
  iteration through the benchmark's own autotuned, graph-replayed path.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_cases import TOL32, TOL64, errors, to_np

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


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_3sat_trajectory(ffs, dtype):
    inst = workloads.config1(workloads.instance_seed(1, 0))
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, 1)
    x0 = workloads.points(50, 1, workloads.point_seed(1000), dtype=np.float64)
    x = torch.from_numpy(x0).to(DEV, dtype)
    tol = TOL32 if dtype == torch.float32 else TOL64
    worst = 0.0
    for step in range(200):
        out = plan.eval(x, want_con=True)
        chk = plan.round_check(x)
        xn = x.cpu().numpy().astype(np.float64)
        ref = oracle.eval_batch(inst, xn, want_con=True)
        e = errors(inst, to_np(out), ref)
        worst = max(worst, max(e.values()))
        assert max(e.values()) <= tol, (step, e)
        rc = oracle.check(inst, xn)
        assert int(chk["n_sat"].item()) == int(rc["n_sat"][0])
        assert np.array_equal(chk["assign_bits"].cpu().numpy().view(np.uint32), rc["assign_bits"])
        plan.step(x, out["grad"], 0.05)
    print("worst natural-scale error over 200 steps:", worst)


def _sampled(ffs, inst, B, cols, dists, autotune=False):
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, B, autotune=autotune)
    res = {}
    for dist in dists:
        x = workloads.points(inst.n_vars, B, 77, dist=dist)
        xt = torch.from_numpy(x).to(DEV)
        out = to_np(plan.eval(xt, want_con=True))
        chk = to_np(plan.round_check(xt))
        sub = np.ascontiguousarray(x[:, cols].astype(np.float64))
        ref = oracle.eval_batch(inst, sub, want_con=True)
        e = errors(inst, out, ref, cols=cols)
        rc = oracle.check(inst, sub)
        assert np.array_equal(chk["n_sat"][cols], rc["n_sat"])
        assert np.array_equal(chk["unsat_bits"].view(np.uint32)[cols], rc["unsat_bits"])
        res[dist] = e
        assert max(e.values()) <= TOL32, (dist, e)
    return res


def test_mixed_n2000_b1024_sampled(ffs):
    inst = workloads.config2(workloads.instance_seed(2, 0))
    cols = np.array([0, 1, 63, 64, 511, 777, 1000, 1023])
    print(_sampled(ffs, inst, 1024, cols, ["uniform", "near_corner"], autotune=True))


def test_mixed_n2000_b1024_fused_iteration_bench_path(ffs):
    """The benchmark's own path (autotuned plan, graph-replayed fused
    iteration with check, projected step and ERWA) at full size: F on sampled
    restarts, satisfied counts and U over all restarts (bit-exact), the
    stepped points on sampled restarts and the new weights, against the
    oracle at the same starting points."""
    from gpu_cases import var_scale
    inst = workloads.config2(workloads.instance_seed(2, 0))
    B, eta, alpha = 1024, 0.05, 0.4
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, B, autotune=True)
    x0 = workloads.points(inst.n_vars, B, workloads.point_seed(workloads.instance_seed(2, 0)))
    xt = torch.from_numpy(x0).to(DEV)
    w0 = np.ones(inst.m)
    prob.set_weights(w0.astype(np.float32))
    out = to_np(plan.run_iters(xt, 1, eta, alpha))
    x1 = xt.cpu().numpy()
    w1 = prob.get_weights().cpu().numpy()
    cols = np.array([0, 5, 63, 64, 500, 1023])
    ref = oracle.eval_batch(inst, np.ascontiguousarray(x0[:, cols].astype(np.float64)), want_g=True)
    wsum = float(inst.m)
    assert np.max(np.abs(out["F"][cols] - ref["F"])) / wsum <= TOL32
    chk = oracle.check(inst, x0.astype(np.float64))
    assert np.array_equal(out["n_sat"], chk["n_sat"]) and np.array_equal(out["U"], chk["U"])
    want_x1 = np.clip(x0[:, cols].astype(np.float64) - eta * ref["g"], -1.0, 1.0)
    S = var_scale(inst)[:, None]
    assert np.max(np.abs(x1[:, cols] - want_x1) / (eta * S)) <= TOL32 + 1e-6
    want_w1 = oracle.erwa(chk["U"], w0, alpha)
    assert np.max(np.abs(w1 - want_w1)) <= 1e-6


def test_large_n100000_b256_fused_iteration_bench_path(ffs):
    """The large instance in the benchmark's configuration (autotuned plan:
    launch structure and pull class as the bench picks them, FP64 bins from
    128 literals, graph-replayed fused iteration with check, projected step
    and ERWA): F and the stepped point on sampled restarts against the
    oracle, satisfied counts and U over all 256 restarts bit-exact, the new
    weights against the oracle's update."""
    from gpu_cases import var_scale
    inst = workloads.config3(workloads.instance_seed(3, 0))
    B, eta, alpha = 256, 0.05, 0.4
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, B, autotune=True)
    print(plan.describe()["mode"], plan.describe()["pull"])
    x0 = workloads.points(inst.n_vars, B, workloads.point_seed(workloads.instance_seed(3, 0)))
    xt = torch.from_numpy(x0).to(DEV)
    w0 = np.ones(inst.m)
    prob.set_weights(w0.astype(np.float32))
    out = to_np(plan.run_iters(xt, 1, eta, alpha))
    x1 = xt.cpu().numpy()
    w1 = prob.get_weights().cpu().numpy()
    cols = np.array([0, 131, 255])
    ref = oracle.eval_batch(inst, np.ascontiguousarray(x0[:, cols].astype(np.float64)), want_g=True)
    assert np.max(np.abs(out["F"][cols] - ref["F"])) / float(inst.m) <= TOL32
    chk = oracle.check(inst, x0.astype(np.float64))
    assert np.array_equal(out["n_sat"], chk["n_sat"]) and np.array_equal(out["U"], chk["U"])
    want_x1 = np.clip(x0[:, cols].astype(np.float64) - eta * ref["g"], -1.0, 1.0)
    S = var_scale(inst)[:, None]
    assert np.max(np.abs(x1[:, cols] - want_x1) / (eta * S)) <= TOL32 + 1e-6
    assert np.max(np.abs(w1 - oracle.erwa(chk["U"], w0, alpha))) <= 1e-6


def test_large_mixed_n100000_b256_sampled(ffs):
    inst = workloads.config3(workloads.instance_seed(3, 0))
    cols = np.array([0, 131, 255])
    print(_sampled(ffs, inst, 256, cols, ["uniform"]))
