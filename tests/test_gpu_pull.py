"""The pulled gradient of short transform-free constraints (k_pull) against
the oracle and against the slot path (needs an MI355X).

With the pull path a wave owns a chunk of variables and 64 restarts and
gathers the other literals of every short OR / AND / XOR / constant
constraint that holds a variable, instead of the evaluation writing one
slot per literal and the reduction reading it back.  The objective and the
exact check of those constraints are taken at their first literal.  These
tests cover both pull classes (length <= 3, <= 7), chunk sizes that leave a
ragged last chunk, restart counts that leave a ragged last wave, the fused
check (bit-exact), the projected step in place (through the second buffer),
the step loop and the fused iterations with an odd and an even number of
steps (ping-pong between two buffers), graphs and eager launches.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_cases import TOL32, errors, every_bin_instance, points, to_np, var_scale

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


@pytest.fixture(scope="module")
def mixed(ffs):
    inst = every_bin_instance()
    return inst, ffs.Problem(inst, device=0)


def _x(inst, B, seed, dist="uniform"):
    return torch.from_numpy(np.ascontiguousarray(points(inst, B, seed, dist))).to(DEV)


@pytest.mark.parametrize("pull,vc", [("le3", 1), ("le3", 7), ("le7", 3), ("le7", 8)])
@pytest.mark.parametrize("B,dist", [(1, "uniform"), (70, "mixed_edge"), (130, "corner")])
def test_pull_eval_against_oracle(ffs, mixed, pull, vc, B, dist):
    inst, prob = mixed
    plan = ffs.Plan(prob, B, pull=pull, pull_vc=vc)
    d = plan.describe()
    assert d["pull"] == (3 if pull == "le3" else 7) and any(b["pulled"] for b in d["bins"]["f32"])
    x = _x(inst, B, 300 + B + vc, dist)
    out = plan.eval(x, want_check=True)   # no per-constraint values: the pull path serves it
    torch.cuda.synchronize()
    g = to_np(out)
    xn = x.cpu().numpy().astype(np.float64)
    ref = oracle.eval_batch(inst, xn)
    e = errors(inst, g, ref)
    assert max(e.values()) <= TOL32, e
    rc = oracle.check(inst, xn)
    assert np.array_equal(g["n_sat"], rc["n_sat"])
    assert np.array_equal(g["U"], rc["U"])
    assert np.array_equal(g["unsat_bits"].view(np.uint32), rc["unsat_bits"])


def test_pull_equals_slot_gradient(ffs, mixed):
    inst, prob = mixed
    B = 96
    x = _x(inst, B, 411)
    slot = ffs.Plan(prob, B, pull="off")
    ref = to_np(slot.eval(x))
    for pull in ("le3", "le7"):
        got = to_np(ffs.Plan(prob, B, pull=pull).eval(x))
        S = var_scale(inst)[:, None]
        assert np.max(np.abs(got["grad"] - ref["grad"]) / S) <= 1e-6
        assert np.max(np.abs(got["F"] - ref["F"])) / np.abs(inst.weights).sum() <= 1e-6


def test_pull_eval_step_in_place(ffs, mixed):
    inst, prob = mixed
    B, eta = 70, 0.07
    x0 = _x(inst, B, 512)
    a, b = x0.clone(), x0.clone()
    pa = ffs.Plan(prob, B, pull="le7", pull_vc=5)
    pb = ffs.Plan(prob, B, pull="off")
    oa = pa.eval_step(a, eta)
    ob = pb.eval_step(b, eta)
    torch.cuda.synchronize()
    S = var_scale(inst)[:, None]
    assert np.max(np.abs(a.cpu().numpy() - b.cpu().numpy()) / (eta * S)) <= 1e-6
    assert torch.equal(oa["n_sat"], ob["n_sat"]) and torch.equal(oa["U"], ob["U"])


@pytest.mark.parametrize("T", [1, 4, 5])
@pytest.mark.parametrize("use_graphs,side_streams", [(True, True), (False, True), (True, False)])
def test_pull_iterations_follow_slot_path(ffs, mixed, T, use_graphs, side_streams):
    """T fused iterations (check, step, adaptive weights) with the pull path
    alternate between two point buffers; the result must land in x for odd
    and even T and follow the slot path's trajectory."""
    inst, prob = mixed
    B, eta, alpha = 64, 0.05, 0.4
    x0 = _x(inst, B, 77)
    w0 = inst.weights_or_ones().astype(np.float32)
    res = {}
    for pull in ("off", "le7"):
        prob.set_weights(w0)
        plan = ffs.Plan(prob, B, pull=pull, use_graphs=use_graphs, side_streams=side_streams)
        x = x0.clone()
        out = plan.run_iters(x, T, eta, alpha)
        out = plan.run_iters(x, T, eta, alpha, out=out)   # a second replay of the same graph
        torch.cuda.synchronize()
        res[pull] = (x.cpu().numpy(), to_np(out), prob.get_weights().cpu().numpy())
    xs, os_, ws = res["off"]
    xp, op, wp = res["le7"]
    assert np.max(np.abs(xs - xp)) <= 1e-4
    assert np.max(np.abs(ws - wp)) <= 1e-5
    assert np.max(np.abs(os_["F"] - op["F"])) / np.abs(w0).sum() <= 1e-4


@pytest.mark.parametrize("T", [3, 4])
def test_pull_run_steps_equals_eager_steps(ffs, mixed, T):
    inst, prob = mixed
    B, eta = 70, 0.05
    prob.set_weights(inst.weights_or_ones().astype(np.float32))
    x0 = _x(inst, B, 91)
    plan = ffs.Plan(prob, B, pull="le3")
    xa = x0.clone()
    plan.run_steps(xa, T, eta)
    xb = x0.clone()
    for _ in range(T):
        plan.eval_step(xb, eta, want_F=False, want_check=False)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)   # same kernels, same order


def test_pull_3sat_part_of_large_instance_sampled(ffs):
    """The 3-SAT part of the large instance (n = 100000, 420000 clauses, 256
    restarts) through the pull path in the tuned launch shape: sampled
    restarts of F and the gradient against the oracle; all restarts' checks
    bit-exact."""
    inst = workloads.config3a(workloads.instance_seed(3, 0))
    B = 256
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, B, pull="le3")
    x0 = workloads.points(inst.n_vars, B, workloads.point_seed(3000))
    x = torch.from_numpy(x0).to(DEV)
    out = to_np(plan.eval(x, want_check=True))
    cols = np.array([0, 63, 64, 200, 255])
    ref = oracle.eval_batch(inst, np.ascontiguousarray(x0[:, cols].astype(np.float64)))
    e = errors(inst, {"F": out["F"], "grad": out["grad"]}, ref, cols=cols)
    assert max(e.values()) <= TOL32, e
    rc = oracle.check(inst, x0.astype(np.float64))
    assert np.array_equal(out["n_sat"], rc["n_sat"]) and np.array_equal(out["U"], rc["U"])
