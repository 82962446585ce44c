"""The unit-circle form (FFSAT_FLAG_UNIT_CIRCLE, the paper's own basis kept as
an ablation) on the GPU against the FP64 oracle: parity where that form is
well conditioned (short constraints, or points near the centre of the box),
every segment shape, and the precision loss it shows for long constraints
near the corners, next to the bounded basis on the same inputs."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_cases import TOL32, errors, points, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL_UC64 = 1e-10   # FP64 unit-circle form in its well-conditioned range


@pytest.fixture(scope="module")
def ffs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_15020_amd as P
    P.lib()
    return P


def _eval(plan, x, dtype):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(DEV, dtype)
    out = plan.eval(xt, want_con=True)
    torch.cuda.synchronize()
    return to_np(out)


def _short_instance():
    # every kind through the transform (FORCE_DFT), lengths 1..32: segment
    # shapes (4, 1), (8, 1), (16, 1), (16, 2); thresholds inside and outside [1, k]
    inst = workloads.random_hybrid(300, 21, n_or=60, or_len=(1, 9), n_xor=60, xor_len=(1, 32),
                                   n_card=80, card_len=(1, 32), card_t=(0, 20), weights="uniform")
    return inst


@pytest.mark.parametrize("dist", ["uniform", "mixed_edge"])
def test_f64_short_constraints(ffs, dist):
    inst = _short_instance()
    prob = ffs.Problem(inst, device=0, flags=ffs.FLAG_UNIT_CIRCLE | ffs.FLAG_FORCE_DFT)
    B = 67
    plan = ffs.Plan(prob, B)
    x = points(inst, B, 5, dist).astype(np.float64)
    g = _eval(plan, x, torch.float64)
    ref = oracle.eval_batch(inst, x, want_con=True)
    e = errors(inst, g, ref)
    print(dist, e)
    assert e["con_val"] <= TOL_UC64 and e["F"] <= TOL_UC64 and e["grad"] <= TOL_UC64, e


def test_fp32_io_fp64_arithmetic(ffs):
    """FP32 evaluation with every root-of-unity bin in FP64 arithmetic."""
    inst = _short_instance()
    prob = ffs.Problem(inst, device=0, fp64_min_len=1, flags=ffs.FLAG_UNIT_CIRCLE | ffs.FLAG_FORCE_DFT)
    B = 70
    plan = ffs.Plan(prob, B)
    x = points(inst, B, 6, "uniform")
    g = _eval(plan, x, torch.float32)
    ref = oracle.eval_batch(inst, x.astype(np.float64), want_con=True)
    e = errors(inst, g, ref)
    assert e["con_val"] <= TOL32 and e["F"] <= TOL32 and e["grad"] <= TOL32, e


def test_f32_short_constraints(ffs):
    """FP32 arithmetic in the unit-circle form holds 1e-5 for short constraints."""
    inst = workloads.random_hybrid(200, 22, n_or=40, or_len=(1, 8), n_card=60, card_len=(2, 12),
                                   weights="uniform")
    prob = ffs.Problem(inst, device=0, flags=ffs.FLAG_UNIT_CIRCLE)
    B = 65
    plan = ffs.Plan(prob, B)
    x = points(inst, B, 8, "uniform")
    g = _eval(plan, x, torch.float32)
    ref = oracle.eval_batch(inst, x.astype(np.float64), want_con=True)
    e = errors(inst, g, ref)
    assert e["con_val"] <= TOL32 and e["grad"] <= TOL32, e


def test_f64_long_shapes_near_centre(ffs):
    """Lengths up to 512 (L = 4 .. 32 lanes of 16) at points with |x| <= 0.2,
    where the unit-circle products stay well scaled."""
    n = 900
    rng = np.random.default_rng(3)
    groups = []
    for k, t in [(40, 10), (64, 32), (100, 25), (128, 64), (200, 50), (256, 128), (300, 75), (400, 399),
                 (512, 128), (511, 255)]:
        v = rng.choice(n, size=k, replace=False) + 1
        sg = np.where(rng.random(k) < 0.5, -1, 1)
        groups.append((2, [t], [(v * sg).astype(np.int32)]))
    inst = workloads.assemble(n, groups)
    inst.weights = rng.uniform(0.5, 1.5, inst.m).astype(np.float32)
    prob = ffs.Problem(inst, device=0, flags=ffs.FLAG_UNIT_CIRCLE)
    B = 66
    plan = ffs.Plan(prob, B)
    x = 0.2 * points(inst, B, 9, "uniform").astype(np.float64)
    g = _eval(plan, x, torch.float64)
    ref = oracle.eval_batch(inst, x, want_con=True)
    e = errors(inst, g, ref)
    print(e)
    assert e["con_val"] <= TOL_UC64 and e["F"] <= TOL_UC64 and e["grad"] <= TOL_UC64, e


def test_precision_loss_near_corners(ffs):
    """At |x| = 0.99 the unit-circle form in FP64 loses all accuracy at k = 128
    (the terms f~[a] prod (omega^a + l) reach ~1e19 and cancel to a value of
    size <= 1) while it is exact to ~1e-13 at k = 16; the bounded basis stays
    at rounding level for both.  The integer check is unaffected."""
    n = 400
    rng = np.random.default_rng(4)
    groups = []
    for k in (16, 128):
        for _ in range(4):
            v = rng.choice(n, size=k, replace=False) + 1
            groups.append((2, [k // 4], [v.astype(np.int32)]))
    inst = workloads.assemble(n, groups)
    B = 64
    x = points(inst, B, 10, "near_corner").astype(np.float64)
    ref = oracle.eval_batch(inst, x, want_con=True)
    p_uc = ffs.Problem(inst, device=0, flags=ffs.FLAG_UNIT_CIRCLE)
    p_pb = ffs.Problem(inst, device=0)
    g_uc = _eval(ffs.Plan(p_uc, B), x, torch.float64)
    g_pb = _eval(ffs.Plan(p_pb, B), x, torch.float64)
    err_uc = np.abs(g_uc["con_val"] - ref["con_val"])
    err_pb = np.abs(g_pb["con_val"] - ref["con_val"])
    short, long_ = slice(0, 4), slice(4, 8)
    print("uc k=16 %.2e  uc k=128 %.2e  pb %.2e" % (err_uc[short].max(), err_uc[long_].max(), err_pb.max()))
    assert err_uc[short].max() <= 1e-10
    assert np.median(err_uc[long_]) >= 1.0
    assert err_pb.max() <= 1e-12
    plan = ffs.Plan(p_uc, B)
    chk = plan.round_check(torch.from_numpy(x.astype(np.float32)).to(DEV), want=("n_sat", "unsat_bits"))
    want = oracle.check(inst, x.astype(np.float32).astype(np.float64))
    assert np.array_equal(chk["n_sat"].cpu().numpy(), want["n_sat"])
    assert np.array_equal(chk["unsat_bits"].cpu().numpy().view(np.uint32), want["unsat_bits"])


def test_ablation_harness_runs(ffs, monkeypatch):
    """The basis ablation end to end on two short lengths: every cell present,
    the bounded basis in FP64 agrees with itself, the unit circle in FP64 is
    accurate at these lengths."""
    import argparse
    from paper_2308_15020_amd import ablation
    monkeypatch.setattr(ablation, "KS", (8, 16))
    rows = ablation.run(argparse.Namespace(B=64, per_k=3, reps=2))
    assert len(rows) == 2 * 2 * 2 * 2
    for r in rows:
        assert r["max_err"] is not None and r["nonfinite"] == 0.0 and r["ms_per_eval"] > 0
        if r["basis"] == "pb" and r["dtype"] == "float64":
            assert r["max_err"] == 0.0
        if r["basis"] == "uc" and r["dtype"] == "float64":
            assert r["max_err"] <= 1e-10
