"""HIP path against the FP64 oracle (needs an MI355X).

Every comparison uses the same seeded inputs on both sides; floating-point
results are compared at the natural scale (per-constraint values to 1e-5
absolute, the objective relative to sum |w|, the gradient of a variable
relative to the weight of its constraints), integer results bit-exactly.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_cases import TOL32, TOL64, errors, every_bin_instance, points, to_np, var_scale

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
    prob = ffs.Problem(inst, device=0)
    return inst, prob


def _gpu_eval(plan, x, dtype=torch.float32, con=True):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(DEV, dtype)
    out = plan.eval(xt, want_con=con)
    torch.cuda.synchronize()
    return to_np(out)


@pytest.fixture(scope="module")
def mixed_fp32(ffs):
    """The same instance with FP32 root-of-unity products up to 256 literals
    (FP64 only beyond): the FP32 kernels' long shapes."""
    inst = every_bin_instance()
    prob = ffs.Problem(inst, device=0, fp64_min_len=257)
    return inst, prob


def test_problem_bins_cover_all_variants(mixed):
    inst, prob = mixed
    info = prob.info()
    assert info["n_cons"] == inst.m and info["nnz"] == inst.nnz and info["max_len"] == 512
    assert info["n_bins_f32"] >= 12 and info["n_bins_f64"] >= 8


@pytest.mark.parametrize("dist", ["uniform", "near_corner", "corner", "mixed_edge"])
@pytest.mark.parametrize("B", [1, 70])
def test_eval_f32_every_bin(ffs, mixed, dist, B):
    inst, prob = mixed
    plan = ffs.Plan(prob, B)
    x = points(inst, B, 100 + B, dist)
    g = _gpu_eval(plan, x)
    ref = oracle.eval_batch(inst, x.astype(np.float64), want_con=True)
    e = errors(inst, g, ref)
    print(dist, B, e)
    assert e["con_val"] <= TOL32 and e["F"] <= TOL32 and e["grad"] <= TOL32, e


@pytest.mark.parametrize("dist", ["uniform", "near_corner", "corner", "mixed_edge"])
def test_eval_f32_long_root_of_unity_fp32(ffs, mixed_fp32, dist):
    inst, prob = mixed_fp32
    B = 70
    plan = ffs.Plan(prob, B)
    x = points(inst, B, 170, dist)
    g = _gpu_eval(plan, x)
    ref = oracle.eval_batch(inst, x.astype(np.float64), want_con=True)
    e = errors(inst, g, ref)
    print(dist, e)
    assert e["con_val"] <= TOL32 and e["F"] <= TOL32 and e["grad"] <= TOL32, e


@pytest.mark.parametrize("dist", ["uniform", "near_corner", "mixed_edge"])
def test_eval_f64_every_bin(ffs, mixed, dist):
    inst, prob = mixed
    B = 67
    plan = ffs.Plan(prob, B)
    x = points(inst, B, 7, dist).astype(np.float64)
    g = _gpu_eval(plan, x, torch.float64)
    ref = oracle.eval_batch(inst, x, want_con=True)
    e = errors(inst, g, ref)
    print(dist, e)
    assert e["con_val"] <= TOL64 and e["F"] <= TOL64 and e["grad"] <= TOL64, e


@pytest.mark.parametrize("fg", [2, 4])
def test_fp64_frequency_split(ffs, mixed, tmp_path, fg):
    """Per-bin FP64 root-of-unity launches with each constraint's frequencies
    split over fg waves of a workgroup (the waves' moments added through LDS
    in wave order before the gradient pass), forced through the tune cache:
    values and gradients against the oracle."""
    import json
    inst, prob = mixed
    B = 64
    cache = str(tmp_path / "tune.json")
    ffs.Plan(prob, B, autotune=True, tune_cache=cache, mode="per_bin").close()
    c = json.load(open(cache))
    keys = [k for k in c if "|c1|t1|" in k]   # root-of-unity class, FP64 arithmetic
    assert keys
    for k in keys:
        c[k] = [1, 1, fg]
    json.dump(c, open(cache, "w"))
    plan = ffs.Plan(prob, B, autotune=True, tune_cache=cache, mode="per_bin")
    d = plan.describe()
    f64 = [b for b in d["bins"]["f32"] if b["ct"] == "f64" and b["class"] == "dft"]
    assert f64 and all(b["fg"] == fg for b in f64)
    for dist in ("uniform", "near_corner"):
        x = points(inst, B, 55, dist)
        g = _gpu_eval(plan, x)
        ref = oracle.eval_batch(inst, x.astype(np.float64), want_con=True)
        e = errors(inst, g, ref)
        print(fg, dist, e)
        assert e["con_val"] <= TOL32 and e["F"] <= TOL32 and e["grad"] <= TOL32, e
    plan.close()


def test_force_dft_matches_closed_forms(ffs):
    """OR and XOR through the root-of-unity path against the closed forms."""
    inst = workloads.random_hybrid(600, 5, n_or=120, or_len=(1, 64), n_xor=120, xor_len=(1, 300),
                                   n_card=10, card_len=(2, 40), weights="uniform")
    prob = ffs.Problem(inst, device=0, flags=ffs.FLAG_FORCE_DFT)
    B = 65
    plan = ffs.Plan(prob, B)
    for dist in ("uniform", "near_corner"):
        x = points(inst, B, 3, dist)
        g = _gpu_eval(plan, x)
        ref = oracle.eval_batch(inst, x.astype(np.float64), want_con=True, route=oracle.ROUTE_AUTH)
        e = errors(inst, g, ref)
        print(dist, e)
        assert e["con_val"] <= TOL32 and e["grad"] <= TOL32, e


def test_fp64_threshold_option(ffs, mixed):
    """fp64_min_len moves long root-of-unity products to FP64; values agree."""
    inst, _ = mixed
    prob = ffs.Problem(inst, device=0, fp64_min_len=20)
    B = 64
    plan = ffs.Plan(prob, B)
    x = points(inst, B, 9, "uniform")
    g = _gpu_eval(plan, x)
    ref = oracle.eval_batch(inst, x.astype(np.float64), want_con=True)
    e = errors(inst, g, ref)
    assert e["con_val"] <= TOL32 and e["grad"] <= TOL32, e


def test_step_bit_exact(ffs, mixed):
    inst, prob = mixed
    B = 77
    plan = ffs.Plan(prob, B)
    rng = np.random.default_rng(4)
    x = rng.uniform(-1.2, 1.2, (inst.n_vars, B)).astype(np.float32)
    gr = rng.normal(size=(inst.n_vars, B)).astype(np.float32)
    eb = rng.uniform(0, 0.5, B).astype(np.float32)
    for eta, use_b in ((0.05, False), (0.3, True)):
        xt = torch.from_numpy(x).to(DEV)
        plan.step(xt, torch.from_numpy(gr).to(DEV), eta, torch.from_numpy(eb).to(DEV) if use_b else None)
        want = oracle.step_f32(x, gr, eta, eb if use_b else None)
        assert np.array_equal(xt.cpu().numpy(), want)
    x64 = x.astype(np.float64)
    xt = torch.from_numpy(x64).to(DEV)
    plan.step(xt, torch.from_numpy(gr.astype(np.float64)).to(DEV), 0.1)
    assert np.array_equal(xt.cpu().numpy(), oracle.step_f64(x64, gr.astype(np.float64), 0.1))


@pytest.mark.parametrize("dist", ["uniform", "corner", "mixed_edge"])
def test_round_check_bit_exact(ffs, mixed, dist):
    inst, prob = mixed
    B = 100
    plan = ffs.Plan(prob, B)
    x = points(inst, B, 12, dist)
    for dt in (torch.float32, torch.float64):
        xt = torch.from_numpy(x).to(DEV, dt)
        out = to_np(plan.round_check(xt))
        ref = oracle.check(inst, x.astype(np.float64))
        assert np.array_equal(out["n_sat"], ref["n_sat"])
        assert np.array_equal(out["U"], ref["U"])
        assert np.array_equal(out["unsat_bits"].view(np.uint32), ref["unsat_bits"])
        assert np.array_equal(out["assign_bits"].view(np.uint32), ref["assign_bits"])


@pytest.mark.parametrize("dist", ["uniform", "mixed_edge"])
def test_eval_check_fused(ffs, mixed, dist):
    """Value, gradient and exact check of the same point from one pass."""
    inst, prob = mixed
    B = 90
    plan = ffs.Plan(prob, B)
    x = points(inst, B, 51, dist)
    xt = torch.from_numpy(x).to(DEV)
    fused = to_np(plan.eval(xt, want_con=True, want_check=True))
    plain = to_np(plan.eval(xt, want_con=True))
    for k in ("F", "grad", "con_val"):
        assert np.array_equal(fused[k], plain[k]), k
    ref = oracle.check(inst, x.astype(np.float64))
    assert np.array_equal(fused["n_sat"], ref["n_sat"])
    assert np.array_equal(fused["U"], ref["U"])
    assert np.array_equal(fused["unsat_bits"].view(np.uint32), ref["unsat_bits"])
    # check only (no value outputs requested)
    import ctypes as C
    from paper_2308_15020_amd._lib import check as chk, lib
    ns = torch.empty(B, dtype=torch.int32, device=DEV)
    U = torch.empty(inst.m, dtype=torch.int32, device=DEV)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    chk(lib().ffsat_eval_check(plan.handle, C.c_void_p(xt.data_ptr()), None, None, None,
                               C.c_void_p(ns.data_ptr()), None, C.c_void_p(U.data_ptr()), s))
    assert np.array_equal(ns.cpu().numpy(), ref["n_sat"]) and np.array_equal(U.cpu().numpy(), ref["U"])


def test_weights_erwa_and_weight_gradient(ffs, mixed):
    inst, prob = mixed
    B = 96
    plan = ffs.Plan(prob, B)
    w0 = prob.get_weights().cpu().numpy()
    assert np.array_equal(w0, inst.weights)
    x = points(inst, B, 21, "uniform")
    xt = torch.from_numpy(x).to(DEV)
    U = plan.round_check(xt, want=("U",))["U"]
    plan.erwa_update(U, 0.4)
    w1 = prob.get_weights().cpu().numpy()
    want = oracle.erwa(U.cpu().numpy(), w0.astype(np.float64), 0.4)
    assert np.max(np.abs(w1 - want)) <= 1e-6
    # zero counts: r = 0
    plan.erwa_update(torch.zeros(inst.m, dtype=torch.int32, device=DEV), 0.4)
    w2 = prob.get_weights().cpu().numpy()
    assert np.max(np.abs(w2 - 0.6 * w1.astype(np.float64))) <= 1e-6
    # the objective uses the updated weights
    out = plan.eval(xt, want_con=True)
    ref = oracle.eval_batch(inst, x.astype(np.float64), w=w2.astype(np.float64), want_con=True)
    e = errors(inst, to_np(out), ref)
    assert e["F"] <= TOL32 and e["grad"] <= TOL32
    gF = torch.from_numpy(np.random.default_rng(2).normal(size=B).astype(np.float32)).to(DEV)
    gw = plan.weight_grad(out["con_val"], gF).cpu().numpy()
    want = oracle.wgrad(ref["con_val"], gF.cpu().numpy().astype(np.float64))
    assert np.max(np.abs(gw - want)) <= TOL32 * np.abs(gF.cpu().numpy()).sum()
    prob.set_weights(inst.weights)
    assert np.array_equal(prob.get_weights().cpu().numpy(), inst.weights)


def test_erwa_large_m_two_pass(ffs):
    """More than 65536 constraints: partial maxima, then the update."""
    rng = np.random.default_rng(17)
    m, n = 70001, 500
    lits = np.stack([rng.choice(n, 3, replace=False) + 1 for _ in range(64)])
    lits = lits[rng.integers(0, 64, m)] * np.where(rng.random((m, 3)) < 0.5, -1, 1)
    inst = workloads.assemble(n, [(0, np.zeros(m, np.int32), list(lits.astype(np.int32)))])
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, 64)
    w0 = rng.uniform(0.5, 1.5, m).astype(np.float32)
    prob.set_weights(w0)
    Un = rng.integers(0, 64, m).astype(np.int32)
    Un[12345] = 977   # the maximum sits in one block's range
    plan.erwa_update(torch.from_numpy(Un).to(DEV), 0.3)
    want = oracle.erwa(Un, w0.astype(np.float64), 0.3)
    assert np.max(np.abs(prob.get_weights().cpu().numpy() - want)) <= 1e-6


def test_determinism(ffs, mixed):
    """Bitwise-equal results on repeated calls, with bins on side streams or
    all on one stream."""
    inst, prob = mixed
    B = 128
    plan = ffs.Plan(prob, B)
    one = ffs.Plan(prob, B, side_streams=False)
    x = torch.from_numpy(points(inst, B, 5, "uniform")).to(DEV)
    a = to_np(plan.eval(x, want_con=True, want_check=True))
    b = to_np(plan.eval(x, want_con=True, want_check=True))
    c = to_np(one.eval(x, want_con=True, want_check=True))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k


def test_run_steps_graph_equals_eager_loop(ffs, mixed):
    inst, prob = mixed
    B = 72
    x0 = points(inst, B, 31, "uniform")
    T, eta = 7, 0.05
    res = []
    for graphs in (True, False):
        plan = ffs.Plan(prob, B, use_graphs=graphs)
        x = torch.from_numpy(x0).to(DEV)
        F = torch.empty(B, device=DEV)
        plan.run_steps(x, T, eta, F)
        plan.run_steps(x, T, eta, F)        # replay of the cached graph
        res.append((x.cpu().numpy(), F.cpu().numpy()))
    plan = ffs.Plan(prob, B)
    x = torch.from_numpy(x0).to(DEV)
    for t in range(2 * T):
        out = plan.eval(x, want_F=(t == 2 * T - 1))
        if t == 2 * T - 1:
            Flast = out["F"].cpu().numpy()
        plan.step(x, out["grad"], eta)
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][0], x.cpu().numpy())
    assert np.array_equal(res[0][1], res[1][1])
    assert np.max(np.abs(res[0][1] - Flast)) <= 1e-6 * np.abs(inst.weights).sum()


def test_eval_step_equals_eval_then_step(ffs, mixed):
    inst, prob = mixed
    B = 75
    plan = ffs.Plan(prob, B)
    x0 = points(inst, B, 61, "uniform")
    xa = torch.from_numpy(x0).to(DEV)
    xb = torch.from_numpy(x0).to(DEV)
    for _ in range(3):
        fused = to_np(plan.eval_step(xa, 0.07))
        ref = to_np(plan.eval(xb, want_check=True))
        plan.step(xb, torch.from_numpy(ref["grad"]).to(DEV), 0.07)
        assert np.array_equal(fused["F"], ref["F"]) and np.array_equal(fused["n_sat"], ref["n_sat"])
        assert np.array_equal(fused["U"], ref["U"])
        assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy())


@pytest.mark.parametrize("mode", ["group_all", "group_dft"])
def test_grouped_launch_matches_per_bin_launches(ffs, mixed, mode):
    """Grouped FP32 launches against one launch per bin (side streams on):
    objective and gradient to the FP32 tolerance, integer outputs exactly."""
    inst, prob = mixed
    B = 200
    x = torch.from_numpy(points(inst, B, 83, "uniform")).to(DEV)
    pg = ffs.Plan(prob, B, mode=mode)
    pb = ffs.Plan(prob, B, mode="per_bin")
    dg = pg.describe()
    assert dg["grouped"] and dg["mode"] == mode and not pb.describe()["grouped"]
    a = to_np(pg.eval(x, want_con=True))
    b = to_np(pb.eval(x, want_con=True))
    S = var_scale(inst)[:, None]
    assert np.max(np.abs(a["grad"] - b["grad"]) / S) <= TOL32
    assert np.max(np.abs(a["con_val"] - b["con_val"])) <= TOL32
    assert np.max(np.abs(a["F"] - b["F"])) <= 1e-6 * np.abs(inst.weights).sum()
    ca = to_np(pg.round_check(x))
    cb = to_np(pb.round_check(x))
    for k in ("assign_bits", "n_sat", "unsat_bits", "U"):
        assert np.array_equal(ca[k], cb[k]), k


@pytest.mark.parametrize("mode,gc,gf", [("group_all", 4, 1), ("group_all", 16, 1), ("group_all", 8, 4),
                                         ("group_dft", 0, 4), ("group_dft", 0, 1)])
def test_grouped_shapes_match_per_bin_launches(ffs, mixed, tmp_path, mode, gc, gf):
    """Every grouped shape the tuner may pick (transform-free constraints per
    wave inside the all-bin group, root-of-unity frequency split), forced
    through the tune cache, against one launch per bin: FP32 tolerance for
    values, exact for the check; the fused iterations stay bitwise equal
    between graph replay and eager launches."""
    import json
    inst, prob = mixed
    B = 96
    cache = str(tmp_path / "tune.json")
    ffs.Plan(prob, B, autotune=True, tune_cache=cache, mode=mode).close()
    c = json.load(open(cache))
    key = [k for k in c if "|mode|" in k]
    assert len(key) == 1
    codes = {"group_all": 2, "group_dft": 3}
    c[key[0]] = [codes[mode], 0, 8 * gc + gf]
    json.dump(c, open(cache, "w"))
    pg = ffs.Plan(prob, B, autotune=True, tune_cache=cache, mode=mode)
    d = pg.describe()
    assert d["tuned_modes"] == [] and (d["group_real_cpw"], d["group_dft_fg"]) == (gc, gf)
    ing = [b for b in d["bins"]["f32"] if b["in_group"]]
    assert ing and all(b["fg"] == gf for b in ing if b["class"] == "dft")
    if mode == "group_all":
        assert any(b["class"] == "real" for b in ing)
    pb = ffs.Plan(prob, B, mode="per_bin")
    x = torch.from_numpy(points(inst, B, 91, "mixed_edge")).to(DEV)
    a = to_np(pg.eval(x, want_con=True))
    b = to_np(pb.eval(x, want_con=True))
    S = var_scale(inst)[:, None]
    assert np.max(np.abs(a["grad"] - b["grad"]) / S) <= TOL32
    assert np.max(np.abs(a["con_val"] - b["con_val"])) <= TOL32
    assert np.max(np.abs(a["F"] - b["F"])) <= 1e-6 * np.abs(inst.weights).sum()
    ca, cb = to_np(pg.round_check(x)), to_np(pb.round_check(x))
    for k in ("n_sat", "unsat_bits", "U"):
        assert np.array_equal(ca[k], cb[k]), k
    w0 = prob.get_weights().clone()
    xr, xe = x.clone(), x.clone()
    orr = pg.run_iters(xr, 3, 0.05, 0.4)
    wr = prob.get_weights().clone()
    prob.set_weights(w0.cpu().numpy())
    pe = ffs.Plan(prob, B, autotune=True, tune_cache=cache, mode=mode, use_graphs=False)
    oe = pe.run_iters(xe, 3, 0.05, 0.4)
    torch.cuda.synchronize()
    assert torch.equal(xr, xe) and torch.equal(wr, prob.get_weights())
    assert torch.equal(orr["F"], oe["F"]) and torch.equal(orr["n_sat"], oe["n_sat"])
    prob.set_weights(inst.weights)


def test_run_iters_graph_equals_eager(ffs, mixed):
    """Graph-replayed fused iterations (with ERWA) against the same calls made
    eagerly: bitwise, on three replays with eager work and syncs between."""
    inst, prob = mixed
    B, T, eta, alpha = 96, 3, 0.05, 0.4
    x0 = torch.from_numpy(points(inst, B, 61, "uniform")).to(DEV)
    pg = ffs.Plan(prob, B, use_graphs=True)
    pe = ffs.Plan(prob, B, use_graphs=False)
    w0 = prob.get_weights().clone()
    xg, xe = x0.clone(), x0.clone()
    outg = {}
    for rep in range(3):
        prob.set_weights(w0)
        og = outg = pg.run_iters(xg, T, eta, alpha, out=outg)   # same arguments: one graph, replayed
        torch.cuda.synchronize()
        wg = prob.get_weights().clone()
        prob.set_weights(w0)
        for _ in range(T):
            oe = pe.eval_step(xe, eta)
            pe.erwa_update(oe["U"], alpha)
        torch.cuda.synchronize()
        we = prob.get_weights().clone()
        assert torch.equal(xg, xe), rep
        assert torch.equal(wg, we), rep
        assert torch.equal(og["F"], oe["F"]) and torch.equal(og["n_sat"], oe["n_sat"]), rep
        assert torch.equal(og["U"], oe["U"]), rep
        w0 = we.clone()
        xe.mul_(0.5)                                     # eager work between replays
        xg.copy_(xe)
    prob.set_weights(inst.weights)


@pytest.mark.parametrize("B", [70, 200, 1024])
@pytest.mark.parametrize("use_graphs,side_streams,mode", [
    (False, True, "auto"), (True, True, "auto"), (True, False, "auto"), (False, False, "auto"),
    (True, True, "per_bin"), (True, True, "group_all"), (False, True, "per_bin")])
def test_run_iters_variants_equal_eval_step_sequence(ffs, mixed, B, use_graphs, side_streams, mode):
    """ffsat_run_iters (graph or eager; with the side stream that takes the
    weights, the reset of U and the level-2 sums, or sequential without side
    streams; every launch structure) against eval_step + erwa_update calls of
    a plan with the same launch structure: bitwise, T = 1 and T = 4 (the last
    iteration's U is kept for the caller, earlier ones are reset)."""
    inst, prob = mixed
    eta, alpha = 0.05, 0.4
    x0 = torch.from_numpy(points(inst, B, 62, "uniform")).to(DEV)
    pr = ffs.Plan(prob, B, use_graphs=use_graphs, side_streams=side_streams, mode=mode)
    pe = ffs.Plan(prob, B, use_graphs=False, mode=mode)   # same launch structure: same rounding
    w0 = prob.get_weights().clone()
    for T in (1, 4):
        prob.set_weights(w0)
        xr = x0.clone()
        o = pr.run_iters(xr, T, eta, alpha)
        torch.cuda.synchronize()
        wr = prob.get_weights().clone()
        prob.set_weights(w0)
        xe = x0.clone()
        for _ in range(T):
            oe = pe.eval_step(xe, eta)
            pe.erwa_update(oe["U"], alpha)
        torch.cuda.synchronize()
        assert torch.equal(xr, xe) and torch.equal(wr, prob.get_weights()), T
        assert torch.equal(o["F"], oe["F"]) and torch.equal(o["n_sat"], oe["n_sat"]) and torch.equal(o["U"], oe["U"]), T
    prob.set_weights(inst.weights)


def test_autotune_keeps_results(ffs, mixed, tmp_path):
    inst, prob = mixed
    B = 130
    x = torch.from_numpy(points(inst, B, 41, "uniform")).to(DEV)
    p0 = ffs.Plan(prob, B)
    a = to_np(p0.eval(x, want_con=True))
    cache = str(tmp_path / "tune.json")
    p1 = ffs.Plan(prob, B, autotune=True, tune_cache=cache)
    d = p1.describe()
    assert d["tuned"] and len(d["bins"]["f32"]) >= 12
    b = to_np(p1.eval(x, want_con=True))
    # the tuner may split a root-of-unity bin's frequencies differently (a
    # different summation grouping): equal to the FP32 parity tolerance
    S = var_scale(inst)[:, None]
    assert np.max(np.abs(a["grad"] - b["grad"]) / S) <= TOL32
    assert np.max(np.abs(a["con_val"] - b["con_val"])) <= TOL32
    assert np.max(np.abs(a["F"] - b["F"])) <= 1e-6 * np.abs(inst.weights).sum()
    p2 = ffs.Plan(prob, B, autotune=True, tune_cache=cache)     # served from the cache file
    d2 = p2.describe()
    assert d2["tuned_modes"] == []     # launch structure and pull class read back, not timed again
    assert d2["bins"] == d["bins"]
    keys = ("mode", "pull", "group_real_cpw", "group_dft_fg")
    assert [d2[k] for k in keys] == [d[k] for k in keys]


def test_debug_nonfinite(ffs):
    inst = workloads.random_hybrid(20, 1, n_or=10, or_len=(2, 3))
    prob = ffs.Problem(inst, device=0, flags=ffs.FLAG_DEBUG_CHECKS)
    plan = ffs.Plan(prob, 4)
    x = torch.zeros(20, 4, device=DEV)
    plan.eval(x)
    x[3, 2] = float("nan")
    with pytest.raises(ffs.FFSatError) as ei:
        plan.eval(x)
    assert ei.value.code == "E_NONFINITE"


@pytest.mark.parametrize("B", [1, 2, 63, 64, 65, 129])
def test_tiny_and_ragged(ffs, B):
    """n = 1 / m = 1 problems, length-1 constraints, thresholds out of range."""
    cases = [
        workloads.assemble(1, [(0, [0], [np.array([-1], np.int32)])]),
        workloads.assemble(1, [(1, [0], [np.array([1], np.int32)])]),
        workloads.assemble(1, [(2, [1], [np.array([1], np.int32)])]),
        workloads.assemble(3, [(2, [0], [np.array([1, -2, 3], np.int32)]),
                               (2, [4], [np.array([1, 2, 3], np.int32)]),
                               (2, [3], [np.array([-1, -2, -3], np.int32)]),
                               (1, [1], [np.array([2], np.int32)])]),
    ]
    for inst in cases:
        prob = ffs.Problem(inst, device=0)
        plan = ffs.Plan(prob, B)
        x = workloads.points(inst.n_vars, B, B, dist="mixed_edge")
        g = _gpu_eval(plan, x)
        ref = oracle.eval_batch(inst, x.astype(np.float64), want_con=True)
        e = errors(inst, g, ref)
        assert max(e.values()) <= TOL32, e
        out = to_np(plan.round_check(torch.from_numpy(x).to(DEV)))
        rc = oracle.check(inst, x.astype(np.float64))
        assert np.array_equal(out["n_sat"], rc["n_sat"]) and np.array_equal(out["U"], rc["U"])


def test_device_mismatch(ffs):
    inst = workloads.random_hybrid(10, 1, n_or=3)
    with pytest.raises(ffs.FFSatError) as ei:
        ffs.Problem(inst, device=torch.cuda.device_count())
    assert ei.value.code == "E_DEVICE_MISMATCH"
