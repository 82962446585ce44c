"""FISTA with backtracking on the GPU (ffsat_fista) against the FP64
reference, one iteration at a time from the GPU's own state (so precision
differences do not compound); step-size decisions are compared where the
reference's sufficient-decrease slack exceeds the objective's FP32 error."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_cases import var_scale
from oracle import fista as ofista

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


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("which", ["3sat", "mixed"])
def test_fista_iterations_match_reference(ffs, which):
    if which == "3sat":
        inst = workloads.config1(workloads.instance_seed(1, 0))
        B, eta0 = 64, 0.5
    else:
        inst = workloads.random_hybrid(120, 5, n_or=300, or_len=(2, 6), n_xor=30, xor_len=(2, 9),
                                       n_card=12, card_len=(8, 40))
        B, eta0 = 70, 0.2
    prob = ffs.Problem(inst, device=0)
    plan = ffs.Plan(prob, B)
    x = torch.from_numpy(workloads.points(inst.n_vars, B, 77)).to(DEV)
    st = plan.fista_state(x, eta0)
    st["eta"][::9] = 1e-13                     # stopped restarts stay untouched
    S = var_scale(inst)[:, None]
    fscale = float(np.abs(inst.weights_or_ones()).sum())
    compared = 0
    for it in range(6):
        xs, ys, es, ts = _np(x), _np(st["y"]), _np(st["eta"]), _np(st["t"])
        x_before, y_before = x.clone(), st["y"].clone()
        F = torch.full((B,), float("nan"), device=DEV)
        plan.fista(x, st, 1, max_ls=15, F=F)
        ox, oy, oe, ot, OFy, OFx, trials, margin = ofista.iterate(inst, xs, ys, es, ts)
        ge, gt, gx, gy, gF = _np(st["eta"]), _np(st["t"]), _np(x), _np(st["y"]), _np(F)
        stopped = es < 1e-12
        assert torch.equal(x[:, stopped], x_before[:, stopped]) and torch.equal(st["y"][:, stopped],
                                                                               y_before[:, stopped])
        decided = (~stopped) & (margin > 1e-4 * fscale)
        assert np.array_equal(ge[decided], oe[decided]), (it, ge[decided], oe[decided])
        c = decided
        tol = 2e-5 * np.maximum(1.0, oe[c][None, :] * S)
        assert np.all(np.abs(gx[:, c] - ox[:, c]) <= tol), it
        assert np.all(np.abs(gy[:, c] - oy[:, c]) <= 2 * tol), it
        assert np.allclose(gt[~stopped], ot[~stopped], rtol=1e-6)
        assert np.all(np.abs(gF[c] - OFx[c]) <= 1e-5 * fscale)
        compared += int(c.sum())
    assert compared >= 4 * B                   # most decisions are far from the boundary


def test_solver_with_fista(ffs):
    from paper_2308_15020_amd.solver import solve
    inst, hidden = workloads.planted_hybrid(300, 13, n_or=1000, or_len=(3, 4), n_xor=10, xor_len=(2, 3),
                                            n_card=10, card_len=(5, 20))
    prob = ffs.Problem(inst, device=0)
    res = solve(prob, B=128, rounds=40, T=20, eta=0.5, optimizer="fista", seed=3)
    print("fista", res.solved, res.rounds, res.best_sat, inst.m, f"{res.seconds:.3f}s")
    assert res.solved
    x = np.where(res.assignment, -1.0, 1.0)[:, None]
    assert int(oracle.check(inst, x)["n_sat"][0]) == inst.m
