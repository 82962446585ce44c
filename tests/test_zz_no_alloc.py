"""ffsat_eval_noalloc (the objective and gradient with no plan and no device
allocation, its slots in the library's fixed device array) against
ffsat_eval, through the C ABI (needs an MI355X).

Two calls in a row, the second with fewer restarts, so that the second
reuses the array the first filled; and a call too large for the array,
rejected before any launch."""
import ctypes as C

import numpy as np
import pytest

import workloads
from gpu_cases import TOL32, every_bin_instance, points, var_scale

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


def _noalloc(ffs, prob, x, B):
    from paper_2308_15020_amd._lib import check, lib
    F = torch.full((B,), float("nan"), device=DEV)
    g = torch.full((prob.n, B), float("nan"), device=DEV)
    s = torch.cuda.current_stream().cuda_stream
    check(lib().ffsat_eval_noalloc(prob.handle, B, C.c_void_p(x.data_ptr()), C.c_void_p(F.data_ptr()),
                                   C.c_void_p(g.data_ptr()), C.c_void_p(s)))
    return F, g


def test_noalloc_matches_eval_two_calls(ffs):
    inst = every_bin_instance()
    prob = ffs.Problem(inst, device=0)
    S = var_scale(inst)[:, None]
    wsum = float(np.abs(inst.weights).sum())
    for B, seed in ((130, 5), (37, 6)):   # the second call is smaller
        x = torch.from_numpy(np.ascontiguousarray(points(inst, B, seed, "mixed_edge"))).to(DEV)
        F, g = _noalloc(ffs, prob, x, B)
        ref = ffs.Plan(prob, B, pull="off").eval(x)
        torch.cuda.synchronize()
        dF = np.max(np.abs(F.cpu().numpy() - ref["F"].cpu().numpy())) / wsum
        dg = np.max(np.abs(g.cpu().numpy() - ref["grad"].cpu().numpy()) / S)
        assert dF <= TOL32 and dg <= TOL32, (B, dF, dg)


def test_noalloc_rejects_too_large(ffs):
    from paper_2308_15020_amd._lib import lib
    inst = workloads.config3a(workloads.instance_seed(3, 0))   # nnz * 256 * 4 bytes = 1.29 GB
    prob = ffs.Problem(inst, device=0)
    B = 256
    x = torch.zeros(inst.n_vars, B, device=DEV)
    F = torch.empty(B, device=DEV)
    st = lib().ffsat_eval_noalloc(prob.handle, B, C.c_void_p(x.data_ptr()), C.c_void_p(F.data_ptr()), None,
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st != 0 and b"scratch" in lib().ffsat_last_error()
