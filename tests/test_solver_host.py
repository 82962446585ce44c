"""Host-side argument checks of the search loop (no GPU: they fail before
any plan is made)."""
import pytest

pytest.importorskip("torch")


def test_search_rejects_bad_policy_and_optimizer():
    from paper_2308_15020_amd.solver import Search
    with pytest.raises(ValueError):
        Search(None, 4, policy="ROX")
    with pytest.raises(ValueError):
        Search(None, 4, policy="")
    with pytest.raises(ValueError):
        Search(None, 4, optimizer="adam")


def test_portfolio_needs_one_problem_per_arm():
    from paper_2308_15020_amd.solver import Arm, solve_portfolio
    with pytest.raises(ValueError):
        solve_portfolio(None, [Arm(8), Arm(8)], problems=[object()])


def test_portfolio_rejects_a_shared_problem():
    from paper_2308_15020_amd.solver import Arm, solve_portfolio
    shared = object()
    with pytest.raises(ValueError):
        solve_portfolio(None, [Arm(8), Arm(8)], problems=[shared, shared])


class _FakeProblem:
    """Stands in for a Problem on the CPU: records weight reads and writes."""

    def __init__(self, n, m):
        import torch
        self.n, self.m, self.device = n, m, torch.device("cpu")
        self.w = torch.ones(m)

    def set_weights(self, w):
        import torch
        self.w = torch.as_tensor(w, dtype=torch.float32).clone()

    def get_weights(self):
        return self.w


class _FakePlan:
    """Records the rephase calls Search.adapt makes (no kernels run)."""

    def __init__(self):
        self.calls = []

    def rephase(self, x, mode, seed=0, mask=None):
        self.calls.append(("rephase", mode))
        if mode == 1:
            x.neg_()

    def erwa_update(self, U, alpha):
        self.calls.append(("erwa", float(alpha)))


def test_random_phase_hook_replaces_only_random_phases():
    """With a random-phase hook, the phases 'R' of the policy take the hook's
    points and 'O' / 'F' still go to the library (original: keep, flipped:
    negate); without a hook every phase goes to the library."""
    import torch
    from paper_2308_15020_amd.solver import Search
    n, B = 5, 4
    prob, plan = _FakeProblem(n, 3), _FakePlan()
    drawn = []

    def hook(r):
        drawn.append(r)
        return torch.full((n, B), 0.25 + r)

    x0 = torch.linspace(-1, 1, n * B).reshape(n, B)
    S = Search(prob, B, policy="ROF", x0=x0, plan=plan, weighting=False, random_phase=hook)
    plan.calls.clear()
    S.adapt(0)                         # 'R': the hook
    assert drawn == [0] and torch.all(S.x == 0.25) and plan.calls == []
    S.adapt(1)                         # 'O': the library keeps x
    assert drawn == [0] and plan.calls == [("rephase", 0)] and torch.all(S.x == 0.25)
    S.adapt(2)                         # 'F': the library flips x
    assert drawn == [0] and plan.calls[-1] == ("rephase", 1) and torch.all(S.x == -0.25)
    S.adapt(3)                         # 'R' again
    assert drawn == [0, 3] and torch.all(S.x == 3.25)

    plan2 = _FakePlan()
    S2 = Search(prob, B, policy="R", x0=x0, plan=plan2, weighting=False)
    plan2.calls.clear()
    S2.adapt(0)
    assert plan2.calls == [("rephase", 2)]


def test_search_keeps_its_iterate_buffer():
    """x_buf holds the iterate (the library keys captured graphs by buffer)."""
    import torch
    from paper_2308_15020_amd.solver import Search
    n, B = 3, 2
    buf = torch.zeros(n, B)
    x0 = torch.ones(n, B) * 0.5
    S = Search(_FakeProblem(n, 2), B, policy="O", x0=x0, plan=_FakePlan(), weighting=False, x_buf=buf)
    assert S.x.data_ptr() == buf.data_ptr() and torch.all(buf == 0.5)
