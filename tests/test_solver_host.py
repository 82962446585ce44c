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
