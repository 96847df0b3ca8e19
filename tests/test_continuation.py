"""p-refinement driver logic against stand-in solvers (no GPU): when it
switches order, when it stops, how it reports a failed state check."""
import types

import pytest

from paper_1208_4772_amd import continuation


class FakeSolver:
    """Residual 10^(-steps/100) at order P (each order starts from 1)."""
    log = []

    def __init__(self, P, fail_at=None):
        self.P = P
        self.steps = 0
        self.fail_at = fail_at
        FakeSolver.log.append(("make", P))

    def state(self, U0):
        return dict(P=self.P)

    def prolong_from(self, other, U, stream=None):
        FakeSolver.log.append(("prolong", other.P, self.P, other.steps))
        return dict(P=self.P)

    def run(self, U, k, stream=None, check=True):
        self.steps += k
        bad = self.fail_at is not None and self.steps >= self.fail_at
        res = 10.0 ** (-self.steps / 100.0)
        return types.SimpleNamespace(status=-4 if bad else 0, t=1e-3 * k, dt_min=1e-3, dt_max=1e-3,
                                     residual=(res, res / 2, res / 3, res / 4))

    def close(self):
        FakeSolver.log.append(("close", self.P))


def test_switches_when_residual_falls_below_threshold():
    FakeSolver.log = []
    r = continuation.run(lambda P: FakeSolver(P), None, (2, 3, 4), check_every=50,
                         switch_residual=1e-2, final_residual=1e-5, max_steps_per_order=10000)
    assert r.converged and r.status == 0
    # residual 10^-(steps/100) <= 1e-2 first at 200 steps; <= 1e-5 at 500
    assert [leg.steps for leg in r.legs] == [200, 200, 500]
    assert [leg.reason for leg in r.legs] == ["switch", "switch", "converged"]
    assert ("prolong", 2, 3, 200) in FakeSolver.log and ("prolong", 3, 4, 200) in FakeSolver.log
    assert ("close", 2) in FakeSolver.log and ("close", 3) in FakeSolver.log
    assert r.steps == 900


def test_per_order_thresholds_and_step_limit():
    r = continuation.run(lambda P: FakeSolver(P), None, (2, 3), check_every=100,
                         switch_residual={2: 1e-1}, final_residual=1e-30, max_steps_per_order=300)
    assert [leg.steps for leg in r.legs] == [100, 300]
    assert r.legs[-1].reason == "step limit" and not r.converged


def test_failed_state_check_stops_the_continuation():
    r = continuation.run(lambda P: FakeSolver(P, fail_at=150 if P == 3 else None), None, (2, 3),
                         check_every=50, switch_residual=1e-2, final_residual=1e-9)
    assert r.status == -4 and not r.converged
    assert r.legs[-1].P == 3 and r.legs[-1].reason == "state check failed"


def test_orders_must_increase():
    with pytest.raises(ValueError):
        continuation.run(lambda P: FakeSolver(P), None, (3, 2))


def test_fixed_iterations_per_order():
    """The paper's way: the lower orders run a fixed number of iterations
    (switch residual 0), the last until the final residual."""
    r = continuation.run(lambda P: FakeSolver(P), None, (2, 3, 4), check_every=100,
                         switch_residual={2: 0.0, 3: 0.0, 4: 0.0}, final_residual=1e-4,
                         max_steps_per_order={2: 300, 3: 200, 4: 10000})
    assert [leg.steps for leg in r.legs] == [300, 200, 400]
    assert [leg.reason for leg in r.legs] == ["step limit", "step limit", "converged"]
    assert r.converged
