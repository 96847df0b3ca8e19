"""p-refinement continuation to a steady state with residual monitoring.

The paper's p-refinement (Section 5, the p-refinement paragraph, and the
table of p-refinement runs): start at a low order, iterate until the flow has
settled at that order, prolong the state to the next order by padding its
hierarchical modal coefficients with zeros, and continue; the residual
infinity norm ||dU/dt||_inf is checked only every `check_every` steps
because a norm is a global reduction.

Every step, residual and prolongation runs in the library (dg_run, whose
statistics carry the residual of the final state, and dg_prolong); this
module only decides when to switch.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

from . import dg


@dataclass
class OrderLeg:
    P: int
    steps: int = 0
    t: float = 0.0
    wall_s: float = 0.0
    residuals: list = field(default_factory=list)   # (steps at this order, max over fields)
    dt_min: float = math.inf
    dt_max: float = 0.0
    reason: str = ""


@dataclass
class ContinuationResult:
    legs: list
    state: object          # final device state (torch tensor) of the last order
    solver: object         # the last order's solver (caller closes it)
    converged: bool
    status: int = 0

    @property
    def steps(self):
        return sum(leg.steps for leg in self.legs)

    @property
    def wall_s(self):
        return sum(leg.wall_s for leg in self.legs)

    def summary(self):
        return dict(converged=self.converged, status=self.status, steps=self.steps,
                    wall_s=self.wall_s,
                    legs=[dict(P=leg.P, steps=leg.steps, t=leg.t, wall_s=leg.wall_s,
                               dt_min=leg.dt_min, dt_max=leg.dt_max, reason=leg.reason,
                               residual_first=leg.residuals[0][1] if leg.residuals else None,
                               residual_last=leg.residuals[-1][1] if leg.residuals else None)
                          for leg in self.legs])


def run(make_solver, U0, orders, check_every=1000, switch_residual=1e-4, final_residual=1e-9,
        max_steps_per_order=100000, stream=None):
    """Continuation over `orders` (increasing).

    make_solver(P) -> dg.Solver for the mesh at order P (all the same
    elements and precision).  U0: host (K, 4, Np) start state at orders[0].
    At each order the solve runs `check_every` steps at a time and reads the
    residual of the state it reached; it moves to the next order once the
    residual is at most `switch_residual` (a float, or a dict per order),
    and stops at the last order once it is at most `final_residual`, or at
    any order after `max_steps_per_order` steps (an int, or a dict per
    order: the paper fixes the iterations of its lower orders by hand, with
    a switch residual of 0 that is the same).  A state check failure
    (non-finite state, rho <= 0 or p <= 0) stops the continuation with
    status DG_ENONFINITE."""
    orders = list(orders)
    if not orders or any(b <= a for a, b in zip(orders, orders[1:])):
        raise ValueError("orders must be a non-empty increasing sequence")
    legs = []
    solver = make_solver(orders[0])
    U = solver.state(U0)
    converged = False
    status = 0
    for n, P in enumerate(orders):
        if n > 0:
            nxt = make_solver(P)
            U = nxt.prolong_from(solver, U, stream=stream)
            solver.close()
            solver = nxt
        last = n == len(orders) - 1
        target = final_residual if last else (switch_residual[P] if isinstance(switch_residual, dict)
                                              else switch_residual)
        leg = OrderLeg(P)
        legs.append(leg)
        limit = max_steps_per_order[P] if isinstance(max_steps_per_order, dict) else max_steps_per_order
        while leg.steps < limit:
            k = min(check_every, limit - leg.steps)
            t0 = time.perf_counter()
            st = solver.run(U, k, stream=stream, check=False)
            leg.wall_s += time.perf_counter() - t0
            leg.steps += k
            leg.t += st.t
            leg.dt_min = min(leg.dt_min, st.dt_min)
            leg.dt_max = max(leg.dt_max, st.dt_max)
            res = max(abs(r) for r in st.residual)
            leg.residuals.append((leg.steps, res))
            if st.status != 0 or not math.isfinite(res):
                status = st.status or dg.DG_ENONFINITE
                leg.reason = "state check failed"
                return ContinuationResult(legs, U, solver, False, status)
            if res <= target:
                leg.reason = "converged" if last else "switch"
                break
        else:
            leg.reason = "step limit"
        if last and leg.reason == "converged":
            converged = True
    return ContinuationResult(legs, U, solver, converged, status)


def main(argv=None):
    """The cylinder case (M = 0.38) driven to a steady state with and without
    p-refinement: steps, time and residuals per order, as the paper's
    p-refinement table reports them."""
    import argparse
    import json

    import meshgen
    ap = argparse.ArgumentParser(description=main.__doc__.split("\n")[0])
    ap.add_argument("--scale", type=float, default=0.25, help="element-count scale of the 20,000-element cylinder")
    ap.add_argument("--orders", default="2,3,4")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--check-every", type=int, default=1000)
    ap.add_argument("--switch-residual", type=float, default=1e-4)
    ap.add_argument("--final-residual", type=float, default=1e-9)
    ap.add_argument("--max-steps", type=int, default=100000)
    ap.add_argument("--steps-per-order", default=None,
                    help="fixed iterations of the lower orders, e.g. 2:40000,3:40000 (no residual switch there)")
    ap.add_argument("--mach", type=float, default=0.38)
    ap.add_argument("--form", default="nodal", choices=["nodal", "weak"])
    ap.add_argument("--start", default="potential", choices=["potential", "freestream", "damped"])
    a = ap.parse_args(argv)
    orders = [int(p) for p in a.orders.split(",")]

    def case_at(P):
        r, s = dg.reference_nodes(P)
        return meshgen.make_case("cylinder", r, s, scale=a.scale, P=P, mach=a.mach, start=a.start)

    def make_solver(P):
        return dg.Solver.from_case(case_at(P), a.precision, form=a.form)

    switch, limits = a.switch_residual, a.max_steps
    if a.steps_per_order:
        fixed = {int(k): int(v) for k, v in (kv.split(":") for kv in a.steps_per_order.split(","))}
        switch = {P: 0.0 for P in orders}
        limits = {P: fixed.get(P, a.max_steps) for P in orders}
    out = {}
    for label, ords in (("p_refinement", orders), ("single_order", orders[-1:])):
        c0 = case_at(ords[0])
        res = run(make_solver, c0.U0, ords, a.check_every, switch, a.final_residual, limits)
        res.solver.close()
        out[label] = res.summary()
        print(json.dumps({label: out[label]}), flush=True)
    out["K"] = case_at(orders[0]).K
    out["form"] = a.form
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
