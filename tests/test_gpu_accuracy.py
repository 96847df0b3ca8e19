"""Reduced-precision results against the FP64 oracle at stated times: state
L2 and maximum error, entropy error, wall loads (lift, drag) on small
versions of the cylinder and transonic airfoil cases."""
import numpy as np
import pytest

import meshgen
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

# FP32: the run bound of the parity tests; BF16x3: its split-product bound
STATE_TOL = {"fp32": 2e-5, "bf16x3": 3 * 2.0 ** -16 * 110}
# loads: the state bound times the O(1) sensitivity of a pressure
# coefficient to a relative state change at these Mach numbers (p / q_dyn
# = 1 / (0.7 M^2) <= 10), with room for the integral
LOAD_TOL = {"fp32": 1e-3, "bf16x3": 5e-2}


def run_case(kind, P, scale, stations, precisions):
    import torch
    from paper_1208_4772_amd import accuracy, dg
    r, s = dg.reference_nodes(P)
    case = meshgen.make_case(kind, r, s, scale=scale, P=P)
    geo = accuracy.Geometry(case)
    o = orc.Oracle.for_case(case)
    results = {p: accuracy.run_stations(case, p, stations) for p in precisions}
    U, done = case.U0.copy(), 0
    rows = []
    for i, n in enumerate(stations):
        U, info = o.run(U, n - done)
        done = n
        ref_loads = geo.wall_loads(U, case.freestream)
        ref_s = geo.entropy_error(U, case.freestream)
        for p in precisions:
            rr = results[p][i]
            assert rr["status"] == 0, (p, n)
            e = accuracy.state_errors(rr["U"], U)
            loads = geo.wall_loads(rr["U"], case.freestream)
            rows.append((p, n, e, geo.entropy_error(rr["U"], case.freestream), ref_s, loads, ref_loads))
    torch.cuda.synchronize()
    return case, rows


@pytest.mark.parametrize("kind,P,scale,stations", [
    ("cylinder", 4, 0.05, (50, 100, 200)),
    ("airfoil", 3, 0.02, (40, 80, 160)),
])
def test_reduced_precision_against_oracle_at_stated_times(kind, P, scale, stations):
    case, rows = run_case(kind, P, scale, stations, ("fp32", "bf16x3"))
    for p, n, e, s_err, s_ref, loads, ref in rows:
        print(f"[{kind} K={case.K} P={P} {p} step {n}] state rel L2 {e['rel_l2']:.2e} max {e['max_abs']:.2e}; "
              f"entropy error {s_err:.4e} (oracle {s_ref:.4e}); CL {loads['CL']:.6f} (oracle {ref['CL']:.6f}) "
              f"CD {loads['CD']:.6f} (oracle {ref['CD']:.6f})")
        assert e["rel_l2"] <= STATE_TOL[p]
        # s = p / rho^gamma moves by at most (1 + gamma) times the relative
        # state change per node, with room for the RMS
        assert abs(s_err - s_ref) <= 10 * STATE_TOL[p]
        assert abs(loads["CL"] - ref["CL"]) <= LOAD_TOL[p]
        assert abs(loads["CD"] - ref["CD"]) <= LOAD_TOL[p]
