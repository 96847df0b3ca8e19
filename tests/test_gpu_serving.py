"""Serving loop on the GPU: every request finishes, and a request's result
is the same bits as the solve run alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_server_runs_mix_and_matches_alone():
    import torch
    from paper_1208_4772_amd import dg, serving
    reqs = serving.make_requests(8, mean_gap=0.005, seed=7, K_range=(800, 3000),
                                 steps_range=(10, 40))
    biggest = max(dg.estimate_footprint(r.case.K, r.P, "fp32", r.av) for r in reqs)
    srv = serving.Server(hbm_budget_bytes=3 * biggest, max_slots=4, chunk_steps=7, keep_states=True)
    rep = srv.run(reqs)
    s = rep.summary()
    assert s["failed"] == 0 and s["n_requests"] == 8, [(r.rid, r.status) for r in reqs]
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
    assert 1 <= rep.peak_slots <= 4
    # the step graph is captured again only when a new kind of solve
    # (order; all requests here are FP32 and viscous) joins, not at every
    # admission or release
    kinds = len({r.P for r in reqs})
    assert s["solve_kinds"] == kinds and s["graph_captures"] <= kinds, s
    for r in reqs[:3]:
        sol = dg.Solver.from_case(r.case, "fp32")
        U = sol.state(r.case.U0)
        st = sol.run(U, r.steps)
        torch.cuda.synchronize()
        assert st.status == 0 and st.t == r.t_sim
        assert np.array_equal(U.double().cpu().numpy(), r.final_state), r.rid


def test_server_results_match_oracle_subset():
    """Eight seeded requests of the mix (small meshes, few steps) through the
    server, each final state against the FP64 oracle run of the same case.
    FP32 bars: the run tolerance of the parity tests on the state; on the
    change from the start, that bound widened by the FP32 change of the
    sensor's log10 S (about 1e-6 relative) times the ramp slope and by the
    small size of a few steps' change against the state."""
    import torch
    from oracle import oracle as orc
    from paper_1208_4772_amd import dg, serving
    reqs = serving.make_requests(8, mean_gap=0.002, seed=11, K_range=(600, 1500),
                                 steps_range=(8, 16))
    biggest = max(dg.estimate_footprint(r.case.K, r.P, "fp32", r.av) for r in reqs)
    srv = serving.Server(hbm_budget_bytes=4 * biggest, max_slots=4, chunk_steps=5, keep_states=True)
    srv.run(reqs)
    torch.cuda.synchronize()
    for r in reqs:
        assert r.status == 0, (r.rid, r.status)
        o = orc.Oracle.for_case(r.case)
        # both sides start from the FP32 state the server was handed (the
        # rounding of a non-uniform start is otherwise a large part of a
        # few steps' change)
        U0 = r.case.U0.astype(np.float32).astype(np.float64)
        Ur, info = o.run(U0, r.steps)
        # the state against the FP32 run bar of the parity tests, and the
        # change from the start (the states are dominated by the freestream,
        # and a potential-flow start changes little in a few steps, so that
        # FP32 rounding of the nearly cancelling rhs weighs more there)
        err_state = float(np.linalg.norm((r.final_state - Ur).ravel()) / np.linalg.norm(Ur.ravel()))
        dU = r.final_state - U0
        err = float(np.linalg.norm((dU - (Ur - U0)).ravel()) / np.linalg.norm((Ur - U0).ravel()))
        print(f"[serving vs oracle] req {r.rid} {r.kind} K={r.case.K} P={r.P} M={r.mach:.2f} "
              f"steps={r.steps}: rel L2 of the state {err_state:.2e}, of the update {err:.2e}, "
              f"t {r.t_sim:.6g} vs {info['t']:.6g}")
        assert err_state <= 2e-5, (r.rid, err_state)
        assert err <= 1e-3, (r.rid, err)
        assert abs(r.t_sim - info["t"]) <= 1e-5 * info["t"]
