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
    for r in reqs[:3]:
        sol = dg.Solver.from_case(r.case, "fp32")
        U = sol.state(r.case.U0)
        st = sol.run(U, r.steps)
        torch.cuda.synchronize()
        assert st.status == 0 and st.t == r.t_sim
        assert np.array_equal(U.double().cpu().numpy(), r.final_state), r.rid
