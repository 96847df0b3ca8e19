"""Batching (continuous batching of independent solves): every result is the
same bits as the same solve run alone, whatever else shares the launches."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu


def dg():
    from paper_1208_4772_amd import dg as _dg
    return _dg


def make(kind, P, scale, precision="fp32", mach=None, av=False):
    r, s = dg().reference_nodes(P)
    case = meshgen.make_case(kind, r, s, scale=scale, P=P, mach=mach,
                             **({"start": "damped"} if kind == "airfoil" else {}))
    case.av = av
    sol = dg().Solver.from_case(case, precision)
    return case, sol


def run_alone(kind, P, scale, steps, precision="fp32", mach=None, av=False):
    case, sol = make(kind, P, scale, precision, mach, av)
    U = sol.state(case.U0)
    st = sol.run(U, steps)
    return U.double().cpu().numpy(), st


def test_batch_results_equal_alone_bitwise():
    """Inviscid and viscous handles of several orders and precisions share
    the launches (viscous ones of one order: one sensor, one gradient and
    one stage launch per stage); a request joins after the first finishes."""
    import torch
    reqs = [("cylinder", 4, 0.02, 7, "fp32", 0.38, False), ("vortex", 2, 1.0, 12, "fp32", None, False),
            ("cylinder", 3, 0.03, 20, "fp32", 0.6, False), ("airfoil", 3, 0.01, 9, "fp32", 0.5, False),
            ("cylinder", 5, 0.01, 11, "fp64", 0.3, False), ("cylinder", 3, 0.02, 6, "bf16x3", 0.45, False),
            ("cylinder", 1, 0.05, 10, "fp32", 0.4, False), ("airfoil", 3, 0.01, 13, "fp32", 0.8, True),
            ("airfoil", 3, 0.015, 8, "fp32", 0.7, True), ("cylinder", 2, 0.03, 12, "fp32", 0.5, True),
            ("airfoil", 4, 0.01, 7, "bf16x3", 0.75, True), ("cylinder", 3, 0.02, 9, "fp64", 0.55, True)]
    late = ("airfoil", 2, 0.02, 8, "fp32", 0.8, True)
    b = dg().Batch(1 << 34, 16)
    live = {}
    for req in reqs:
        kind, P, scale, steps, prec, mach, av = req
        case, sol = make(kind, P, scale, prec, mach, av)
        U = sol.state(case.U0)
        slot = b.admit(sol, U, steps)
        assert slot is not None
        live[slot] = (req, sol, U)
    finished = {}
    admitted_late = False
    while live:
        n = b.advance(5)
        assert n > 0
        for slot in b.poll():
            req, sol, U = live.pop(slot)
            st = b.stats(slot)
            assert st.steps == req[3] and st.status == 0, req
            finished[req] = (U.double().cpu().numpy(), st)
            b.release(slot)
            if not admitted_late:
                kind2, P2, sc2, st2, pr2, m2, av2 = late
                case, sol2 = make(kind2, P2, sc2, pr2, m2, av2)
                U2 = sol2.state(case.U0)
                s2 = b.admit(sol2, U2, st2)
                live[s2] = (late, sol2, U2)
                admitted_late = True
    torch.cuda.synchronize()
    assert len(finished) == len(reqs) + 1
    for req, (Ub, stb) in finished.items():
        Ua, sta = run_alone(*req)
        assert np.array_equal(Ua, Ub), (req, np.abs(Ua - Ub).max())
        assert sta.t == stb.t and sta.dt_min == stb.dt_min, req


def test_admission_by_footprint():
    case, s1 = make("cylinder", 4, 0.02)
    _, s2 = make("cylinder", 4, 0.02)
    f1, f2 = s1.footprint(), s2.footprint()
    assert f1 > 0
    assert dg().estimate_footprint(case.K, 4) >= f1
    b = dg().Batch(f1 + f2 // 2, 4)
    U1 = s1.state(case.U0)
    U2 = s2.state(case.U0)
    a = b.admit(s1, U1, 3)
    assert a is not None
    assert b.admit(s2, U2, 3) is None          # over budget: stays queued
    while b.advance(10):
        pass
    assert b.poll() == [a]
    b.release(a)
    c = b.admit(s2, U2, 3)                      # room again
    assert c is not None
    slots = dg().Batch(1 << 34, 1)
    assert slots.admit(s1, U1, 2) is not None
    assert slots.admit(s2, U2, 2) is None       # no free slot


def test_joins_and_leaves_of_known_kinds_do_not_recapture():
    """The batched launches read their work lists' lengths from device
    memory: once the kinds of solve (order, precision, viscosity) present
    have been captured, solves joining and leaving reuse the graph; a new
    kind captures once more.  Results stay those of the solves alone."""
    import torch
    b = dg().Batch(1 << 34, 8)
    kinds = [("cylinder", 3, 0.02, "fp32", 0.4, False), ("airfoil", 2, 0.01, "fp32", 0.6, True)]
    live = {}

    def admit(kind, P, scale, prec, mach, av, steps):
        case, sol = make(kind, P, scale, prec, mach, av)
        U = sol.state(case.U0)
        slot = b.admit(sol, U, steps)
        assert slot is not None
        live[slot] = ((kind, P, scale, steps, prec, mach, av), sol, U)

    for k in kinds:
        admit(*k, 6)
    results = []
    captures = []
    for round_ in range(4):
        while live:
            b.advance(4)
            for slot in b.poll():
                req, sol, U = live.pop(slot)
                results.append((req, U.double().cpu().numpy()))
                b.release(slot)
            captures.append(b.info()[0])
        # the same kinds again, other sizes and step counts
        for k in kinds:
            kind, P, scale, prec, mach, av = k
            admit(kind, P, scale * (1.2 + 0.3 * round_), prec, mach, av, 6 + 2 * round_)
    while live:
        b.advance(4)
        for slot in b.poll():
            req, sol, U = live.pop(slot)
            results.append((req, U.double().cpu().numpy()))
            b.release(slot)
    torch.cuda.synchronize()
    ncap, ngroups = b.info()
    assert ngroups == 2
    assert ncap == 1, captures
    # a new kind (another order) captures once more
    admit("cylinder", 4, 0.02, "fp32", 0.4, False, 4)
    while live:
        b.advance(4)
        for slot in b.poll():
            req, sol, U = live.pop(slot)
            results.append((req, U.double().cpu().numpy()))
            b.release(slot)
    assert b.info() == (2, 3)
    for req, Ub in results:
        Ua, _ = run_alone(*req)
        assert np.array_equal(Ua, Ub), req


def test_reused_slot_with_fp64_handles_matches_alone():
    """FP64 handles step one by one inside the batch's captured graph, whose
    launches carry their handles' tables and buffers.  A solve finishes, its
    handle is closed, and new solves take the same slot (one slot only; the
    third has the second's shape, so the allocators may hand out the same
    addresses again): each needs its own graph, and each result equals the
    same solve run alone."""
    import torch
    reqs = [("cylinder", 3, 0.02, 6, "fp64", 0.4, True), ("airfoil", 2, 0.01, 7, "fp64", 0.7, True),
            ("airfoil", 2, 0.01, 5, "fp64", 0.6, True)]
    b = dg().Batch(1 << 34, 1)
    for n, req in enumerate(reqs):
        kind, P, scale, steps, prec, mach, av = req
        print(f"[reuse fp64] request {n}: {req}", flush=True)
        case, sol = make(kind, P, scale, prec, mach, av)
        U = sol.state(case.U0)
        assert b.admit(sol, U, steps) == 0
        done = []
        while not done:
            assert b.advance(4) > 0
            done = b.poll()
        assert done == [0]
        st = b.stats(0)
        assert st.steps == steps and st.status == 0
        torch.cuda.synchronize()
        Ub = U.double().cpu().numpy()
        b.release(0)
        sol.close()
        del U
        Ua, sta = run_alone(*req)
        assert np.array_equal(Ua, Ub), (req, np.abs(Ua - Ub).max())
        assert sta.t == st.t
        captures, _ = b.info()
        assert captures == n + 1
