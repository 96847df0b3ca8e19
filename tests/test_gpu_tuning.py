"""The tuning table on the device: dg_autotune records its choice per kind
of handle, later handles and batch groups take it, and results do not depend
on the workgroup shape."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu


def dg():
    from paper_1208_4772_amd import dg as _dg
    return _dg


@pytest.fixture(autouse=True)
def empty_table():
    dg().Tuning.clear()
    yield
    dg().Tuning.clear()


def make(kind, P, scale, precision="fp32", mach=None, av=False):
    r, s = dg().reference_nodes(P)
    case = meshgen.make_case(kind, r, s, scale=scale, P=P, mach=mach,
                             **({"start": "damped"} if kind == "airfoil" else {}))
    case.av = av
    return case, dg().Solver.from_case(case, precision)


def test_autotune_records_and_later_handles_reuse_it():
    import torch
    T = dg().Tuning
    arch = T.device_arch()
    assert arch.startswith("gfx")
    case, s1 = make("cylinder", 4, 0.05)
    w, us = s1.autotune(s1.state(case.U0))
    print(f"[tuning] {arch} P=4 fp32 inviscid -> {w} waves, {us:.1f} us", flush=True)
    assert w in (2, 4, 8) and us > 0
    assert T.lookup(arch, 4, "fp32", False) == w
    assert T.lookup(arch, 4, "fp32", True) == 0
    # a second handle of the same kind takes the entry without timing
    c2, s2 = make("cylinder", 4, 0.02, mach=0.5)
    assert s2.autotune(s2.state(c2.U0)) == (w, 0.0)
    # viscous handles are tuned too (the stage kernel with the viscous terms);
    # the rhs and a run are the same bits before and after
    ca, sa = make("airfoil", 3, 0.01, mach=0.8, av=True)
    U = sa.state(ca.U0)
    r0 = sa.rhs(U).clone()
    U0 = U.clone()
    sa.run(U0, 5)
    wa, usa = sa.autotune(U)
    print(f"[tuning] P=3 fp32 viscous -> {wa} waves, {usa:.1f} us", flush=True)
    assert wa in (2, 4, 8) and usa > 0
    assert T.lookup(arch, 3, "fp32", True) == wa
    r1 = sa.rhs(U)
    U1 = U.clone()
    sa.run(U1, 5)
    torch.cuda.synchronize()
    assert torch.equal(r0, r1) and torch.equal(U0, U1)


@pytest.mark.parametrize("waves", [2, 8])
def test_batch_groups_take_the_tuned_shape_bitwise(waves):
    """Every kind in the mix is set to `waves` wavefronts per workgroup; the
    batch results equal the same solves run alone with the default shape."""
    import torch
    T = dg().Tuning
    arch = T.device_arch()
    reqs = [("cylinder", 3, 0.03, 9, "fp32", 0.5, False), ("airfoil", 3, 0.01, 7, "fp32", 0.8, True),
            ("cylinder", 4, 0.02, 8, "bf16x3", 0.4, False), ("cylinder", 2, 0.03, 6, "fp32", 0.6, True),
            ("cylinder", 5, 0.01, 5, "fp32", 0.38, False)]
    alone = {}
    for req in reqs:
        kind, P, scale, steps, prec, mach, av = req
        case, sol = make(kind, P, scale, prec, mach, av)
        U = sol.state(case.U0)
        st = sol.run(U, steps)
        alone[req] = (U.double().cpu().numpy(), st.t)
    for req in reqs:
        T.set(arch, req[1], req[4], req[6], waves)
    b = dg().Batch(1 << 34, 8)
    live = {}
    for req in reqs:
        kind, P, scale, steps, prec, mach, av = req
        case, sol = make(kind, P, scale, prec, mach, av)
        U = sol.state(case.U0)
        live[b.admit(sol, U, steps)] = (req, sol, U)
    done = {}
    while live:
        assert b.advance(4) > 0
        for slot in b.poll():
            req, sol, U = live.pop(slot)
            st = b.stats(slot)
            assert st.steps == req[3] and st.status == 0, req
            done[req] = (U.double().cpu().numpy(), st.t)
            b.release(slot)
    torch.cuda.synchronize()
    for req in reqs:
        Ua, ta = alone[req]
        Ub, tb = done[req]
        print(f"[tuning batch W={waves}] {req} max diff {np.abs(Ua - Ub).max():.3e}", flush=True)
        assert np.array_equal(Ua, Ub) and ta == tb, req
