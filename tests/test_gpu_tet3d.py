"""GPU parity of the 3D tetrahedral path (include/dg3.h) against the FP64
CPU oracle on the same seeded inputs: the rhs and short runs, FP64 and FP32,
periodic and walled cubes, P = 1..4, the full benchmark mesh, the automatic
time step and the error path.

Bars as in 2D: FP64 within 1e-12 relative L2 of the oracle, or twice the
oracle's own spread over valid evaluation orders where that is larger (the
benchmark mesh: spread 6.5e-13); FP32 within
max(2e-5, u kappa), u = 2^-24 and kappa the cancellation of the flux
derivatives in the rhs (rhs_condition3: about 700 on the small periodic
P = 4 mesh, 3900 on the benchmark mesh, where h = 1/16 makes the metric
terms large; measured errors 0.16-0.18 u kappa)."""
import numpy as np
import pytest

from meshgen.tets import affine_node_coordinates, cube_tets, entropy_wave3, smooth_state3
from oracle import tet3d as T

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5}


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def setup(N, P, precision, periodic=True, jitter=0.15, seed=3, cfl=0.5):
    from paper_1208_4772_amd import dg3
    g = cube_tets(N, 1.0, jitter, seed, periodic=periodic)
    o = T.Oracle3D(T.TetMesh(g.EToV, g.X, g.period), P, cfl=cfl)
    s = dg3.Solver3D.from_mesh(g, P, precision=precision, cfl=cfl)
    r, st, t = dg3.reference_nodes3(P)
    xyz = affine_node_coordinates(g, r, st, t)
    return g, o, s, xyz


def rhs_condition3(o, U, rhs):
    """kappa = || sum over (a, d) of |d r_a / d x_d| |D_a| |F_d| || / ||rhs||:
    how much the volume term's flux derivatives cancel in the rhs (a
    rounding error u per operation moves the rhs by about u kappa)."""
    F = T.fluxes(U, o.g)
    D = (np.abs(o.R.Dr), np.abs(o.R.Ds), np.abs(o.R.Dt))
    acc = np.zeros_like(U)
    for a in range(3):
        for d in range(3):
            acc += np.abs(o.geo.drdx[:, a, d])[:, None, None] * np.einsum("ij,kcj->kci", D[a], np.abs(F[d]))
    return float(np.linalg.norm(acc) / np.linalg.norm(rhs))


def oracle_spread3(o, U):
    """Largest relative L2 difference between valid FP64 evaluations of the
    oracle's rhs: as built, with Dr, Ds, Dt re-rounded to exact zero row
    sums, and with the volume term contracted in the contravariant order
    (metric terms times fluxes first, then the derivative matrices)."""
    import copy
    base = o.rhs(U)
    o2 = copy.copy(o)
    R = T.RefTet(o.P)
    for D in (R.Dr, R.Ds, R.Dt):
        n = D.shape[0]
        D[np.arange(n), np.arange(n)] = 0.0
        D[np.arange(n), np.arange(n)] = -D.sum(1)
    o2.R = R
    F, a = T.fluxes(U, o.g), o.geo.drdx
    vol_o, vol_c = np.zeros_like(U), np.zeros_like(U)
    for D, row in ((o.R.Dr, 0), (o.R.Ds, 1), (o.R.Dt, 2)):
        for col in range(3):
            vol_o -= a[:, row, col][:, None, None] * np.einsum("ij,kcj->kci", D, F[col])
        vol_c -= np.einsum("ij,kcj->kci", D, sum(a[:, row, d][:, None, None] * F[d] for d in range(3)))
    rs = [base, o2.rhs(U), base - vol_o + vol_c]
    return max(rel_l2(x, y) for i, x in enumerate(rs) for y in rs[:i])


def rhs_tol(precision, o, U, rhs):
    if precision == "fp64":
        # as in 2D: where the rhs is ill-conditioned the bar is twice the
        # oracle's own spread, never below 1e-12
        spread = oracle_spread3(o, U)
        print(f"oracle spread {spread:.3e}")
        return max(TOL["fp64"], 2.0 * spread)
    kappa = rhs_condition3(o, U, rhs)
    print(f"kappa {kappa:.1f}")
    return max(TOL["fp32"], 2.0 ** -24 * kappa)


def host(U):
    return U.double().cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_rhs_periodic(P, precision):
    print(f"[tet3d rhs periodic P={P} {precision}]", flush=True)
    g, o, s, xyz = setup(3, P, precision)
    np.testing.assert_allclose(np.stack(xyz), np.stack(o.xyz), atol=1e-15)
    U0 = smooth_state3(xyz, seed=P)
    ref = o.rhs(U0)
    got = host(s.rhs(s.state(U0)))
    e = rel_l2(got, ref)
    print(f"rel L2 {e:.3e}")
    assert e < rhs_tol(precision, o, U0, ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("P", [2, 4])
def test_rhs_walled_box(P, precision):
    print(f"[tet3d rhs walls P={P} {precision}]", flush=True)
    g, o, s, xyz = setup(3, P, precision, periodic=False, jitter=0.1, seed=7)
    assert (g.bc == 1).any()
    U0 = smooth_state3(xyz, seed=10 + P)
    ref = o.rhs(U0)
    got = host(s.rhs(s.state(U0)))
    e = rel_l2(got, ref)
    print(f"rel L2 {e:.3e}")
    assert e < rhs_tol(precision, o, U0, ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_freestream_and_rest_state(precision):
    print(f"[tet3d freestream {precision}]", flush=True)
    for periodic, vel in ((True, (0.4, -0.3, 0.2)), (False, (0.0, 0.0, 0.0))):
        g, o, s, xyz = setup(3, 3, precision, periodic=periodic)
        one = np.ones_like(xyz[0])
        U0 = T.primitive_to_conserved(1.3 * one, vel[0] * one, vel[1] * one, vel[2] * one, 0.9 * one)
        got = host(s.rhs(s.state(U0)))
        # FP32: the rows of Dr, Ds, Dt sum to zero only up to rounding:
        # |row| ~ 15, flux ~ 1.3, metric ~ 6 per term, three terms, 2^-24
        # gives about 2e-5 at worst
        assert np.abs(got).max() < (1e-12 if precision == "fp64" else 1e-4), np.abs(got).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("P", [1, 3])
def test_run_fixed_and_automatic_step(P, precision):
    """Three LSERK steps at the automatic (CFL) step and three at a fixed
    step, against the oracle's run; the automatic step equals the oracle's
    FP64 bound."""
    print(f"[tet3d run P={P} {precision}]", flush=True)
    g, o, s, xyz = setup(3, P, precision, periodic=False, jitter=0.1, seed=11)
    U0 = smooth_state3(xyz, seed=5)
    dt0 = o.dt(U0)
    Uref, dts = U0, []
    for _ in range(3):
        dts.append(o.dt(Uref))
        Uref, _ = o.run(Uref, 1, dt=dts[-1])
    t = sum(dts)
    U = s.state(U0)
    st = s.run(U, 3)
    assert st.steps == 3 and st.status == 0
    rtol = 1e-13 if precision == "fp64" else 1e-5
    assert abs(st.dt_max - max(dts)) <= rtol * dt0 and abs(st.dt_min - min(dts)) <= rtol * dt0
    assert abs(st.t - t) <= rtol * t
    e = rel_l2(host(U), Uref)
    print(f"auto-step rel L2 {e:.3e} dt {st.dt_min:.6e}..{st.dt_max:.6e} (oracle {min(dts):.6e}..{max(dts):.6e})")
    assert e < TOL[precision]
    Uref2, _ = o.run(Uref, 3, dt=0.5 * dt0)
    st2 = s.run(U, 3, dt=0.5 * dt0)
    assert st2.dt_min == st2.dt_max == 0.5 * dt0
    e2 = rel_l2(host(U), Uref2)
    print(f"fixed-step rel L2 {e2:.3e}")
    assert e2 < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_benchmark_mesh_rhs_and_step(precision):
    """The benchmark's workload (16 x 16 x 17 cubes, 26,112 tetrahedra,
    P = 4, the entropy wave along x): the full rhs and one step against the
    oracle."""
    print(f"[tet3d 26112 tets P=4 {precision}]", flush=True)
    g, o, s, xyz = setup((16, 16, 17), 4, precision, jitter=0.1, seed=3)
    assert g.K == 26112
    U0 = entropy_wave3(xyz, along=(1, 0, 0))
    ref = o.rhs(U0)
    e = rel_l2(host(s.rhs(s.state(U0))), ref)
    print(f"rhs rel L2 {e:.3e}")
    assert e < rhs_tol(precision, o, U0, ref)
    U = s.state(U0)
    st = s.run(U, 1)
    Uref, t = o.run(U0, 1)
    e1 = rel_l2(host(U), Uref)
    print(f"one step rel L2 {e1:.3e}, dt {st.dt_max:.4e} vs {t:.4e}")
    assert e1 < TOL[precision]


def test_bad_state_is_reported():
    from paper_1208_4772_amd import dg
    print("[tet3d negative density]", flush=True)
    g, o, s, xyz = setup(3, 2, "fp64")
    U0 = smooth_state3(xyz, seed=2)
    U0[5, 0, 3] = -1.0
    U = s.state(U0)
    with pytest.raises(dg.DGError) as e:
        s.run(U, 1)
    assert e.value.code == dg.DG_ENONFINITE
    st = s.run(s.state(smooth_state3(xyz, seed=2)), 2)
    assert st.status == 0 and st.steps == 2


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_periodic_run_conserves(precision):
    """Twenty steps on the periodic mesh keep the five totals (exact L2
    weights of the nodal interpolant) to rounding."""
    print(f"[tet3d conservation {precision}]", flush=True)
    g, o, s, xyz = setup(3, 3, precision)
    U0 = smooth_state3(xyz, seed=9)
    U = s.state(U0)
    s.run(U, 20)
    t0, t1 = o.totals(U0), o.totals(host(U))
    scale = np.abs(o.totals(np.abs(U0)))
    drift = np.abs(t1 - t0) / scale
    print(f"relative drift {drift}")
    assert drift.max() < (1e-13 if precision == "fp64" else 2e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_element_with_four_walls(precision):
    """One tetrahedron whose four faces are walls (the smallest ragged tile:
    one element of a 12-element block) at P = 1..4."""
    from paper_1208_4772_amd import dg3
    from meshgen.tets import TetGrid, connect3
    X = np.array([[[0.1, 0.0, 0.05], [1.0, 0.1, 0.0], [0.05, 0.9, 0.1], [0.0, 0.1, 1.1]]])
    EToV = np.array([[0, 1, 2, 3]])
    g = TetGrid(EToV, X, None)
    g.EToE, g.EToF, g.bc = connect3(EToV)
    assert (g.bc == 1).all()
    for P in (1, 2, 3, 4):
        print(f"[tet3d one element P={P} {precision}]", flush=True)
        o = T.Oracle3D(T.TetMesh(EToV, X, None), P)
        s = dg3.Solver3D.from_mesh(g, P, precision=precision)
        r, st, t = dg3.reference_nodes3(P)
        U0 = smooth_state3(affine_node_coordinates(g, r, st, t), seed=P)
        ref = o.rhs(U0)
        e = rel_l2(host(s.rhs(s.state(U0))), ref)
        print(f"rel L2 {e:.3e}")
        assert e < TOL[precision]
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_equal_eager_steps(precision):
    """Runs of 2 and 4 steps replay a captured two-step graph; runs of one
    step launch eagerly: after the same number of steps the states agree
    bitwise, replay after replay, with eager work and synchronisation in
    between."""
    print(f"[tet3d graph vs eager {precision}]", flush=True)
    g, o, s, xyz = setup(3, 3, precision, periodic=False, jitter=0.1, seed=13)
    U0 = smooth_state3(xyz, seed=21)
    Ug, Ue = s.state(U0), s.state(U0)
    for rep in range(3):
        s.run(Ug, 4 if rep != 1 else 2)
        for _ in range(4 if rep != 1 else 2):
            s.run(Ue, 1)
        s.rhs(Ue)
        assert np.array_equal(host(Ug), host(Ue)), rep
