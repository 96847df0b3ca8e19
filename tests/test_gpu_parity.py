"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle
on the same seeded inputs.

Bars: FP64 path within 1e-12 relative L2 of the oracle (rhs and 100-step
runs); FP32 path within the bound derived from FP32 rounding of the
contractions (FP32_RHS_TOL, FP32_RUN_TOL below), with the measured errors
printed.
"""
import math

import numpy as np
import pytest

import meshgen
from oracle import oracle as orc
from oracle.refelem import ref

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
# FP32: unit roundoff 6e-8 times the cancellation in the flux derivatives
# (|Dr| |F| / |Dr F| of order 10-100 on these meshes); see the derivation
# next to the parity bars in the design notes.
FP32_RHS_TOL = 2e-5
FP32_RUN_TOL = 2e-5
# BF16x3 products: per product |AB - (Ah Bh + Ah Bl + Al Bh)| <= 3 * 2^-16 |A||B|
# (BF16 unit roundoff 2^-8, squared), times the same cancellation factor
# (~110) that the FP32 bar allows for 2^-24.
BF3_RHS_TOL = 3 * 2.0 ** -16 * 110
BF3_RUN_TOL = BF3_RHS_TOL
TOL = {"fp64": FP64_TOL, "fp32": FP32_RHS_TOL, "bf16x3": BF3_RHS_TOL}
RUN_TOL = {"fp64": FP64_TOL, "fp32": FP32_RUN_TOL, "bf16x3": BF3_RUN_TOL}


def dg():
    from paper_1208_4772_amd import dg as _dg
    return _dg


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def perturbed_state(x, y, q, amp=0.1):
    """Smooth perturbation of the state q (rho, rho u, rho v, E)."""
    rho0, u0, v0 = q[0], q[1] / q[0], q[2] / q[0]
    p0 = 0.4 * (q[3] - 0.5 * rho0 * (u0 * u0 + v0 * v0))
    rho = rho0 * (1 + amp * np.sin(x) * np.cos(0.7 * y))
    u = u0 + amp * np.sin(0.9 * y)
    v = v0 + amp * np.cos(1.1 * x)
    p = p0 * (1 + amp * np.cos(x + 0.5 * y))
    return meshgen.primitive_to_conserved(rho, u, v, p)


UNIT_ROUNDOFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 3 * 2.0 ** -16}


def rhs_condition(x, y, U, R, rhs):
    """kappa = || |rx| |Dr| |F| + |sx| |Ds| |F| + |ry| |Dr| |G| + |sy| |Ds| |G| || / ||rhs||:
    how much the volume term's flux derivatives cancel in the rhs.  A
    rounding error u per operation in either evaluation moves the rhs by
    about u kappa relative; fine meshes (|rx| ~ 2/h) make kappa large."""
    rho, mx, my, E = U[:, 0], U[:, 1], U[:, 2], U[:, 3]
    p = 0.4 * (E - 0.5 * (mx * mx + my * my) / rho)
    F = np.stack([mx, mx * mx / rho + p, mx * my / rho, (E + p) * mx / rho], 1)
    G = np.stack([my, mx * my / rho, my * my / rho + p, (E + p) * my / rho], 1)
    xr, xs, yr, ys = x @ R.Dr.T, x @ R.Ds.T, y @ R.Dr.T, y @ R.Ds.T
    J = xr * ys - xs * yr
    rx, sx, ry, sy = ys / J, -yr / J, -xs / J, xr / J
    aDr, aDs = np.abs(R.Dr), np.abs(R.Ds)
    T = np.zeros_like(U)
    for c in range(4):
        aF, aG = np.abs(F[:, c]), np.abs(G[:, c])
        T[:, c] = (np.abs(rx) * (aF @ aDr.T) + np.abs(sx) * (aF @ aDs.T)
                   + np.abs(ry) * (aG @ aDr.T) + np.abs(sy) * (aG @ aDs.T))
    return float(np.linalg.norm(T) / np.linalg.norm(rhs))


def cond_tol(precision, kappa):
    """The reduced precisions' bar, widened where the rhs is worse
    conditioned than on the small parity meshes: C u kappa with C = 1 for
    FP32 (measured 0.3: the matrix-core accumulation rounds less than the
    worst case) and 0.1 for BF16x3 (measured 0.02 against its per-product
    bound 3 * 2^-16: the dropped lo*lo terms and split roundings are
    uncorrelated and partly cancel).  FP64 is held to a multiple of the
    oracle's own spread instead (fp64_spread_tol)."""
    C = {"fp32": 1.0, "bf16x3": 0.1}[precision]
    return max(TOL[precision], C * UNIT_ROUNDOFF[precision] * kappa)


def fp64_spread_tol(case, U):
    """FP64 bar on an ill-conditioned mesh: twice the largest difference
    between four valid FP64 evaluations of the oracle itself (with and
    without contraction, operators as built or re-rounded to exact zero row
    sums), measured here on the same input; never below 1e-12."""
    from test_oracle_reorder import oracle_spread
    return max(FP64_TOL, 2.0 * oracle_spread(case, U))


def subset_errors(mesh, got, ref_rhs, curved=None):
    """Relative L2 error over the elements with a wall face, with a far-field
    face and (if given) the curved ones, so that an error confined to the
    few boundary elements cannot hide in the global norm; and the largest
    pointwise error scaled by the largest reference value."""
    out = {}
    sel = {"wall": (mesh.bc == meshgen.BC_WALL).any(axis=1),
           "farfield": (mesh.bc == meshgen.BC_FARFIELD).any(axis=1)}
    if curved is not None:
        sel["curved"] = curved
    for k, m in sel.items():
        if m.any() and np.linalg.norm(ref_rhs[m]) > 0:
            out[k] = rel_l2(got[m], ref_rhs[m])
    out["max_scaled"] = float(np.abs(got - ref_rhs).max() / np.abs(ref_rhs).max())
    return out


def assert_subsets(mesh, got, ref_rhs, tol, curved=None, label=""):
    errs = subset_errors(mesh, got, ref_rhs, curved)
    print(f"[{label}] subsets " + ", ".join(f"{k} {v:.3e}" for k, v in errs.items()))
    for k, v in errs.items():
        # a pointwise error may exceed the L2 one by the ratio of norms;
        # 10x the L2 bar bounds it on every mesh here
        assert v <= (10 * tol if k == "max_scaled" else tol), (k, v, tol)


def case_pair(mesh, P, q, precision, av=False, **kw):
    R = ref(P)
    x, y = meshgen.node_coordinates(mesh, R.r, R.s)
    o = orc.Oracle(mesh, P, x, y, freestream=q, av=av, **kw)
    s = dg().Solver(mesh.EToE, mesh.EToF, mesh.bc, x, y, P, precision, freestream=q, av=av,
                    **{k: v for k, v in kw.items() if k in ("cfl", "av_eps0", "av_kappa", "av_s0", "riemann")})
    return o, s, x, y


def meshes_for_rhs():
    qv = np.array([1.0, 1.0, 0.0, 1.0 / 0.4 + 0.5])
    out = []
    for P in (1, 2, 3, 4, 5):
        out.append((f"curved_periodic_P{P}", lambda: meshgen.periodic_square(5, perm_seed=11, curved_amplitude=0.05), P, qv))
    out.append(("vortex_config_P2", lambda: meshgen.periodic_square(16), 2, qv))
    out.append(("ragged_P5_K18", lambda: meshgen.periodic_square(3, perm_seed=5), 5, qv))
    out.append(("cylinder_small_P4", lambda: meshgen.cylinder_annulus(24, 6), 4, meshgen.freestream_state(0.38)))
    out.append(("farfield_annulus_P3", lambda: meshgen.cylinder_annulus(20, 5, inner_bc=meshgen.BC_FARFIELD), 3,
                meshgen.freestream_state(0.5, 5.0)))
    out.append(("airfoil_small_P3", lambda: meshgen.naca4_ogrid(40, 8), 3, meshgen.freestream_state(0.8, 1.25)))
    # P = 1 tiles hold more elements than a quarter of the workgroup's
    # threads: several tiles, walls and far field
    out.append(("airfoil_small_P1", lambda: meshgen.naca4_ogrid(40, 8), 1, meshgen.freestream_state(0.66, 1.25)))
    out.append(("cylinder_small_P1", lambda: meshgen.cylinder_annulus(24, 6), 1, meshgen.freestream_state(0.38)))
    # M = 1.5 through a far-field-only annulus: the inner circle sees
    # supersonic inflow and outflow as well as subsonic normal velocities
    out.append(("supersonic_farfield_P3", lambda: meshgen.cylinder_annulus(24, 4, R2=3.0, inner_bc=meshgen.BC_FARFIELD),
                3, meshgen.freestream_state(1.5, 5.0)))
    return out


@pytest.mark.parametrize("name,mk,P,q", meshes_for_rhs(), ids=[m[0] for m in meshes_for_rhs()])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_rhs_matches_oracle(name, mk, P, q, precision):
    import torch
    mesh = mk()
    o, s, x, y = case_pair(mesh, P, q, precision)
    U = perturbed_state(x, y, q)
    ref_rhs = o.rhs(U)
    got = s.rhs(s.state(U)).double().cpu().numpy()
    torch.cuda.synchronize()
    err = rel_l2(got, ref_rhs)
    print(f"[{name} {precision}] K={mesh.K} rel L2 {err:.3e} max {np.abs(got - ref_rhs).max():.3e}")
    assert err <= TOL[precision]
    curved = None
    if mesh.curve is not None:
        curved = (mesh.bc == meshgen.BC_WALL).any(axis=1)
    elif mesh.node_displacement is not None:
        curved = np.ones(mesh.K, bool)
    assert_subsets(mesh, got, ref_rhs, TOL[precision], curved, f"{name} {precision}")


def test_supersonic_farfield_branches_are_exercised():
    """The supersonic parity case above does reach both supersonic far-field
    branches and the subsonic ones."""
    mesh = meshgen.cylinder_annulus(24, 4, R2=3.0, inner_bc=meshgen.BC_FARFIELD)
    R = ref(3)
    x, y = meshgen.node_coordinates(mesh, R.r, R.s)
    q = meshgen.freestream_state(1.5, 5.0)
    U = perturbed_state(x, y, q)
    ks, fs = np.nonzero(mesh.bc == meshgen.BC_FARFIELD)
    o = orc.Oracle(mesh, 3, x, y, freestream=q)
    kinds = set()
    for k, f in zip(ks, fs):
        for j in range(R.Nfp):
            v = R.Fmask[f, j]
            u = U[k, :, v]
            q_ = f * R.Nfp + j
            vn = (u[1] * o.geo["nx"][k, q_] + u[2] * o.geo["ny"][k, q_]) / u[0]
            c = math.sqrt(1.4 * 0.4 * (u[3] - 0.5 * (u[1] ** 2 + u[2] ** 2) / u[0]) / u[0])
            kinds.add("sup_in" if vn <= -c else "sup_out" if vn >= c else "sub")
    assert kinds == {"sup_in", "sup_out", "sub"}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_single_element_all_walls(precision):
    """K = 1: one triangle whose three faces are slip walls (a single,
    ragged tile in the matrix-core path)."""
    VX = np.array([0.0, 1.0, 0.2])
    VY = np.array([0.0, 0.1, 0.9])
    m = meshgen.Mesh(VX, VY, np.array([[0, 1, 2]]), np.zeros((1, 3), np.int32),
                     np.array([[0, 1, 2]], np.int32), np.ones((1, 3), np.int8))
    q = meshgen.freestream_state(0.3)
    for P in (1, 2, 3, 4, 5):
        o, s, x, y = case_pair(m, P, q, precision)
        U = perturbed_state(x, y, q)
        got = s.rhs(s.state(U)).double().cpu().numpy()
        ref_rhs = o.rhs(U)
        err = rel_l2(got, ref_rhs)
        print(f"[K=1 walls {precision} P={P}] rel L2 {err:.3e}")
        assert err <= TOL[precision]
        assert np.abs(got - ref_rhs).max() <= 10 * TOL[precision] * np.abs(ref_rhs).max()
        s.close()


@pytest.mark.parametrize("name", ["airfoil", "periodic"])
def test_permuted_mesh_gives_permuted_rhs_fp64(name):
    """The same mesh with its elements in a random order: the FP64 rhs is the
    same permutation of the original's to 1e-15 (each element's arithmetic
    does not depend on where it is stored)."""
    P = 3
    R = ref(P)
    if name == "airfoil":
        base = meshgen.naca4_ogrid(40, 8)
        q = meshgen.freestream_state(0.8, 1.25)
    else:
        base = meshgen.periodic_square(12, perm_seed=None, curved_amplitude=0.05)
        q = np.array([1.0, 1.0, 0.0, 1.0 / 0.4 + 0.5])
    perm = np.random.default_rng(17).permutation(base.K)
    pm = meshgen.permute_elements(base, perm)
    out = []
    for mesh in (base, pm):
        x, y = meshgen.node_coordinates(mesh, R.r, R.s)
        s = dg().Solver(mesh.EToE, mesh.EToF, mesh.bc, x, y, P, "fp64", freestream=q)
        U = perturbed_state(x, y, q)
        out.append(s.rhs(s.state(U)).cpu().numpy())
        s.close()
    a, b = out
    err = rel_l2(b, a[perm])
    print(f"[permuted {name} fp64] rel L2 {err:.3e}, bitwise {bool((b == a[perm]).all())}")
    assert err <= 1e-15


def test_run_fp64_vortex_config_100_steps():
    """512 jittered, permuted triangles, P=2, isentropic vortex, CFL 0.5,
    100 CFL steps: state, time and totals against the oracle."""
    P = 2
    R = ref(P)
    case = meshgen.make_case("vortex", R.r, R.s)
    o = orc.Oracle.for_case(case)
    s = dg().Solver.from_case(case, "fp64")
    Ur, info = o.run(case.U0, case.steps)
    Ud = s.state(case.U0)
    st = s.run(Ud, case.steps)
    got = Ud.cpu().numpy()
    err = rel_l2(got, Ur)
    print(f"[vortex fp64] rel L2 {err:.3e} t {st.t} vs {info['t']}")
    assert err <= FP64_TOL
    assert abs(st.t - info["t"]) <= 1e-12 * info["t"]
    assert abs(st.dt_min - info["dt_min"]) <= 1e-12 * info["dt_min"]
    np.testing.assert_allclose(st.totals, o.totals(Ur), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(s.totals(Ud), o.totals(Ur), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(st.residual, o.residual(Ur), rtol=1e-10, atol=1e-12)
    assert st.status == 0


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_run_fp32_vortex_config_100_steps(precision):
    P = 2
    R = ref(P)
    case = meshgen.make_case("vortex", R.r, R.s)
    o = orc.Oracle.for_case(case)
    s = dg().Solver.from_case(case, precision)
    Ur, info = o.run(case.U0, case.steps)
    Ud = s.state(case.U0)
    st = s.run(Ud, case.steps)
    got = Ud.double().cpu().numpy()
    err = rel_l2(got, Ur)
    mx = np.abs(got - Ur).max()
    print(f"[vortex {precision}] rel L2 {err:.3e} max {mx:.3e} t {st.t} vs {info['t']}")
    assert err <= RUN_TOL[precision]
    assert abs(st.t - info["t"]) <= 1e-5 * info["t"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fixed_dt_steps_match_oracle(precision):
    mesh = meshgen.cylinder_annulus(24, 6)
    q = meshgen.freestream_state(0.38)
    o, s, x, y = case_pair(mesh, 4, q, precision)
    U = perturbed_state(x, y, q, amp=0.02)
    Ur, _ = o.run(U, 3, dt=1e-3)
    Ud = s.state(U)
    for _ in range(3):
        s.step(Ud, dt=1e-3)
    got = Ud.double().cpu().numpy()
    err = rel_l2(got, Ur)
    print(f"[fixed dt {precision}] rel L2 {err:.3e}")
    assert err <= (FP64_TOL if precision == "fp64" else FP32_RUN_TOL)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_bench_config_full_size(precision):
    """The benchmark workload at full size (cylinder, 20,000 curved-wall
    triangles, P=4, slip wall + far field): rhs of a perturbed state over all
    20,000 elements, and 10 CFL steps from the impulsive freestream start."""
    R = ref(4)
    case = meshgen.make_case("cylinder", R.r, R.s)
    assert case.K == 20000
    o = orc.Oracle.for_case(case)
    s = dg().Solver.from_case(case, precision)
    U = perturbed_state(case.x, case.y, case.freestream, amp=0.05)
    got = s.rhs(s.state(U)).double().cpu().numpy()
    ref_rhs = o.rhs(U)
    err = rel_l2(got, ref_rhs)
    print(f"[cylinder full rhs {precision}] rel L2 {err:.3e}")
    assert err <= TOL[precision]
    assert_subsets(case.mesh, got, ref_rhs, TOL[precision], (case.mesh.bc == meshgen.BC_WALL).any(axis=1),
                   f"cylinder full {precision}")
    Ur, info = o.run(case.U0, 10)
    Ud = s.state(case.U0)
    st = s.run(Ud, 10)
    got = Ud.double().cpu().numpy()
    # compare the change from the start (the state itself is dominated by
    # the uniform freestream)
    err = rel_l2(got - case.U0, Ur - case.U0)
    print(f"[cylinder full 10 steps {precision}] rel L2 of the update {err:.3e}")
    assert err <= {"fp64": FP64_TOL * 10, "fp32": 1e-3, "bf16x3": 1e-2}[precision]
    assert abs(st.t - info["t"]) <= (1e-12 if precision == "fp64" else 1e-5) * info["t"]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_roofline_config_full_size(precision):
    """The roofline mesh at full size (999,698 jittered straight triangles,
    P=5, periodic): rhs over every element and 2 CFL steps; and the rhs of
    the all-curved variant of the same mesh.  The input is a smooth
    perturbation of the freestream everywhere (the vortex alone leaves
    almost every element at a freestream rhs of zero, so the norm the error
    is measured against comes from a small region).  On elements this small
    the flux derivatives cancel ~1800-fold in the rhs (kappa), so the bar
    is the precision's bar widened by kappa (cond_tol)."""
    import torch
    R = ref(5)
    for name in ("roofline", "roofline_curved"):
        case = meshgen.make_case(name, R.r, R.s)
        assert case.K == 999698
        o = orc.Oracle.for_case(case)
        s = dg().Solver.from_case(case, precision)
        U = perturbed_state(case.x, case.y, case.freestream, amp=0.05)
        got = s.rhs(s.state(U)).double().cpu().numpy()
        ref_rhs = o.rhs(U)
        err = rel_l2(got, ref_rhs)
        kappa = rhs_condition(case.x, case.y, U, R, ref_rhs)
        tol = fp64_spread_tol(case, U) if precision == "fp64" else cond_tol(precision, kappa)
        print(f"[{name} full rhs {precision}] rel L2 {err:.3e}, kappa {kappa:.0f}, "
              f"{err / (UNIT_ROUNDOFF[precision] * kappa):.1f} u kappa, bar {tol:.3e}")
        assert err <= tol
        assert np.abs(got - ref_rhs).max() <= 10 * tol * np.abs(ref_rhs).max()
        if name == "roofline":
            if precision != "fp64":
                U = U.astype(np.float32).astype(np.float64)
            Ur, info = o.run(U, 2)
            Ud = s.state(U)
            st = s.run(Ud, 2)
            torch.cuda.synchronize()
            got = Ud.double().cpu().numpy()
            err = rel_l2(got - U, Ur - U)
            print(f"[{name} full 2 steps {precision}] rel L2 of the update {err:.3e}")
            assert err <= {"fp64": FP64_TOL * 10, "fp32": 1e-3, "bf16x3": 1e-2}[precision]
            assert abs(st.t - info["t"]) <= (1e-12 if precision == "fp64" else 1e-5) * info["t"]
        s.close()
        del o


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_airfoil_config_full_size(precision):
    """The transonic airfoil at full size (120,000 triangles, curved wall,
    P=3, sensor and artificial viscosity): viscosity and rhs of a perturbed
    state with a density step over every element, and 10 CFL steps from
    it."""
    import torch
    R = ref(3)
    case = meshgen.make_case("airfoil", R.r, R.s, start="damped")
    assert case.K == 120000 and case.av
    o = orc.Oracle.for_case(case)
    s = dg().Solver.from_case(case, precision)
    U = perturbed_state(case.x, case.y, case.freestream, amp=0.02)
    U[:, 0] *= np.where(case.x < 0.4, 1.0, 2.5)
    U[:, 3] *= np.where(case.x < 0.4, 1.0, 2.5)
    eps_ref = o.sensor(U)
    eps = s.viscosity(s.state(U)).cpu().numpy()
    assert (eps_ref > 0).sum() > 100
    np.testing.assert_allclose(eps, eps_ref, rtol=0,
                               atol=(1e-12 if precision == "fp64" else 1e-4) * eps_ref.max())
    got = s.rhs(s.state(U)).double().cpu().numpy()
    ref_rhs = o.rhs(U)
    err = rel_l2(got, ref_rhs)
    print(f"[airfoil full rhs {precision}] rel L2 {err:.3e}, {int((eps_ref > 0).sum())} viscous elements")
    assert err <= TOL[precision]
    assert_subsets(case.mesh, got, ref_rhs, TOL[precision], (case.mesh.bc == meshgen.BC_WALL).any(axis=1),
                   f"airfoil full {precision}")
    # the run starts from the same perturbed state (a global signal: from
    # the damped start the first steps change only the flow near the wall,
    # and the relative error of that change is the FP32 rounding noise of
    # the freestream's nearly cancelling rhs over the whole mesh)
    U0 = U.astype(np.float32).astype(np.float64) if precision != "fp64" else U
    Ur, info = o.run(U0, 10)
    Ud = s.state(U0)
    st = s.run(Ud, 10)
    torch.cuda.synchronize()
    got = Ud.double().cpu().numpy()
    err = rel_l2(got - U0, Ur - U0)
    print(f"[airfoil full 10 steps {precision}] rel L2 of the update {err:.3e}")
    assert err <= {"fp64": FP64_TOL * 10, "fp32": 1e-3, "bf16x3": 1e-2}[precision]
    assert abs(st.t - info["t"]) <= (1e-12 if precision == "fp64" else 1e-5) * info["t"]


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_viscosity_and_av_rhs_match_oracle(precision, P):
    mesh = meshgen.naca4_ogrid(40, 8)
    q = meshgen.freestream_state(0.8, 1.25)
    # at P = 1 the default s0 = -4 log10 P = 0 sets the threshold at a
    # top-mode energy fraction of 0.1, above what the density step reaches
    # on these elements; s0 = -1 brings the sensor in
    extra = {"av_s0": -1.0} if P == 1 else {}
    o, s, x, y = case_pair(mesh, P, q, precision, av=True, av_kappa=1.0, av_eps0=0.3, **extra)
    U = perturbed_state(x, y, q, amp=0.02)
    # a density step across x = 0.4 triggers the sensor near the airfoil
    U[:, 0] *= np.where(x < 0.4, 1.0, 2.5)
    U[:, 3] *= np.where(x < 0.4, 1.0, 2.5)
    eps_ref = o.sensor(U)
    eps = s.viscosity(s.state(U)).cpu().numpy()
    assert (eps_ref > 0).sum() > 0
    # FP32: the sensor's log10 of a ratio of FP32 sums moves s_k by ~1e-6,
    # and the ramp slope (pi/2) eps_max / kappa turns that into ~1e-6 eps_max
    np.testing.assert_allclose(eps, eps_ref, rtol=0,
                               atol=(1e-12 if precision == "fp64" else 1e-4) * eps_ref.max())
    got = s.rhs(s.state(U)).double().cpu().numpy()
    err = rel_l2(got, o.rhs(U))
    print(f"[airfoil AV rhs {precision} P={P}] rel L2 {err:.3e}, {int((eps_ref > 0).sum())} viscous elements")
    assert err <= TOL[precision]


def test_clockwise_element_is_a_geometry_error():
    m = meshgen.periodic_square(4, perm_seed=None)
    m.EToV[0, 1], m.EToV[0, 2] = m.EToV[0, 2], m.EToV[0, 1]
    R = ref(2)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    with pytest.raises(dg().DGError) as e:
        dg().Solver(m.EToE, m.EToF, m.bc, x, y, 2, "fp64")
    assert e.value.code == dg().DG_EGEOM


def test_nonfinite_state_is_reported():
    P = 2
    R = ref(P)
    case = meshgen.make_case("vortex", R.r, R.s)
    s = dg().Solver.from_case(case, "fp32")
    U = case.U0.copy()
    U[7, 0, 3] = -1.0   # negative density
    Ud = s.state(U)
    with pytest.raises(dg().DGError) as e:
        s.run(Ud, 1)
    assert e.value.code == dg().DG_ENONFINITE


def test_runs_are_bitwise_deterministic():
    P = 4
    R = ref(P)
    case = meshgen.make_case("cylinder", R.r, R.s, scale=0.05)
    s = dg().Solver.from_case(case, "fp32")
    a = s.state(case.U0)
    b = s.state(case.U0)
    s.run(a, 20)
    s.run(b, 20)
    assert bool((a == b).all())


def test_graph_replay_equals_eager_bitwise():
    """dg_run replays a captured two-step graph; the result must be the same
    bits as the eager launches, across several calls with eager work and
    synchronisations between them."""
    import torch
    P = 4
    R = ref(P)
    case = meshgen.make_case("cylinder", R.r, R.s, scale=0.05)
    s = dg().Solver.from_case(case, "fp32")
    eager = s.state(case.U0)
    graph = s.state(case.U0)
    s.set_graphs(False)
    for _ in range(3):
        s.run(eager, 7)
    s.set_graphs(True)
    for _ in range(3):
        s.run(graph, 7)
        torch.cuda.synchronize()
        _ = (graph * 2.0).sum().item()   # unrelated eager work between replays
    assert bool((eager == graph).all())


def test_autotune_keeps_results_bitwise():
    """The autotuner only changes the launch shape of the stage kernel: the
    rhs and a run are the same bits before and after it."""
    import torch
    dg().Tuning.clear()     # time the candidates (no table entry)
    R = ref(4)
    case = meshgen.make_case("cylinder", R.r, R.s, scale=0.1)
    s = dg().Solver.from_case(case, "fp32")
    U = s.state(case.U0)
    r0 = s.rhs(U).clone()
    U0 = U.clone()
    s.run(U0, 6)
    blocks, us = s.autotune(U)
    assert blocks >= 1 and us > 0
    r1 = s.rhs(U)
    U1 = U.clone()
    s.run(U1, 6)
    torch.cuda.synchronize()
    assert torch.equal(r0, r1) and torch.equal(U0, U1)
    f = dg().Solver.from_case(case, "fp64")
    assert f.autotune(f.state(case.U0)) == (0, 0.0)
    dg().Tuning.clear()


@pytest.mark.parametrize("av", [True, False], ids=["av", "inviscid"])
@pytest.mark.parametrize("P", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_airfoil_run_matches_oracle(precision, P, av):
    """12 CFL steps from the impulsive start on a small airfoil O-grid (the
    shape of the serving requests), with and without the viscous terms:
    state update and simulated time against the oracle."""
    import torch
    mesh = meshgen.naca4_ogrid(40, 8)
    q = meshgen.freestream_state(0.66, 1.25)
    kw = dict(av_kappa=1.0, av_eps0=0.3) if av else {}
    o, s, x, y = case_pair(mesh, P, q, precision, av=av, **kw)
    U0 = meshgen.uniform((mesh.K, x.shape[1]), q)
    Ur, info = o.run(U0, 12)
    Ud = s.state(U0)
    st = s.run(Ud, 12, check=False)
    torch.cuda.synchronize()
    got = Ud.double().cpu().numpy()
    assert np.all(np.isfinite(Ur)) and st.status == 0, st.status
    err = rel_l2(got - U0, Ur - U0)
    print(f"[airfoil {'AV' if av else 'inviscid'} run {precision} P={P}] rel L2 of the update {err:.3e}")
    assert err <= (FP64_TOL * 10 if precision == "fp64" else 1e-3)
    assert abs(st.t - info["t"]) <= (1e-12 if precision == "fp64" else 1e-5) * info["t"]


@pytest.mark.parametrize("av", [False, True], ids=["inviscid", "av"])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_fp32_runs_compose_bitwise(precision, av):
    """dg_run of N steps twice gives the same bits as one dg_run of 2N steps
    (N odd, so the second call starts at the other step parity): the first
    step of a call takes the same FP64 per-node time-step bound a fused last
    stage would have left."""
    import torch
    mesh = meshgen.naca4_ogrid(40, 8)
    q = meshgen.freestream_state(0.66, 1.25)
    kw = dict(av_kappa=1.0, av_eps0=0.3) if av else {}
    o, s, x, y = case_pair(mesh, 3, q, precision, av=av, **kw)
    U0 = perturbed_state(x, y, q, amp=0.02)
    a = s.state(U0)
    b = s.state(U0)
    N = 7
    s.run(a, N)
    s.run(a, N)
    s.run(b, 2 * N)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_viscous_rhs_can_be_captured(precision):
    """dg_rhs of a viscous handle allocates nothing, so it can be captured
    into a graph; every replay (with eager work and synchronisation between
    replays) equals the eager call."""
    import torch
    mesh = meshgen.naca4_ogrid(40, 8)
    q = meshgen.freestream_state(0.8, 1.25)
    o, s, x, y = case_pair(mesh, 3, q, precision, av=True, av_kappa=1.0, av_eps0=0.3)
    U = perturbed_state(x, y, q, amp=0.02)
    U[:, 0] *= np.where(x < 0.4, 1.0, 2.5)
    U[:, 3] *= np.where(x < 0.4, 1.0, 2.5)
    Ud = s.state(U)
    eager = s.rhs(Ud).clone()
    out = s.empty_state()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        s.rhs(Ud, out=out)          # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.rhs(Ud, out=out)
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
        _ = (Ud * 2).sum().item()


def hllc_cases():
    return [
        ("curved_periodic_P3", lambda: meshgen.periodic_square(5, perm_seed=11, curved_amplitude=0.05), 3,
         np.array([1.0, 1.0, 0.0, 1.0 / 0.4 + 0.5])),
        ("cylinder_small_P4", lambda: meshgen.cylinder_annulus(24, 6), 4, meshgen.freestream_state(0.38)),
        ("airfoil_small_P2", lambda: meshgen.naca4_ogrid(40, 8), 2, meshgen.freestream_state(0.8, 1.25)),
        ("supersonic_farfield_P3", lambda: meshgen.cylinder_annulus(24, 4, R2=3.0, inner_bc=meshgen.BC_FARFIELD),
         3, meshgen.freestream_state(1.5, 5.0)),
        ("ragged_P5_K18", lambda: meshgen.periodic_square(3, perm_seed=5), 5,
         np.array([1.0, 1.0, 0.0, 1.0 / 0.4 + 0.5])),
    ]


@pytest.mark.parametrize("name,mk,P,q", hllc_cases(), ids=[c[0] for c in hllc_cases()])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_hllc_rhs_matches_oracle(name, mk, P, q, precision):
    """The HLLC flux on the GPU against the oracle's, on states with density
    steps (contacts) and supersonic faces, so that every branch of the flux
    is taken."""
    mesh = mk()
    o, s, x, y = case_pair(mesh, P, q, precision, riemann="hllc")
    U = perturbed_state(x, y, q)
    U[:, 0] *= np.where(np.sin(x + 0.3 * y) > 0, 1.0, 1.6)
    ref_rhs = o.rhs(U)
    got = s.rhs(s.state(U)).double().cpu().numpy()
    err = rel_l2(got, ref_rhs)
    print(f"[hllc {name} {precision}] K={mesh.K} rel L2 {err:.3e}")
    assert err <= TOL[precision]
    assert_subsets(mesh, got, ref_rhs, TOL[precision], None, f"hllc {name} {precision}")
    s.close()


@pytest.mark.parametrize("av", [False, True], ids=["inviscid", "av"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_hllc_airfoil_run_matches_oracle(precision, av):
    import torch
    mesh = meshgen.naca4_ogrid(40, 8)
    q = meshgen.freestream_state(0.66, 1.25)
    kw = dict(av_kappa=1.0, av_eps0=0.3) if av else {}
    o, s, x, y = case_pair(mesh, 3, q, precision, av=av, riemann="hllc", **kw)
    U0 = meshgen.uniform((mesh.K, x.shape[1]), q)
    Ur, info = o.run(U0, 12)
    Ud = s.state(U0)
    st = s.run(Ud, 12, check=False)
    torch.cuda.synchronize()
    got = Ud.double().cpu().numpy()
    assert st.status == 0
    err = rel_l2(got - U0, Ur - U0)
    print(f"[hllc airfoil run {precision} av={av}] rel L2 of the update {err:.3e}")
    assert err <= (FP64_TOL * 10 if precision == "fp64" else 1e-3)
    assert abs(st.t - info["t"]) <= (1e-12 if precision == "fp64" else 1e-5) * info["t"]


@pytest.mark.parametrize("P,Q", [(1, 2), (2, 3), (2, 4), (3, 5), (4, 5)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_prolongation_matches_oracle(precision, P, Q):
    """dg_prolong against the oracle's prolongation (p-refinement)."""
    mesh = meshgen.naca4_ogrid(40, 8)
    q = meshgen.freestream_state(0.5, 1.25)
    Rp, Rq = ref(P), ref(Q)
    xp, yp = meshgen.node_coordinates(mesh, Rp.r, Rp.s)
    xq, yq = meshgen.node_coordinates(mesh, Rq.r, Rq.s)
    sp = dg().Solver(mesh.EToE, mesh.EToF, mesh.bc, xp, yp, P, precision, freestream=q)
    sq = dg().Solver(mesh.EToE, mesh.EToF, mesh.bc, xq, yq, Q, precision, freestream=q)
    U = perturbed_state(xp, yp, q)
    Ud = sp.state(U)
    got = sq.prolong_from(sp, Ud).double().cpu().numpy()
    want = orc.prolong(Ud.double().cpu().numpy(), P, Q)
    err = rel_l2(got, want)
    print(f"[prolong {P}->{Q} {precision}] rel L2 {err:.3e}")
    assert err <= (1e-15 if precision == "fp64" else 2e-7)


def test_p_refinement_continuation_matches_oracle():
    """The continuation driver on the GPU (10 steps at P = 2, prolongation,
    20 steps at P = 3) against the oracle running the same schedule."""
    import torch
    from paper_1208_4772_amd import continuation
    mesh = meshgen.cylinder_annulus(24, 6)
    q = meshgen.freestream_state(0.38)

    def xy(P):
        R = ref(P)
        return meshgen.node_coordinates(mesh, R.r, R.s)

    def make_solver(P):
        x, y = xy(P)
        return dg().Solver(mesh.EToE, mesh.EToF, mesh.bc, x, y, P, "fp64", freestream=q)

    x2, y2 = xy(2)
    U0 = meshgen.cylinder_potential(x2, y2, 0.38)
    res = continuation.run(make_solver, U0, (2, 3), check_every=10, switch_residual=1e9,
                           final_residual=1e-30, max_steps_per_order=20)
    assert [leg.steps for leg in res.legs] == [10, 20]
    got = res.state.cpu().numpy()
    res.solver.close()
    o2 = orc.Oracle(mesh, 2, x2, y2, freestream=q)
    U, i2 = o2.run(U0, 10)
    x3, y3 = xy(3)
    o3 = orc.Oracle(mesh, 3, x3, y3, freestream=q)
    U3 = orc.prolong(U, 2, 3)
    Ur, i3 = o3.run(U3, 20)
    err = rel_l2(got - U3, Ur - U3)
    print(f"[continuation 2->3 fp64] rel L2 of the P=3 update {err:.3e}, t {res.legs[0].t} {i2['t']}")
    assert err <= 10 * FP64_TOL
    assert abs(res.legs[0].t - i2["t"]) <= 1e-12 * i2["t"]
    assert abs(res.legs[1].t - i3["t"]) <= 1e-12 * i3["t"]


def weak_cases():
    qv = np.array([1.0, 1.0, 0.0, 1.0 / 0.4 + 0.5])
    return [
        ("curved_periodic_P2", lambda: meshgen.periodic_square(5, perm_seed=11, curved_amplitude=0.05), 2, qv),
        ("curved_periodic_P5", lambda: meshgen.periodic_square(5, perm_seed=11, curved_amplitude=0.05), 5, qv),
        ("cylinder_small_P3", lambda: meshgen.cylinder_annulus(24, 6), 3, meshgen.freestream_state(0.38)),
        ("airfoil_small_P4", lambda: meshgen.naca4_ogrid(40, 8), 4, meshgen.freestream_state(0.7, 1.25)),
        ("supersonic_farfield_P1", lambda: meshgen.cylinder_annulus(24, 4, R2=3.0, inner_bc=meshgen.BC_FARFIELD),
         1, meshgen.freestream_state(1.5, 5.0)),
        ("vortex_config_P2", lambda: meshgen.periodic_square(16), 2, qv),
        # straight elements only, slip walls, K = 42 (two full blocks of 16
        # and a ragged one): FP32 runs the matrix-core kernel here
        ("straight_channel_P1", lambda: meshgen.channel(7, 3, perm_seed=5), 1, qv),
        ("straight_channel_P3", lambda: meshgen.channel(7, 3, perm_seed=5), 3, qv),
        ("straight_channel_P4", lambda: meshgen.channel(7, 3, perm_seed=5), 4, qv),
        ("straight_channel_P5", lambda: meshgen.channel(7, 3, perm_seed=5), 5, qv),
    ]


@pytest.mark.parametrize("name,mk,P,q", weak_cases(), ids=[c[0] for c in weak_cases()])
@pytest.mark.parametrize("riemann", ["lf", "hllc"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_weak_form_rhs_matches_oracle(name, mk, P, q, riemann, precision):
    """The over-integrated weak form on the GPU against the oracle's."""
    mesh = mk()
    R = ref(P)
    x, y = meshgen.node_coordinates(mesh, R.r, R.s)
    o = orc.Oracle(mesh, P, x, y, freestream=q, riemann=riemann, weak=True)
    s = dg().Solver(mesh.EToE, mesh.EToF, mesh.bc, x, y, P, precision, freestream=q, riemann=riemann,
                    form="weak")
    U = perturbed_state(x, y, q)
    ref_rhs = o.rhs(U)
    got = s.rhs(s.state(U)).double().cpu().numpy()
    err = rel_l2(got, ref_rhs)
    tol = TOL[precision]
    if precision == "fp32":
        # the weak form cancels more than the nodal one (V - S of nearly
        # equal volume and surface integrals): the FP64 kernel's distance
        # from the oracle on the same input measures that conditioning, and
        # the same operations in FP32 round 2^29 times coarser
        s64 = dg().Solver(mesh.EToE, mesh.EToF, mesh.bc, x, y, P, "fp64", freestream=q, riemann=riemann,
                          form="weak")
        e64 = rel_l2(s64.rhs(s64.state(U)).cpu().numpy(), ref_rhs)
        s64.close()
        tol = max(tol, 2.0 ** 29 * e64)
    print(f"[weak {name} {riemann} {precision}] K={mesh.K} rel L2 {err:.3e} (bar {tol:.1e})")
    assert err <= tol
    assert_subsets(mesh, got, ref_rhs, tol, None, f"weak {name} {precision}")
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_weak_form_vortex_run_matches_oracle(precision):
    """100 CFL steps of the isentropic vortex configuration (512 permuted,
    jittered triangles, P = 2) in the weak form: state and time."""
    import torch
    P = 2
    R = ref(P)
    case = meshgen.make_case("vortex", R.r, R.s)
    o = orc.Oracle.for_case(case, weak=True)
    s = dg().Solver.from_case(case, precision, form="weak")
    Ur, info = o.run(case.U0, case.steps)
    Ud = s.state(case.U0)
    st = s.run(Ud, case.steps)
    torch.cuda.synchronize()
    got = Ud.double().cpu().numpy()
    err = rel_l2(got, Ur)
    print(f"[weak vortex {precision}] rel L2 {err:.3e}")
    assert err <= RUN_TOL[precision]
    assert abs(st.t - info["t"]) <= (1e-12 if precision == "fp64" else 1e-5) * info["t"]


@pytest.mark.parametrize("form", ["nodal", "weak"])
def test_curved_classification_matches_the_geometry(form):
    """The library treats an element as curved exactly when its map is not
    affine: none on the jittered straight meshes (whose edges nearly
    parallel to an axis give near-zero metric terms, once mistaken for
    varying ones), the wall elements of the cylinder and the airfoil, and
    every element of the all-curved periodic mesh.  FP64 nodal handles take
    per-node metrics everywhere and report -1."""
    checks = [("roofline", 5, 0.02), ("vortex", 2, 1.0), ("cylinder", 4, 0.05), ("airfoil", 3, 0.01),
              ("roofline_curved", 5, 0.005)]
    for name, P, scale in checks:
        R = ref(P)
        case = meshgen.make_case(name, R.r, R.s, P=P, scale=scale)
        m = case.mesh
        if m.node_displacement is not None:
            expect = case.K
        elif m.curve is not None:
            expect = int((m.bc == meshgen.BC_WALL).any(axis=1).sum())
        else:
            expect = 0
        s = dg().Solver.from_case(case, "fp32", form=form, av=False)
        got = s.curved_elements()
        print(f"[curved {form}] {name} K={case.K}: library {got}, geometry {expect}", flush=True)
        assert got == expect, (name, got, expect)
        s.close()
    R = ref(4)
    case = meshgen.make_case("cylinder", R.r, R.s, P=4, scale=0.05)
    assert dg().Solver.from_case(case, "fp64").curved_elements() == -1
