"""Further pins of the oracle: the time-step formula by hand on one element,
each far-field branch against its definition, the viscous slip-wall closure
against the heat equation in a channel, mirror symmetry of the whole
pipeline, the diagnostics (entropy error, wall force, lift and drag, shock
position) and the node family's blending exponents (no GPU)."""
import math

import numpy as np
import pytest

import meshgen
from oracle import diagnostics as dgn
from oracle import oracle as orc
from oracle import refelem
from oracle.refelem import ref

G = 1.4


def one_triangle(bc=meshgen.BC_WALL):
    """The single straight element (0,0), (1,0), (0,1), every face a boundary."""
    VX = np.array([0.0, 1.0, 0.0])
    VY = np.array([0.0, 0.0, 1.0])
    EToV = np.array([[0, 1, 2]])
    EToE = np.zeros((1, 3), np.int32)
    EToF = np.array([[0, 1, 2]], np.int32)
    bcs = np.full((1, 3), bc, np.int8)
    return meshgen.Mesh(VX, VY, EToV, EToE, EToF, bcs, "one_triangle")


def prim(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)])


# -- time step (R11) ---------------------------------------------------------

@pytest.mark.parametrize("P", [1, 2, 3, 5])
@pytest.mark.parametrize("eps", [-1.0, 0.01])
def test_dt_single_element_by_hand(P, eps):
    """dt = CFL / max over face nodes of 1/2 (P+1)^2 Fscale lam + 1/4 (P+1)^4
    Fscale^2 eps.  On the right triangle with legs 1: J = 1/4 (half the area);
    sJ is half the edge length, so Fscale = 2 on the legs and 2 sqrt2 on the
    hypotenuse.  A uniform state has lam = |v| + c at every node, so the
    hypotenuse decides."""
    R = ref(P)
    m = one_triangle()
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    o = orc.Oracle(m, P, x, y, cfl=0.7, eps_override=eps)
    u = prim(1.2, 0.3, -0.4, 0.9)
    U = np.repeat(u[None, :, None], R.Np, axis=2)
    lam = 0.5 + math.sqrt(G * 0.9 / 1.2)
    fs = 2.0 * math.sqrt(2.0)
    e = max(eps, 0.0)
    want = 0.7 / (0.5 * (P + 1) ** 2 * fs * lam + 0.25 * (P + 1) ** 4 * fs * fs * e)
    dt, flag = o.dt(U)
    assert flag == 0
    assert dt == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("P", [2, 4])
def test_dt_takes_each_nodes_own_fscale(P):
    """u = 2 (1 - x - y), v = 0, c = 1: the fastest node (the vertex (0,0),
    |v| + c = 3) lies on the two legs (Fscale 2), while the hypotenuse
    (Fscale 2 sqrt2) carries u = 0, |v| + c = 1.  The bound is 1/2 (P+1)^2 * 6,
    not the product of the element's largest Fscale and largest wave speed."""
    R = ref(P)
    m = one_triangle()
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    o = orc.Oracle(m, P, x, y, cfl=0.5)
    U = np.zeros((1, 4, R.Np))
    for i in range(R.Np):
        U[0, :, i] = prim(1.0, 2.0 * (1.0 - x[0, i] - y[0, i]), 0.0, 1.0 / G)
    dt, _ = o.dt(U)
    assert dt == pytest.approx(0.5 / (0.5 * (P + 1) ** 2 * 6.0), rel=1e-13)


# -- far-field ghost branches (R9) --------------------------------------------

def split(u, nx, ny):
    rho = u[0]
    vx, vy = u[1] / rho, u[2] / rho
    p = (G - 1) * (u[3] - 0.5 * rho * (vx * vx + vy * vy))
    c = math.sqrt(G * p / rho)
    vn = vx * nx + vy * ny
    return rho, vn, (vx - vn * nx, vy - vn * ny), p, c


N30 = (math.cos(math.pi / 6), math.sin(math.pi / 6))


def test_farfield_subsonic_inflow():
    """v_n < 0, |v_n| < c inside: the ghost keeps the outgoing invariant of
    the interior, the incoming invariant, the entropy and the tangential
    velocity of the freestream."""
    nx, ny = N30
    qinf = prim(1.0, -0.5, 0.0, 1.0 / G)           # M = 0.5 towards -x
    um = prim(1.1, -0.3 * nx + 0.2 * ny, -0.3 * ny - 0.2 * nx, 0.8)
    rho_i, vn_i, _, p_i, c_i = split(um, nx, ny)
    assert -c_i < vn_i < 0
    up = orc.ghost(2, um, nx, ny, qinf)
    rho_b, vn_b, vt_b, p_b, c_b = split(up, nx, ny)
    rho_o, vn_o, vt_o, p_o, c_o = split(qinf, nx, ny)
    assert vn_b < 0
    assert vn_b + 2 * c_b / (G - 1) == pytest.approx(vn_i + 2 * c_i / (G - 1), rel=1e-13)
    assert vn_b - 2 * c_b / (G - 1) == pytest.approx(vn_o - 2 * c_o / (G - 1), rel=1e-13)
    assert p_b / rho_b ** G == pytest.approx(p_o / rho_o ** G, rel=1e-13)
    np.testing.assert_allclose(vt_b, vt_o, rtol=0, atol=1e-14)


def test_farfield_subsonic_outflow_keeps_interior_tangential_velocity():
    nx, ny = N30
    qinf = prim(1.0, 0.5, 0.0, 1.0 / G)
    um = prim(0.9, 0.35 * nx - 0.25 * ny, 0.35 * ny + 0.25 * nx, 0.75)
    _, vn_i, vt_i, p_i, c_i = split(um, nx, ny)
    assert 0 < vn_i < c_i
    up = orc.ghost(2, um, nx, ny, qinf)
    rho_b, vn_b, vt_b, p_b, _ = split(up, nx, ny)
    assert vn_b > 0
    np.testing.assert_allclose(vt_b, vt_i, rtol=0, atol=1e-14)
    assert p_b / rho_b ** G == pytest.approx(p_i / um[0] ** G, rel=1e-13)


def test_farfield_supersonic_inflow_is_freestream():
    nx, ny = 1.0, 0.0
    qinf = prim(1.0, -1.5, 0.1, 1.0 / G)           # M = 1.5 into the domain
    um = prim(1.3, -2.0, 0.3, 0.6)                  # v_n = -2 < -c (c = 0.82)
    assert split(um, nx, ny)[1] <= -split(um, nx, ny)[4]
    np.testing.assert_array_equal(orc.ghost(2, um, nx, ny, qinf), qinf)


def test_farfield_supersonic_outflow_is_interior():
    nx, ny = 0.0, -1.0
    qinf = prim(1.0, 0.0, -1.5, 1.0 / G)
    um = prim(0.8, 0.2, -1.9, 0.55)                # v_n = 1.9 > c (c = 0.98)
    assert split(um, nx, ny)[1] >= split(um, nx, ny)[4]
    np.testing.assert_array_equal(orc.ghost(2, um, nx, ny, qinf), um)


# -- viscous slip-wall closure (R13) -------------------------------------------

@pytest.mark.slow
@pytest.mark.parametrize("P", [1, 2, 3])
def test_viscous_wall_closure_solves_channel_heat_equation(P):
    """Inviscid flux off, eps constant, channel [0,10] x [0,4] periodic in x
    with slip walls at y = 0 and y = 4: every field obeys u_t = eps Lap u.
    The mirror ghost makes rho, rho u and E even across a wall (zero normal
    derivative) and rho v odd (zero value), so
      rho = 2 + cos(kx x) e^{-eps kx^2 t},   rho u = cos(ky y) e^{-eps ky^2 t},
      rho v = sin(ky y) e^{-eps ky^2 t},     E = 5 + cos(ky y) cos(kx x) e^{-eps (kx^2+ky^2) t}
    with kx = 2 pi/10, ky = pi/4.  Each field must converge at order >= P+1/2
    and the walls must conserve mass.  (A closure that takes the interior
    sigma Q at the wall for every field does not converge for the even
    fields and leaks mass on a jittered mesh.)"""
    L, H, epsv, T = 10.0, 4.0, 0.5, 1.0
    kx, ky = 2 * math.pi / L, math.pi / H
    R = ref(P)
    errs = []
    for n in (1, 2, 4):
        m = meshgen.channel(5 * n, 2 * n, L, H, 0.1, 3)
        x, y = meshgen.node_coordinates(m, R.r, R.s)
        o = orc.Oracle(m, P, x, y, no_euler_flux=True, eps_override=epsv, cfl=0.5)
        U0 = np.zeros((m.K, 4, R.Np))
        U0[:, 0] = 2.0 + np.cos(kx * x)
        U0[:, 1] = np.cos(ky * y)
        U0[:, 2] = np.sin(ky * y)
        U0[:, 3] = 5.0 + np.cos(ky * y) * np.cos(kx * x)
        dt, _ = o.dt(U0)
        ns = int(np.ceil(T / dt))
        U, info = o.run(U0, ns, dt=T / ns)
        t = info["t"]
        exact = [2.0 + np.cos(kx * x) * math.exp(-epsv * kx ** 2 * t),
                 np.cos(ky * y) * math.exp(-epsv * ky ** 2 * t),
                 np.sin(ky * y) * math.exp(-epsv * ky ** 2 * t),
                 5.0 + np.cos(ky * y) * np.cos(kx * x) * math.exp(-epsv * (kx ** 2 + ky ** 2) * t)]
        errs.append([np.abs(U[:, c] - exact[c]).max() for c in range(4)])
        m0, m1 = o.totals(U0)[0], o.totals(U)[0]
        assert abs(m1 - m0) <= 1e-12 * abs(m0)
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert (rates[-1] >= P + 0.5).all(), rates


# -- mirror symmetry of the whole pipeline ------------------------------------

@pytest.mark.parametrize("body", ["cylinder", "airfoil"])
def test_symmetric_body_at_zero_incidence_has_no_lift(body):
    """A triangulation mirror-symmetric about the x axis, flow at zero
    incidence: the discrete solution is mirror-symmetric, so the lift is
    zero up to rounding while the drag is not.  (A wrong component or sign
    in a wall or far-field ghost state, or any term that treats x and y
    unevenly, breaks the symmetry.)  The airfoil runs with a constant
    viscosity, which takes the viscous terms and their wall closure through
    the same check."""
    P = 3
    R = ref(P)
    if body == "cylinder":
        m = meshgen.cylinder_annulus(24, 6, jitter=0.0, mirror_split=True)
        mach, eps, chord = 0.38, -1.0, 2.0
    else:
        m = meshgen.naca4_ogrid(40, 8, jitter=0.0, mirror_split=True)
        mach, eps, chord = 0.8, 0.002, 1.0
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    q = meshgen.freestream_state(mach, 0.0)
    o = orc.Oracle(m, P, x, y, freestream=q, eps_override=eps)
    U0 = meshgen.uniform((m.K, R.Np), q)
    U, info = o.run(U0, 30)
    assert info["flag"] == 0
    CL, CD = dgn.lift_drag(o, U, q, chord=chord)
    assert abs(CL) <= 1e-12
    assert abs(CD) > 1e-3


# -- diagnostics ---------------------------------------------------------------

def test_entropy_error_closed_forms():
    """Freestream: 0.  Density scaled by a at the freestream pressure:
    e = a^-gamma - 1 everywhere.  p = p_inf (1 + x/10) at rho_inf on [0,10]^2:
    e = x/10, whose RMS over the square is 1/sqrt3 (exact for P >= 2, the
    nodal interpolant of e^2 being exact)."""
    P = 2
    R = ref(P)
    m = meshgen.periodic_square(6)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    q = meshgen.freestream_state(0.5, 10.0)
    o = orc.Oracle(m, P, x, y, freestream=q)
    U = meshgen.uniform((m.K, R.Np), q)
    assert dgn.entropy_error(o, U, q) == 0.0
    a = 1.3
    rho0, u0, v0 = q[0], q[1] / q[0], q[2] / q[0]
    p0 = (G - 1) * (q[3] - 0.5 * rho0 * (u0 * u0 + v0 * v0))
    U2 = meshgen.uniform((m.K, R.Np), prim(a * rho0, u0, v0, p0))
    assert dgn.entropy_error(o, U2, q) == pytest.approx(abs(a ** -G - 1), rel=1e-13)
    U3 = np.stack([np.full_like(x, rho0), 0 * x, 0 * x, p0 * (1 + x / 10) / (G - 1)], 1)
    assert dgn.entropy_error(o, U3, q) == pytest.approx(1 / math.sqrt(3), rel=1e-12)


def _green_area(o, R, ks, fs):
    """Area enclosed by the wall's nodal face polynomials, by Green's theorem
    (area = -1/2 oint (x dy - y dx) over the faces traversed with the fluid
    on the left), with a 20-point Gauss rule in each face parameter."""
    from numpy.polynomial import polynomial as npoly
    tg, wg = np.polynomial.legendre.leggauss(20)
    area = 0.0
    tpar = R.face_parameters()
    for k, f in zip(ks, fs):
        v = R.Fmask[f]
        px = npoly.polyfit(tpar[f], o.x[k, v], R.P)
        py = npoly.polyfit(tpar[f], o.y[k, v], R.P)
        X, Y = npoly.polyval(tg, px), npoly.polyval(tg, py)
        dX, dY = npoly.polyval(tg, npoly.polyder(px)), npoly.polyval(tg, npoly.polyder(py))
        area -= 0.5 * float((wg * (X * dY - Y * dX)).sum())
    return area


@pytest.mark.parametrize("P", [2, 3, 5])
def test_wall_force_of_uniform_and_linear_pressure(P):
    """Uniform pressure on a closed body: no force.  p = p0 + b y: the force
    on the body is the buoyancy (0, -b A), A the area the wall's face
    polynomials enclose (computed independently by Green's theorem)."""
    R = ref(P)
    m = meshgen.cylinder_annulus(24, 6, jitter=0.1, seed=5)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    o = orc.Oracle(m, P, x, y)
    U = np.stack([np.ones_like(x), 0 * x, 0 * x, np.full_like(x, 2.5)], 1)
    Fx, Fy = dgn.wall_force(o, U)
    assert abs(Fx) < 1e-13 and abs(Fy) < 1e-13
    b = 0.37
    U[:, 3] = (1.0 + b * y) / (G - 1)
    Fx, Fy = dgn.wall_force(o, U)
    ks, fs = np.nonzero(m.bc == meshgen.BC_WALL)
    A = _green_area(o, R, ks, fs)
    assert abs(A - math.pi) < 1e-3
    assert abs(Fx) < 1e-13
    assert Fy == pytest.approx(-b * A, rel=1e-12)


@pytest.mark.parametrize("alpha", [0.0, 1.25, 30.0])
def test_lift_and_drag_rotate_with_the_freestream(alpha):
    """A pressure field p = p0 + b y gives the force (0, -b A); with the
    freestream at angle alpha, C_L = -b A cos(alpha) / (q c) and
    C_D = -b A sin(alpha) / (q c)."""
    P = 3
    R = ref(P)
    m = meshgen.cylinder_annulus(24, 6, jitter=0.1, seed=5)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    q = meshgen.freestream_state(0.6, alpha)
    o = orc.Oracle(m, P, x, y, freestream=q)
    b = 0.2
    U = np.stack([np.ones_like(x), 0 * x, 0 * x, (1.0 + b * y) / (G - 1)], 1)
    ks, fs = np.nonzero(m.bc == meshgen.BC_WALL)
    A = _green_area(o, R, ks, fs)
    qdyn = 0.5 * 1.0 * 0.6 ** 2
    CL, CD = dgn.lift_drag(o, U, q, chord=2.0)
    a = math.radians(alpha)
    assert CL == pytest.approx(-b * A * math.cos(a) / (qdyn * 2.0), rel=1e-12, abs=1e-13)
    assert CD == pytest.approx(-b * A * math.sin(a) / (qdyn * 2.0), rel=1e-12, abs=1e-13)


def test_critical_pressure_coefficient_is_sonic():
    """At C_p = C_p* the isentropic local Mach number is one."""
    for M in (0.6, 0.8, 0.85):
        cp = dgn.critical_cp(M)
        p_over_p0 = 1 + 0.5 * G * M * M * cp
        # isentropic: p/p0 = ((1 + (g-1)/2 M^2) / (1 + (g-1)/2 Ml^2))^(g/(g-1))
        ml2 = ((1 + 0.5 * (G - 1) * M * M) / p_over_p0 ** ((G - 1) / G) - 1) / (0.5 * (G - 1))
        assert ml2 == pytest.approx(1.0, rel=1e-12)


def test_shock_position_is_the_upward_crossing():
    """A wall pressure with C_p = C_p* + 2 (x - 0.6) on the upper surface
    crosses C_p* upwards at x = 0.6 exactly (the interpolation is linear in
    x); a pressure that stays above C_p* has no shock; with an earlier
    crossing near the leading edge the shock is still the last one."""
    P = 3
    R = ref(P)
    m = meshgen.naca4_ogrid(60, 6, jitter=0.0)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    M = 0.8
    q = meshgen.freestream_state(M, 1.25)
    o = orc.Oracle(m, P, x, y, freestream=q)
    rho0 = q[0]
    u0, v0 = q[1] / rho0, q[2] / rho0
    p0 = (G - 1) * (q[3] - 0.5 * rho0 * (u0 * u0 + v0 * v0))
    qdyn = 0.5 * rho0 * (u0 * u0 + v0 * v0)
    cstar = dgn.critical_cp(M)
    p = p0 + qdyn * (cstar + 2.0 * (x - 0.6))
    U = np.stack([np.ones_like(x), 0 * x, 0 * x, p / (G - 1)], 1)
    assert dgn.shock_position(o, U, q, M) == pytest.approx(0.6, abs=1e-12)
    p = p0 + qdyn * (cstar + 0.1 + 0 * x)
    U[:, 3] = p / (G - 1)
    assert math.isnan(dgn.shock_position(o, U, q, M))
    # a wiggle near the leading edge (up through C_p* at x = 0.1, down at
    # 0.2) before the shock at 0.6: the shock is the last upward crossing
    cp = np.where(x < 0.15, cstar + (x - 0.1),
                  np.where(x < 0.2, cstar + 0.05 - 2.0 * (x - 0.15), cstar + 2.0 * (x - 0.6)))
    U[:, 3] = (p0 + qdyn * cp) / (G - 1)
    xs, cs = dgn.upper_surface_cp(o, U, q)
    rising = [i for i in range(xs.size - 1) if cs[i] < cstar <= cs[i + 1]]
    assert len(rising) >= 2
    assert dgn.shock_position(o, U, q, M) == pytest.approx(0.6, abs=1e-9)


# -- node family: blending exponents (R3) -------------------------------------

def lebesgue(P, alpha, n=150):
    r, s = refelem.nodes(P, alpha)
    V = refelem.vandermonde(P, r, s)
    pts = np.array([(-1 + 2 * j / n, -1 + 2 * i / n) for i in range(n + 1) for j in range(n + 1 - i)])
    lag = refelem.vandermonde(P, pts[:, 0], pts[:, 1]) @ np.linalg.inv(V)
    return float(np.abs(lag).sum(axis=1).max())


@pytest.mark.slow
@pytest.mark.parametrize("P,published", [(3, 2.11), (4, 2.66), (5, 3.12)])
def test_blending_exponent_minimises_lebesgue_constant(P, published):
    """The table's alpha is (within 0.1%) the Lebesgue-optimal blending
    exponent on [0, 1.5], and the Lebesgue constant it gives rounds to the
    value Warburton (2006) tabulates for alpha-optimised warp-and-blend
    nodes.  A typo in the table (0.2751 -> 2.751 or 0.1001 -> 1.001) fails."""
    lam = lebesgue(P, refelem.ALPHA_OPT[P])
    best = min(lebesgue(P, a) for a in np.linspace(0.0, 1.5, 31))
    assert lam <= best * 1.001
    assert round(lam, 2) == published
