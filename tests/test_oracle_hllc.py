"""Pins of the oracle's HLLC flux (no GPU): consistency, conservation,
exact resolution of contact discontinuities, supersonic upwinding, Toro's
second (flux-difference) form of the same flux, and the whole discretisation
with HLLC (freestream preservation, convergence)."""
import math

import numpy as np
import pytest

import meshgen
from oracle import oracle as orc
from oracle.refelem import ref

G = 1.4


def prim(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)])


def phys_flux(u, nx, ny):
    rho, vx, vy = u[0], u[1] / u[0], u[2] / u[0]
    p = (G - 1) * (u[3] - 0.5 * rho * (vx * vx + vy * vy))
    vn = vx * nx + vy * ny
    return np.array([rho * vn, u[1] * vn + p * nx, u[2] * vn + p * ny, (u[3] + p) * vn]), p, vn


def toro_second_form(ul, ur, nx, ny):
    """HLLC in Toro's flux form (10.75, adapted to a face normal):
    F*_K = [S* (S_K U_K - F_K) + S_K (p_K + rho_L (S_L - u_L)(S* - u_L)) D*] / (S_K - S*),
    D* = (0, n_x, n_y, S*); the same flux as the star-state form in exact
    arithmetic."""
    fl, pl, ul_n = phys_flux(ul, nx, ny)
    fr, pr, ur_n = phys_flux(ur, nx, ny)
    cl = math.sqrt(G * pl / ul[0])
    cr = math.sqrt(G * pr / ur[0])
    SL = min(ul_n - cl, ur_n - cr)
    SR = max(ul_n + cl, ur_n + cr)
    rl, rr = ul[0], ur[0]
    Ss = (pr - pl + rl * ul_n * (SL - ul_n) - rr * ur_n * (SR - ur_n)) / (rl * (SL - ul_n) - rr * (SR - ur_n))
    pLR = 0.5 * (pl + pr + rl * (SL - ul_n) * (Ss - ul_n) + rr * (SR - ur_n) * (Ss - ur_n))
    D = np.array([0.0, nx, ny, Ss])
    if SL >= 0:
        return fl
    if Ss >= 0:
        return (Ss * (SL * ul - fl) + SL * pLR * D) / (SL - Ss)
    if SR > 0:
        return (Ss * (SR * ur - fr) + SR * pLR * D) / (SR - Ss)
    return fr


STATES = [
    (prim(1.0, 0.3, -0.2, 1.0), prim(0.8, 0.1, 0.4, 0.7)),
    (prim(1.2, -0.5, 0.3, 0.9), prim(1.0, -0.6, 0.1, 1.3)),
    (prim(0.6, 0.9, 0.0, 0.5), prim(1.4, -0.2, 0.2, 1.6)),
    (prim(1.0, 0.0, 0.0, 1.0), prim(0.125, 0.0, 0.0, 0.1)),         # Sod
]
NORMALS = [(1.0, 0.0), (0.6, 0.8), (-math.sqrt(0.5), math.sqrt(0.5))]


@pytest.mark.parametrize("ul,ur", STATES)
@pytest.mark.parametrize("n", NORMALS)
def test_hllc_equals_toro_flux_form(ul, ur, n):
    got = orc.hllc_flux(ul, ur, *n)
    want = toro_second_form(ul, ur, *n)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("ul,ur", STATES)
@pytest.mark.parametrize("n", NORMALS)
def test_hllc_consistency_and_conservation(ul, ur, n):
    nx, ny = n
    f, _, _ = phys_flux(ul, nx, ny)
    np.testing.assert_allclose(orc.hllc_flux(ul, ul, nx, ny), f, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(orc.hllc_flux(ul, ur, nx, ny), -orc.hllc_flux(ur, ul, -nx, -ny),
                               rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n", NORMALS)
def test_hllc_resolves_contacts_exactly(n):
    """Equal pressure and velocity, different density: the exact flux is
    that of the upwind side (no mass crosses a stationary contact).  The
    Lax-Friedrichs flux diffuses it."""
    nx, ny = n
    ul, ur = prim(1.0, 0.0, 0.0, 1.0), prim(0.3, 0.0, 0.0, 1.0)
    f = orc.hllc_flux(ul, ur, nx, ny)
    np.testing.assert_allclose(f, [0.0, nx, ny, 0.0], atol=1e-15)
    assert abs(orc.lf_flux(ul, ur, nx, ny)[0]) > 0.1
    # moving contact: velocity (0.4, -0.3); upwind side decides
    ul, ur = prim(1.0, 0.4, -0.3, 1.0), prim(0.3, 0.4, -0.3, 1.0)
    vn = 0.4 * nx - 0.3 * ny
    up = ul if vn > 0 else ur
    want, _, _ = phys_flux(up, nx, ny)
    np.testing.assert_allclose(orc.hllc_flux(ul, ur, nx, ny), want, rtol=1e-13, atol=1e-14)


def test_hllc_upwinds_supersonic_flow():
    ul, ur = prim(1.0, 3.0, 0.5, 1.0), prim(0.7, 2.5, 0.1, 0.6)      # v_n > c on both sides
    f, _, _ = phys_flux(ul, 1.0, 0.0)
    np.testing.assert_array_equal(orc.hllc_flux(ul, ur, 1.0, 0.0), f)
    f, _, _ = phys_flux(ur, -1.0, 0.0)
    np.testing.assert_array_equal(orc.hllc_flux(ul, ur, -1.0, 0.0), f)


@pytest.mark.parametrize("P", [1, 3, 5])
def test_hllc_rhs_preserves_freestream_on_curved_meshes(P):
    R = ref(P)
    q = meshgen.freestream_state(0.5, 20.0)
    m = meshgen.periodic_square(5, perm_seed=11, curved_amplitude=0.05)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    o = orc.Oracle(m, P, x, y, freestream=q, riemann="hllc")
    assert np.abs(o.rhs(meshgen.uniform((m.K, R.Np), q))).max() < 1e-12
    m = meshgen.cylinder_annulus(20, 5, inner_bc=meshgen.BC_FARFIELD)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    o = orc.Oracle(m, P, x, y, freestream=q, riemann="hllc")
    assert np.abs(o.rhs(meshgen.uniform((m.K, R.Np), q))).max() < 1e-12


def test_hllc_rhs_differs_from_lf_and_conserves():
    R = ref(3)
    m = meshgen.periodic_square(8)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    # a density step (a contact): the two fluxes differ where the traces jump
    rho = np.where(x < 5.0, 1.0, 0.6)
    U = meshgen.primitive_to_conserved(rho, 0.5 + 0 * x, 0.2 + 0 * x, 1.0 + 0 * x)
    q = np.array([1.0, 1.0, 0.0, 1.0 / 0.4 + 0.5])
    a = orc.Oracle(m, 3, x, y, freestream=q).rhs(U)
    o = orc.Oracle(m, 3, x, y, freestream=q, riemann="hllc")
    b = o.rhs(U)
    assert np.abs(a - b).max() > 1e-4
    U1, _ = o.run(U, 20)
    np.testing.assert_allclose(o.totals(U1), o.totals(U), rtol=1e-13, atol=1e-12)


@pytest.mark.slow
@pytest.mark.parametrize("P", [1, 2, 3])
def test_hllc_entropy_wave_converges(P):
    """Density wave rho = 1 + 0.2 sin(2 pi (x + y)/10) advected at (1, 1)
    with uniform p: exact solution rho(x - t, y - t); order >= P + 1 - 0.3."""
    R = ref(P)
    T = 1.0
    errs = []
    for N in (4, 8, 16):
        m = meshgen.periodic_square(N, perm_seed=None)
        x, y = meshgen.node_coordinates(m, R.r, R.s)

        def state(t):
            rho = 1.0 + 0.2 * np.sin(2 * np.pi * (x + y - 2 * t) / 10.0)
            return meshgen.primitive_to_conserved(rho, 1.0 + 0 * x, 1.0 + 0 * x, 1.0 + 0 * x)
        q = prim(1.0, 1.0, 1.0, 1.0)
        o = orc.Oracle(m, P, x, y, freestream=q, riemann="hllc", cfl=0.3)
        U0 = state(0.0)
        dt, _ = o.dt(U0)
        n = int(math.ceil(T / dt))
        U, info = o.run(U0, n, dt=T / n)
        errs.append(np.abs(U[:, 0] - state(info["t"])[:, 0]).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] >= P + 1 - 0.3, rates
