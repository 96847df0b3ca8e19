"""Synthetic-input generators: connectivity, orientation, seeds, watertight
curving (no GPU)."""
import numpy as np
import pytest

import meshgen
from meshgen import BC_FARFIELD, BC_WALL
from oracle.refelem import ref


def reciprocal(m):
    k = np.arange(m.K)[:, None]
    f = np.arange(3)[None, :]
    return (m.EToE[m.EToE, m.EToF] == k).all() and (m.EToF[m.EToE, m.EToF] == f).all()


@pytest.mark.parametrize("mk", [
    lambda: meshgen.periodic_square(6),
    lambda: meshgen.periodic_square(5, perm_seed=None, curved_amplitude=0.05),
    lambda: meshgen.cylinder_annulus(24, 6),
    lambda: meshgen.naca4_ogrid(40, 8),
])
def test_connectivity_and_orientation(mk):
    m = mk()
    assert reciprocal(m)
    assert (m.signed_area() > 0).all()
    bnd = m.bc != 0
    k, f = np.nonzero(bnd)
    assert (m.EToE[k, f] == k).all() and (m.EToF[k, f] == f).all()
    k, f = np.nonzero(~bnd)
    assert (m.EToE[k, f] != k).all()


def test_sizes_and_boundaries():
    assert meshgen.periodic_square(16).K == 512
    c = meshgen.cylinder_annulus()
    assert c.K == 20000
    assert (c.bc == BC_WALL).sum() == 200 and (c.bc == BC_FARFIELD).sum() == 200
    a = meshgen.naca4_ogrid()
    assert a.K == 120000 and (a.bc == BC_WALL).sum() == 600


def test_seeds_are_reproducible():
    a = meshgen.periodic_square(8)
    b = meshgen.periodic_square(8)
    np.testing.assert_array_equal(a.EToV, b.EToV)
    np.testing.assert_array_equal(a.VX, b.VX)
    c = meshgen.periodic_square(8, jitter_seed=1)
    assert not np.array_equal(a.VX, c.VX)


def test_permutation_keeps_geometry():
    a = meshgen.periodic_square(6, perm_seed=None)
    b = meshgen.periodic_square(6, perm_seed=4772)
    perm = np.random.default_rng(4772).permutation(a.K)
    np.testing.assert_array_equal(b.EToV, a.EToV[perm])
    assert reciprocal(b)


@pytest.mark.parametrize("P", [1, 3, 5])
@pytest.mark.parametrize("mk", [
    lambda: meshgen.cylinder_annulus(24, 6),
    lambda: meshgen.naca4_ogrid(40, 8),
    lambda: meshgen.periodic_square(5, perm_seed=7, curved_amplitude=0.05),
])
def test_curved_meshes_are_watertight(P, mk):
    """Shared face nodes of neighbours coincide (modulo the period)."""
    m = mk()
    R = ref(P)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    Nfp = P + 1
    Lp = m.info.get("periodic")
    for f in range(3):
        ks = np.nonzero(m.bc[:, f] == 0)[0]
        kn = m.EToE[ks, f]
        fn = m.EToF[ks, f]
        for j in range(Nfp):
            vm = R.Fmask[f, j]
            vp = R.Fmask[fn, Nfp - 1 - j]
            dx = x[ks, vm] - x[kn, vp]
            dy = y[ks, vm] - y[kn, vp]
            if Lp:
                dx = dx - Lp[0] * np.round(dx / Lp[0])
                dy = dy - Lp[1] * np.round(dy / Lp[1])
            assert np.abs(dx).max() < 1e-12 and np.abs(dy).max() < 1e-12


def test_vortex_state_is_radially_balanced():
    """The isentropic vortex satisfies dp/dr = rho u_theta^2 / r."""
    r = np.linspace(0.1, 3.0, 50)
    x = 5.0 + r
    y = 5.0 + 0 * r
    h = 1e-6
    def prim(xx):
        U = meshgen.isentropic_vortex(xx, y)
        rho = U[0]
        p = 0.4 * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / rho)
        return rho, U[2] / rho, p
    rho, vt, _ = prim(x)
    dp = (prim(x + h)[2] - prim(x - h)[2]) / (2 * h)
    np.testing.assert_allclose(dp, rho * vt ** 2 / r, rtol=1e-6, atol=1e-9)


def test_cylinder_potential_start():
    """Zero normal velocity on the wall, freestream far away, constant
    total enthalpy (c^2/(gamma-1) + |v|^2/2), and no divergence."""
    th = np.linspace(0, 2 * np.pi, 37)
    U = meshgen.cylinder_potential(np.cos(th), np.sin(th), 0.6)
    rho, u, v = U[0], U[1] / U[0], U[2] / U[0]
    np.testing.assert_allclose(u * np.cos(th) + v * np.sin(th), 0, atol=1e-14)
    far = meshgen.cylinder_potential(np.array([1e6]), np.array([3e5]), 0.6)
    np.testing.assert_allclose(far[:, 0], meshgen.freestream_state(0.6), rtol=1e-9, atol=1e-9)
    x, y = (a.ravel() for a in np.meshgrid(np.linspace(1.5, 4, 7), np.linspace(-3, 3, 7)))
    U = meshgen.cylinder_potential(x, y, 0.6)
    rho, u, v = U[0], U[1] / U[0], U[2] / U[0]
    p = 0.4 * (U[3] - 0.5 * rho * (u * u + v * v))
    H = 1.4 * p / rho / 0.4 + 0.5 * (u * u + v * v)
    np.testing.assert_allclose(H, 1 / 0.4 + 0.18, rtol=1e-13)
    h = 1e-5
    div = ((meshgen.cylinder_potential(x + h, y, 0.6)[1] / meshgen.cylinder_potential(x + h, y, 0.6)[0]
            - meshgen.cylinder_potential(x - h, y, 0.6)[1] / meshgen.cylinder_potential(x - h, y, 0.6)[0])
           + (meshgen.cylinder_potential(x, y + h, 0.6)[2] / meshgen.cylinder_potential(x, y + h, 0.6)[0]
              - meshgen.cylinder_potential(x, y - h, 0.6)[2] / meshgen.cylinder_potential(x, y - h, 0.6)[0])) / (2 * h)
    np.testing.assert_allclose(div, 0, atol=1e-8)


def test_wall_damped_start():
    """At rest on the wall points, the freestream far from them, the
    freestream density and pressure everywhere."""
    r, s = np.array([-1.0, 1.0, -1.0]), np.array([-1.0, -1.0, 1.0])
    case = meshgen.make_case("airfoil", r, s, scale=0.01, start="damped")
    q = case.freestream
    U = case.U0
    rho, u, v = U[:, 0], U[:, 1] / U[:, 0], U[:, 2] / U[:, 0]
    p = 0.4 * (U[:, 3] - 0.5 * rho * (u * u + v * v))
    np.testing.assert_allclose(rho, 1.0, rtol=1e-15)
    np.testing.assert_allclose(p, 1 / 1.4, rtol=1e-13)
    # P = 1 nodes are the vertices: the wall vertices start at rest
    k, f = np.nonzero(case.mesh.bc == meshgen.BC_WALL)
    wall_nodes = np.array([meshgen.FACE_VERTS[ff][0] for ff in f])
    np.testing.assert_allclose(u[k, wall_nodes], 0.0, atol=1e-14)
    np.testing.assert_allclose(v[k, wall_nodes], 0.0, atol=1e-14)
    far = np.hypot(case.x, case.y) > 10
    np.testing.assert_allclose(u[far], q[1], rtol=1e-12)
    np.testing.assert_allclose(v[far], q[2], rtol=1e-12)
    with pytest.raises(ValueError):
        meshgen.make_case("airfoil", r, s, scale=0.01, start="nonsense")


@pytest.mark.parametrize("alpha", [0.0, 1.25, 4.0])
def test_airfoil_panel_solution(alpha):
    """Zero normal velocity at the panel midpoints, the freestream far away,
    lift from the circulation (Kutta-Joukowski) within 2% of thin-airfoil
    theory with the thickness correction, 2 pi alpha (1 + 0.77 t), and
    no lift at zero incidence."""
    import math
    panels, q, g, Vinf = meshgen.airfoil_panels(0.8, alpha)
    ax, ay, bx, by = panels
    L = np.hypot(bx - ax, by - ay)
    nx, ny = (by - ay) / L, -(bx - ax) / L
    u, v = meshgen.airfoil_velocity(0.5 * (ax + bx) + 1e-9 * nx, 0.5 * (ay + by) + 1e-9 * ny, panels, q, g, Vinf,
                                    standoff=0.0)
    assert np.abs(u * nx + v * ny).max() < 1e-6
    uf, vf = meshgen.airfoil_velocity(np.array([3e4]), np.array([-2e4]), panels, q, g, Vinf)
    np.testing.assert_allclose([uf[0], vf[0]], Vinf, atol=1e-4)
    CL = -2 * g * L.sum() / math.hypot(*Vinf)
    thin = 2 * math.pi * math.radians(alpha) * (1 + 0.77 * 0.12)
    if alpha == 0.0:
        assert abs(CL) < 1e-10
    else:
        assert abs(CL / thin - 1) < 0.02, (CL, thin)


def test_airfoil_potential_start():
    """Freestream far away; constant total enthalpy; the airfoil case's
    potential start is that state at the mesh nodes."""
    x = np.array([0.5, -0.3, 2.0, 40.0])
    y = np.array([0.2, 0.05, -0.4, 30.0])
    U = meshgen.airfoil_potential(x, y, 0.6, 1.25)
    rho, u, v = U[0], U[1] / U[0], U[2] / U[0]
    p = 0.4 * (U[3] - 0.5 * rho * (u * u + v * v))
    H = 1.4 * p / rho / 0.4 + 0.5 * (u * u + v * v)
    np.testing.assert_allclose(H, 1 / 0.4 + 0.18, rtol=1e-13)
    np.testing.assert_allclose(U[:, -1], meshgen.freestream_state(0.6, 1.25), rtol=1e-3, atol=1e-3)
    r, s = np.array([-1.0, 1.0, -1.0]), np.array([-1.0, -1.0, 1.0])
    case = meshgen.make_case("airfoil", r, s, scale=0.01, start="potential", mach=0.6)
    np.testing.assert_allclose(case.U0, meshgen.airfoil_potential(case.x, case.y, 0.6, 1.25), rtol=0, atol=0)
