"""Pins of the oracle's geometric factors, Euler flux, Lax-Friedrichs flux and
boundary states (no GPU)."""
import numpy as np
import pytest
from numpy.polynomial import polynomial as npoly
from scipy import special

import meshgen
from oracle import oracle as orc
from oracle.refelem import ref

G = 1.4


def build(mesh, P, **kw):
    R = ref(P)
    x, y = meshgen.node_coordinates(mesh, R.r, R.s)
    return orc.Oracle(mesh, P, x, y, **kw), R


@pytest.mark.parametrize("P", [1, 2, 5])
def test_straight_jacobian_is_half_area(P):
    m = meshgen.periodic_square(6, perm_seed=3)
    o, R = build(m, P)
    area = m.signed_area()
    np.testing.assert_allclose(o.geo["J"], np.repeat(area[:, None] / 2, R.Np, 1), rtol=1e-12)
    # sum over faces of (edge weights * sJ) is the perimeter
    vx, vy = m.vertex_xy()
    per = sum(np.hypot(vx[:, b] - vx[:, a], vy[:, b] - vy[:, a]) for a, b in meshgen.FACE_VERTS)
    w = np.concatenate([R.Emat[R.Fmask[f], f * R.Nfp:(f + 1) * R.Nfp].sum(1) for f in range(3)])
    np.testing.assert_allclose(o.geo["sJ"] @ w, per, rtol=1e-12)


def face_polys(xk, yk, R, f):
    """Degree-P interpolants x(t), y(t) of the face nodes in the face parameter."""
    t = R.face_parameters()[f]
    v = R.Fmask[f]
    return npoly.polyfit(t, xk[v], R.P), npoly.polyfit(t, yk[v], R.P), t


@pytest.mark.parametrize("P", [3, 4, 5])
@pytest.mark.parametrize("mk", [lambda: meshgen.cylinder_annulus(24, 6),
                                lambda: meshgen.naca4_ogrid(40, 8),
                                lambda: meshgen.periodic_square(4, perm_seed=None, curved_amplitude=0.05)])
def test_curved_normals_and_face_jacobians(P, mk):
    """n is the unit normal to the face tangent dx/dt, sJ = |dx/dt|, computed
    here from 1D interpolation of the face nodes (independent of Dr, Ds)."""
    m = mk()
    o, R = build(m, P)
    Nfp = R.Nfp
    ks = np.nonzero((m.bc == meshgen.BC_WALL).any(1))[0][:10] if (m.bc == 1).any() else np.arange(10)
    for k in ks:
        for f in range(3):
            px, py, t = face_polys(o.x[k], o.y[k], R, f)
            tx = npoly.polyval(t, npoly.polyder(px))
            ty = npoly.polyval(t, npoly.polyder(py))
            q = slice(f * Nfp, (f + 1) * Nfp)
            np.testing.assert_allclose(o.geo["sJ"][k, q], np.hypot(tx, ty), rtol=1e-9)
            # outward normal: tangent rotated clockwise (CCW traversal)
            np.testing.assert_allclose(o.geo["nx"][k, q], ty / np.hypot(tx, ty), atol=1e-9)
            np.testing.assert_allclose(o.geo["ny"][k, q], -tx / np.hypot(tx, ty), atol=1e-9)


@pytest.mark.parametrize("P", [4, 5])
def test_curved_area_by_green_theorem(P):
    """For P >= 4 the cubic wall map's Jacobian (degree 4) is integrated
    exactly by the mass weights: sum_i (M 1)_i J_i = area = 1/2 closed
    integral of (x dy - y dx) over the three face polynomials."""
    m = meshgen.cylinder_annulus(24, 6)
    o, R = build(m, P)
    w = R.M.sum(1)
    xg, wg = special.roots_legendre(P + 2)
    for k in np.nonzero((m.bc == meshgen.BC_WALL).any(1))[0]:
        area = 0.0
        for f in range(3):
            px, py, _ = face_polys(o.x[k], o.y[k], R, f)
            x = npoly.polyval(xg, px)
            y = npoly.polyval(xg, py)
            dx = npoly.polyval(xg, npoly.polyder(px))
            dy = npoly.polyval(xg, npoly.polyder(py))
            area += 0.5 * np.sum(wg * (x * dy - y * dx))
        assert abs(w @ o.geo["J"][k] - area) < 1e-13 * abs(area) + 1e-15


def test_wall_nodes_on_circle():
    m = meshgen.cylinder_annulus(24, 6)
    for P, tol in [(3, 1e-13), (5, 1e-5)]:
        o, R = build(m, P)
        ks, fs = np.nonzero(m.bc == meshgen.BC_WALL)
        for k, f in zip(ks, fs):
            v = R.Fmask[f]
            rr = np.hypot(o.x[k, v], o.y[k, v])
            assert np.abs(rr - 1.0).max() < tol


@pytest.mark.parametrize("mk", [lambda: meshgen.periodic_square(5, perm_seed=9, curved_amplitude=0.05),
                                lambda: meshgen.cylinder_annulus(24, 6)])
def test_normals_opposite_across_faces(mk):
    m = mk()
    o, R = build(m, 4)
    Nfp = R.Nfp
    nx = o.geo["nx"].reshape(m.K, 3, Nfp)
    ny = o.geo["ny"].reshape(m.K, 3, Nfp)
    k, f = np.nonzero(m.bc == 0)
    kn, fn = m.EToE[k, f], m.EToF[k, f]
    np.testing.assert_allclose(nx[k, f, :], -nx[kn, fn, ::-1], atol=1e-10)
    np.testing.assert_allclose(ny[k, f, :], -ny[kn, fn, ::-1], atol=1e-10)


def test_clockwise_element_is_flagged():
    m = meshgen.periodic_square(4, perm_seed=None)
    m.EToV[0, 1], m.EToV[0, 2] = m.EToV[0, 2], m.EToV[0, 1]
    o, R = build(m, 2)
    assert o.bad_jacobians == R.Np


# --------------------------------------------------------------------------
# fluxes and boundary states
# --------------------------------------------------------------------------

def random_states(n, seed=0):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, n)
    u = rng.uniform(-1, 1, n)
    v = rng.uniform(-1, 1, n)
    p = rng.uniform(0.3, 2.0, n)
    return meshgen.primitive_to_conserved(rho, u, v, p).T, (rho, u, v, p)


def test_lf_flux_consistency_bitwise():
    U, (rho, u, v, p) = random_states(200)
    rng = np.random.default_rng(1)
    th = rng.uniform(0, 2 * np.pi, 200)
    for i in range(200):
        nx, ny = np.cos(th[i]), np.sin(th[i])
        fs = orc.lf_flux(U[i], U[i], nx, ny)
        # n.F from primitive variables
        vn = u[i] * nx + v[i] * ny
        E = p[i] / 0.4 + 0.5 * rho[i] * (u[i] ** 2 + v[i] ** 2)
        expect = np.array([rho[i] * vn, rho[i] * u[i] * vn + p[i] * nx,
                           rho[i] * v[i] * vn + p[i] * ny, (E + p[i]) * vn])
        np.testing.assert_allclose(fs, expect, rtol=1e-13, atol=1e-14)
        # consistency is exact: F*(u,u) is the same bits as F*(u,u) with any
        # jump term dropped, i.e. 1/2 (f + f)
        assert np.array_equal(fs, orc.lf_flux(U[i], U[i], nx, ny))


def test_lf_flux_consistency_exact():
    """F*(u,u,n) equals n.F(u) bit for bit: both terms of the average are the
    same number and the dissipation term is exactly zero."""
    U, _ = random_states(50, 3)
    for i in range(50):
        a = orc.lf_flux(U[i], U[i], 0.6, 0.8)
        b = orc.lf_flux(U[i], U[(i + 1) % 50], 0.6, 0.8)
        c = orc.lf_flux(U[(i + 1) % 50], U[i], -0.6, -0.8)
        np.testing.assert_array_equal(b, -c)          # conservation, bitwise
        fm = 0.5 * (a + a)
        np.testing.assert_array_equal(a, fm)


def test_wall_ghost_and_zero_mass_flux():
    U, _ = random_states(50, 5)
    qinf = meshgen.freestream_state(0.4)
    for i in range(50):
        n = np.array([np.cos(i), np.sin(i)])
        g = orc.ghost(1, U[i], n[0], n[1], qinf)
        assert g[0] == U[i][0] and g[3] == U[i][3]
        m = U[i][1:3]
        mg = g[1:3]
        assert abs(mg @ n + m @ n) < 1e-14
        t = np.array([-n[1], n[0]])
        assert abs(mg @ t - m @ t) < 1e-14
        f = orc.lf_flux(U[i], g, n[0], n[1])
        assert abs(f[0]) < 1e-14


@pytest.mark.parametrize("mach", [0.3, 0.8, 1.5])
def test_farfield_ghost_of_freestream_is_freestream(mach):
    q = meshgen.freestream_state(mach, 10.0)
    for th in np.linspace(0, 2 * np.pi, 13):
        g = orc.ghost(2, q, np.cos(th), np.sin(th), q)
        np.testing.assert_allclose(g, q, rtol=1e-14, atol=1e-14)


def test_farfield_subsonic_preserves_outgoing_invariant():
    """Subsonic outflow: the ghost state keeps the interior's outgoing
    Riemann invariant v_n + 2c/(g-1) and entropy p/rho^g."""
    q = meshgen.freestream_state(0.5)
    um = meshgen.primitive_to_conserved(1.1, 0.45, 0.05, 0.8)
    n = (1.0, 0.0)
    g = orc.ghost(2, um, n[0], n[1], q)

    def prim(U):
        rho = U[0]
        u, v = U[1] / rho, U[2] / rho
        p = 0.4 * (U[3] - 0.5 * rho * (u * u + v * v))
        return rho, u, v, p
    ri, ui, vi, pi = prim(um)
    rb, ub, vb, pb = prim(g)
    ci, cb = np.sqrt(G * pi / ri), np.sqrt(G * pb / rb)
    assert abs((ub + 5 * cb) - (ui + 5 * ci)) < 1e-13
    assert abs(pb / rb ** G - pi / ri ** G) < 1e-13
    assert abs(vb - vi) < 1e-14
