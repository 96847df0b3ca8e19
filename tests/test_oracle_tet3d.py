"""Pins of the 3D tetrahedral oracle (no GPU): reference operators against
exact polynomial calculus and an independent cubature, geometry and
connectivity invariants, freestream preservation, conservation, exactness
on linear data, rotation symmetry and convergence on an exact solution."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import tet3d as T


def collapsed_tet_rule(n):
    """Gauss rule on the reference tetrahedron from the collapsed (Duffy)
    map: n^3 points, exact to degree 2n - 1 (Gauss-Jacobi in the collapsed
    directions)."""
    a, wa = special.roots_legendre(n)
    b, wb = special.roots_jacobi(n, 1.0, 0.0)
    c, wc = special.roots_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    W = (wa[:, None, None] * wb[None, :, None] * wc[None, None, :]) / 8.0
    r = (1 + A) * (1 - B) * (1 - C) / 4 - 1
    s = (1 + B) * (1 - C) / 2 - 1
    t = C
    return r.ravel(), s.ravel(), t.ravel(), W.ravel() * 8.0 / 8.0


def collapsed_tri_rule(n):
    a, wa = special.roots_legendre(n)
    b, wb = special.roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(a, b, indexing="ij")
    u = (1 + A) * (1 - B) / 4
    v = (1 + B) / 2
    W = np.outer(wa, wb) / 8.0       # unit right triangle (area 1/2)
    return u.ravel(), v.ravel(), W.ravel()


def random_poly(P, rng):
    terms = [(a, b, c, rng.standard_normal()) for a in range(P + 1) for b in range(P + 1 - a)
             for c in range(P + 1 - a - b)]

    def f(r, s, t):
        return sum(k * r ** a * s ** b * t ** c for a, b, c, k in terms)

    def df(r, s, t, d):
        out = 0.0
        for a, b, c, k in terms:
            e = (a, b, c)[d]
            if e == 0:
                continue
            ex = [a, b, c]
            ex[d] -= 1
            out = out + k * e * r ** ex[0] * s ** ex[1] * t ** ex[2]
        return out + 0 * r
    return f, df


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_reference_tetrahedron_operators(P):
    R = T.ref(P)
    assert R.Np == (P + 1) * (P + 2) * (P + 3) // 6 and R.Nfp == (P + 1) * (P + 2) // 2
    rng = np.random.default_rng(P)
    f, df = random_poly(P, rng)
    u = f(R.r, R.s, R.t)
    for D, d in ((R.Dr, 0), (R.Ds, 1), (R.Dt, 2)):
        np.testing.assert_allclose(D @ u, df(R.r, R.s, R.t, d), atol=1e-10 * (1 + np.abs(u).max()))
    # mass matrix against an independent cubature of exact degree >= 2P
    g, _ = random_poly(P, rng)
    v = g(R.r, R.s, R.t)
    r, s, t, w = collapsed_tet_rule(P + 2)
    exact = np.sum(w * f(r, s, t) * g(r, s, t))
    assert abs(u @ R.M @ v - exact) < 1e-11 * (1 + abs(exact))
    assert abs(R.M.sum() - 4.0 / 3.0) < 1e-12
    # face mass matrices and LIFT
    uu, vv, ww = collapsed_tri_rule(P + 2)
    for fc in range(4):
        idx = R.Fmask[fc]
        # the face's own coordinates of its nodes, and of the cubature
        # points mapped into (r, s, t)
        if fc == 0:
            pr, ps, pt = 2 * uu - 1, 2 * vv - 1, -np.ones_like(uu)
        elif fc == 1:
            pr, ps, pt = 2 * uu - 1, -np.ones_like(uu), 2 * vv - 1
        elif fc == 2:
            pr, ps, pt = 2 * (1 - uu - vv) - 1, 2 * uu - 1, 2 * vv - 1
        else:
            pr, ps, pt = -np.ones_like(uu), 2 * uu - 1, 2 * vv - 1
        fu, fv = f(pr, ps, pt), g(pr, ps, pt)
        # face integral with respect to a reference triangle of area 2
        exact = 4.0 * np.sum(ww * fu * fv)
        got = u[idx] @ R.Mface[fc] @ v[idx]
        assert abs(got - exact) < 1e-11 * (1 + abs(exact)), fc
    np.testing.assert_allclose(R.M @ R.LIFT, R.E, atol=1e-12)


def test_geometry_and_connectivity():
    m = T.cube_mesh(3, 2.0, 0.15, 3)
    R = T.ref(2)
    geo = T.Geometry(m, R)
    assert (geo.J > 0).all()
    assert abs((geo.J * 4.0 / 3.0).sum() - 8.0) < 1e-12
    area = 2.0 * geo.sJ
    closure = np.einsum("kf,kfd->kd", area, geo.n)
    assert np.abs(closure).max() < 1e-14
    # reciprocal pairing, no boundary on the periodic cube
    k = np.arange(m.K)[:, None]
    assert (m.bc == 0).all()
    assert (m.EToE[m.EToE, m.EToF] == k).all() and (m.EToF[m.EToE, m.EToF] == np.arange(4)[None, :]).all()
    # the non-periodic box: 2 triangles per cube face on each of 6 sides
    mb = T.cube_mesh(3, 1.0, 0.1, 3, periodic=False)
    assert int((mb.bc == T.WALL).sum()) == 6 * 9 * 2


@pytest.mark.parametrize("P", [1, 2, 3])
def test_freestream_is_preserved(P):
    m = T.cube_mesh(3, 1.0, 0.15, 5)
    o = T.Oracle3D(m, P)
    one = np.ones((m.K, o.R.Np))
    U = T.primitive_to_conserved(1.3 * one, 0.4 * one, -0.3 * one, 0.2 * one, 0.9 * one)
    assert np.abs(o.rhs(U)).max() < 1e-12
    # a walled box at rest
    mb = T.cube_mesh(3, 1.0, 0.1, 5, periodic=False)
    ob = T.Oracle3D(mb, P)
    one = np.ones((mb.K, ob.R.Np))
    U = T.primitive_to_conserved(1.3 * one, 0 * one, 0 * one, 0 * one, 0.9 * one)
    assert np.abs(ob.rhs(U)).max() < 1e-12


@pytest.mark.parametrize("P", [1, 2])
def test_linear_data_is_exact(P):
    """A density linear in space advected at constant velocity and pressure
    (a flux linear in the state): the rhs is the exact constant dU/dt in
    every element away from the walls."""
    m = T.cube_mesh(3, 1.0, 0.1, 7, periodic=False)
    o = T.Oracle3D(m, P)
    x, y, z = o.xyz
    one = np.ones_like(x)
    U = T.primitive_to_conserved(1.0 + 0.1 * (x + 2 * y + 3 * z), 0.3 * one, 0.2 * one, 0.1 * one, one)
    r = o.rhs(U)
    drho = -(0.3 * 0.1 + 0.2 * 0.2 + 0.1 * 0.3)
    inner = (m.bc == 0).all(1)
    assert inner.sum() > 0
    np.testing.assert_allclose(r[inner, 0], drho, atol=1e-13)
    np.testing.assert_allclose(r[inner, 1], 0.3 * drho, atol=1e-13)
    np.testing.assert_allclose(r[inner, 4], 0.5 * (0.3 ** 2 + 0.2 ** 2 + 0.1 ** 2) * drho, atol=1e-13)


def smooth_state(xyz, seed=0):
    x, y, z = xyz
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 6)
    two = 2 * np.pi
    rho = 1.0 + 0.2 * np.sin(two * x + ph[0]) * np.cos(two * y + ph[1])
    u = 0.3 * np.sin(two * z + ph[2])
    v = 0.2 * np.cos(two * x + ph[3])
    w = -0.1 * np.sin(two * y + ph[4])
    p = 1.0 + 0.1 * np.cos(two * (x + z) + ph[5])
    return T.primitive_to_conserved(rho, u, v, w, p)


def test_conservation():
    m = T.cube_mesh(3, 1.0, 0.15, 9)
    o = T.Oracle3D(m, 3)
    U = smooth_state(o.xyz)
    tot = o.totals(o.rhs(U))
    assert np.abs(tot).max() < 1e-13
    # walls: mass and energy still conserved (no flux through a mirror wall)
    mb = T.cube_mesh(3, 1.0, 0.1, 9, periodic=False)
    ob = T.Oracle3D(mb, 3)
    tb = ob.totals(ob.rhs(smooth_state(ob.xyz)))
    assert abs(tb[0]) < 1e-13 and abs(tb[4]) < 1e-13


def test_cyclic_axis_permutation_symmetry():
    """Relabelling the axes (x, y, z) -> (y, z, x) of the mesh and the
    momentum gives the relabelled rhs: no direction is preferred by the face
    orientation handling."""
    m = T.cube_mesh(3, 1.0, 0.15, 11)
    o = T.Oracle3D(m, 2)
    U = smooth_state(o.xyz, 4)
    r = o.rhs(U)
    perm = [1, 2, 0]            # new x = old y, ...
    m2 = T.TetMesh(m.EToV, m.X[:, :, perm], m.period[perm])
    o2 = T.Oracle3D(m2, 2)
    U2 = U.copy()
    U2[:, 1:4] = U[:, [2, 3, 1]]
    r2 = o2.rhs(U2)
    np.testing.assert_allclose(r2[:, 1:4], r[:, [2, 3, 1]], atol=1e-12)
    np.testing.assert_allclose(r2[:, [0, 4]], r[:, [0, 4]], atol=1e-12)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_entropy_wave_converges(P):
    """rho = 1 + 0.2 sin(2 pi (x - u t)), constant velocity (1, 0.5, 0.25)
    and pressure, is an exact solution; the L2 error at t = 0.05 falls at
    order >= P + 0.2 from N = 3 to 6 (measured 1.8, 2.4, 3.8)."""
    def wave(xyz, t=0.0):
        x, y, z = xyz
        one = np.ones_like(x)
        return T.primitive_to_conserved(1.0 + 0.2 * np.sin(2 * np.pi * (x - t)), one, 0.5 * one, 0.25 * one, one)
    errs = []
    for N in (3, 6):
        m = T.cube_mesh(N, 1.0, 0.1, 7)
        o = T.Oracle3D(m, P)
        U0 = wave(o.xyz)
        n = int(math.ceil(0.05 / o.dt(U0)))
        U, t = o.run(U0, n, dt=0.05 / n)
        w = o.geo.J[:, None] * o.R.M.sum(0)[None, :]
        errs.append(math.sqrt((w * (U[:, 0] - wave(o.xyz, t)[:, 0]) ** 2).sum()))
    assert math.log2(errs[0] / errs[1]) >= P + 0.2, errs


def _exact_lift(P):
    """LIFT of the equispaced tetrahedron in exact rational arithmetic, from
    the definitions with the monomial basis: M from the exact simplex
    moments 8 a! b! c! / (a+b+c+3)!, face mass matrices from the exact
    triangle moments 4 a! b! / (a+b+2)! (area 2), LIFT = M^-1 E."""
    from fractions import Fraction as Fr
    f = math.factorial

    def inv(A):
        n = len(A)
        A = [row[:] + [Fr(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
        for c in range(n):
            p = next(r for r in range(c, n) if A[r][c] != 0)
            A[c], A[p] = A[p], A[c]
            d = A[c][c]
            A[c] = [x / d for x in A[c]]
            for r in range(n):
                if r != c and A[r][c] != 0:
                    m = A[r][c]
                    A[r] = [x - m * y for x, y in zip(A[r], A[c])]
        return [row[n:] for row in A]

    def mm(A, B):
        return [[sum(a * b for a, b in zip(row, col)) for col in zip(*B)] for row in A]

    def tr(A):
        return [list(r) for r in zip(*A)]

    lat = T.lattice(P)
    x = [Fr(int(i), P) for i in lat[:, 0]]
    y = [Fr(int(j), P) for j in lat[:, 1]]
    z = [Fr(int(k), P) for k in lat[:, 2]]
    mons = [(a, b, c) for a in range(P + 1) for b in range(P + 1 - a) for c in range(P + 1 - a - b)]
    V = [[x[n] ** a * y[n] ** b * z[n] ** c for a, b, c in mons] for n in range(len(lat))]
    Vi = inv(V)
    Mm = [[Fr(8 * f(a1 + a2) * f(b1 + b2) * f(c1 + c2), f(a1 + a2 + b1 + b2 + c1 + c2 + 3))
           for a2, b2, c2 in mons] for a1, b1, c1 in mons]
    M = mm(mm(tr(Vi), Mm), Vi)
    fm = [(a, b) for a in range(P + 1) for b in range(P + 1 - a)]
    Mfm = [[Fr(4 * f(a1 + a2) * f(b1 + b2), f(a1 + a2 + b1 + b2 + 2)) for a2, b2 in fm] for a1, b1 in fm]
    Np, Nfp = len(lat), len(fm)
    E = [[Fr(0)] * (4 * Nfp) for _ in range(Np)]
    i, j, k = lat[:, 0], lat[:, 1], lat[:, 2]
    for fc, cond in enumerate((k == 0, j == 0, i + j + k == P, i == 0)):
        ids = [int(n) for n in np.nonzero(cond)[0]]
        uv = [(x[n], y[n]) if fc == 0 else (x[n], z[n]) if fc == 1 else (y[n], z[n]) for n in ids]
        Vf = [[u ** a * v ** b for a, b in fm] for u, v in uv]
        Vfi = inv(Vf)
        Mf = mm(mm(tr(Vfi), Mfm), Vfi)
        for a in range(Nfp):
            for b in range(Nfp):
                E[ids[a]][fc * Nfp + b] = Mf[a][b]
    return np.array([[float(v) for v in row] for row in mm(inv(M), E)])


@pytest.mark.parametrize("P", [1, 2, 3])
def test_lift_matches_exact_rational_arithmetic(P):
    """LIFT against its definition evaluated in exact rational arithmetic
    (a different basis and no rounding): agreement to FP64 rounding."""
    np.testing.assert_allclose(T.ref(P).LIFT, _exact_lift(P), rtol=0, atol=5e-14 * (P + 1) ** 2)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_time_step_by_hand_on_one_tetrahedron(P):
    """The corner tetrahedron (0,0,0), (1,0,0), (0,1,0), (0,0,1): J = (1/6) /
    (4/3) = 1/8; the three right-angled faces have area 1/2 (Fscale = 2), the
    slanted one sqrt(3)/2 (Fscale = 2 sqrt 3).  A uniform state rho = 1.2,
    v = (0.3, 0.4, 0), p = 1 has |v| + c = 0.5 + sqrt(1.4 / 1.2), so
    dt = CFL / (1/2 (P+1)^2 2 sqrt3 (0.5 + sqrt(1.4/1.2)))."""
    X = np.array([[[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]])
    m = T.TetMesh(np.array([[0, 1, 2, 3]]), X, None)
    o = T.Oracle3D(m, P, cfl=0.7)
    assert abs(o.geo.J[0] - 1.0 / 8.0) < 1e-15
    np.testing.assert_allclose(np.sort(o.geo.Fscale[0]), [2.0, 2.0, 2.0, 2.0 * math.sqrt(3.0)], rtol=1e-14)
    one = np.ones((1, o.R.Np))
    U = T.primitive_to_conserved(1.2 * one, 0.3 * one, 0.4 * one, 0 * one, one)
    lam = 0.5 + math.sqrt(1.4 / 1.2)
    expect = 0.7 / (0.5 * (P + 1) ** 2 * 2.0 * math.sqrt(3.0) * lam)
    assert abs(o.dt(U) - expect) < 1e-14 * expect
    # the fastest node on a slower face does not set the step: speed up one
    # node that lies on the right-angled faces only (the corner at the origin)
    corner = int(np.argmin(o.R.r + o.R.s + o.R.t))        # (-1, -1, -1)
    U2 = U.copy()
    U2[0, 1, corner] = 1.2 * 0.9                          # u = 0.9 there
    U2[0, 4, corner] = 1.0 / 0.4 + 0.5 * 1.2 * (0.9 ** 2 + 0.4 ** 2)
    lam2 = math.sqrt(0.9 ** 2 + 0.4 ** 2) + math.sqrt(1.4 / 1.2)
    expect2 = 0.7 / (0.5 * (P + 1) ** 2 * max(2.0 * lam2, 2.0 * math.sqrt(3.0) * lam))
    assert abs(o.dt(U2) - expect2) < 1e-14 * expect2
