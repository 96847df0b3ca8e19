"""3D nodal DG for the Euler equations on straight tetrahedra: the CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the solver library.  Plain FP64 NumPy,
vectorised over elements only where the per-element formula is written out
unchanged.

The paper's own setting is three-dimensional: the Euler system with five
conserved fields (Section 5, the Euler equations) discretised by DG on
tetrahedra (Section 2).  This module writes out the nodal strong form of
that discretisation on straight (affine) tetrahedra:

  dU/dt = -(r_x Dr + s_x Ds + t_x Dt) F - (r_y Dr + ...) G - (r_z Dr + ...) H
          + LIFT (Fscale (n.F(U-) - F*)),

with the local Lax-Friedrichs flux F* (Section 2, after eq. weak_dg) and
the low-storage Runge-Kutta update.

Reference tetrahedron: vertices v1 = (-1,-1,-1), v2 = (1,-1,-1),
v3 = (-1,1,-1), v4 = (-1,-1,1).  Faces: f0 = (v1 v2 v3) on t = -1,
f1 = (v1 v2 v4) on s = -1, f2 = (v2 v3 v4) on r + s + t = -1, f3 =
(v1 v3 v4) on r = -1.

Readings (the paper gives the 3D operators by their definitions only):
* nodes: the equispaced lattice (i, j, k) / P on the tetrahedron (the
  paper's 2D node family has no 3D table here; for the orders used, P <= 4,
  the lattice is well conditioned);
* operators from their definitions (any polynomial basis gives the same
  nodal operators): Dr = V_r V^-1 with monomials in x = (1 + r)/2,
  y = (1 + s)/2, z = (1 + t)/2; the mass matrix M = (V_o V_o^T)^-1 from a
  basis orthonormal on the tetrahedron; per face the 2D mass matrix of the
  face's Lagrange basis with respect to a reference triangle of area 2, the
  same way from the orthonormal triangle basis; LIFT = M^-1 E;
* sJ = physical face area / 2, J = physical volume / (4/3), Fscale = sJ / J;
* slip wall: the mirror ghost state (normal momentum reversed);
* time step: dt = CFL / max over face nodes of (P+1)^2 Fscale (|v| + c) / 2,
  as in 2D.
"""
from __future__ import annotations

import functools
import math

import numpy as np

NF = 5          # rho, rho u, rho v, rho w, E
GAMMA = 1.4
WALL = 1

FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))


def n_nodes(P):
    return (P + 1) * (P + 2) * (P + 3) // 6


def n_face_nodes(P):
    return (P + 1) * (P + 2) // 2


def lattice(P):
    """Integer lattice indices (i, j, k) of the nodes, r fastest, then s,
    then t: node (i, j, k) sits at r = -1 + 2i/P, s = -1 + 2j/P,
    t = -1 + 2k/P."""
    out = []
    for k in range(P + 1):
        for j in range(P + 1 - k):
            for i in range(P + 1 - k - j):
                out.append((i, j, k))
    return np.array(out, dtype=np.int64)


def monomials(P):
    return [(a, b, c) for a in range(P + 1) for b in range(P + 1 - a) for c in range(P + 1 - a - b)]


def orthonormal_vandermonde2(P, r, s):
    """Vandermonde matrix of the orthonormal modal basis of the triangle
    (-1,-1), (1,-1), (-1,1) (the 2D oracle's basis)."""
    from .refelem import basis
    return np.stack([basis(r, s, i, j) for i in range(P + 1) for j in range(P + 1 - i)], 1)


def orthonormal_vandermonde3(P, r, s, t):
    """Vandermonde matrix of a basis orthonormal on the reference
    tetrahedron: through the collapsed coordinates a = 2(1+r)/(-s-t) - 1,
    b = 2(1+s)/(1-t) - 1, c = t,
    psi_ijk = 2 sqrt2 p_i(a) p_j^(2i+1,0)(b) (1-b)^i p_k^(2i+2j+2,0)(c) (1-c)^(i+j)
    with p^(alpha,beta) the Jacobi polynomials of unit norm (the product of
    the collapse's Jacobian weights makes the modes orthonormal)."""
    from .refelem import jacobi_normalized as jn
    r, s, t = (np.asarray(v, dtype=np.float64) for v in (r, s, t))
    st = -s - t
    a = np.where(np.abs(st) > 1e-14, 2.0 * (1.0 + r) / np.where(np.abs(st) > 1e-14, st, 1.0) - 1.0, -1.0)
    b = np.where(np.abs(1.0 - t) > 1e-14, 2.0 * (1.0 + s) / np.where(np.abs(1.0 - t) > 1e-14, 1.0 - t, 1.0) - 1.0,
                 -1.0)
    c = t
    cols = []
    for i in range(P + 1):
        for j in range(P + 1 - i):
            for k in range(P + 1 - i - j):
                cols.append(2.0 * math.sqrt(2.0) * jn(a, 0, 0, i) * jn(b, 2 * i + 1, 0, j) * (1.0 - b) ** i
                            * jn(c, 2 * i + 2 * j + 2, 0, k) * (1.0 - c) ** (i + j))
    return np.stack(cols, 1)


@functools.lru_cache(maxsize=None)
def ref(P):
    return RefTet(P)


class RefTet:
    def __init__(self, P):
        if P < 1:
            raise ValueError("P >= 1")
        self.P = P
        self.Np = n_nodes(P)
        self.Nfp = n_face_nodes(P)
        L = lattice(P)
        self.lat = L
        self.r = -1.0 + 2.0 * L[:, 0] / P
        self.s = -1.0 + 2.0 * L[:, 1] / P
        self.t = -1.0 + 2.0 * L[:, 2] / P
        x, y, z = L[:, 0] / P, L[:, 1] / P, L[:, 2] / P
        mons = monomials(P)
        V = np.stack([x ** a * y ** b * z ** c for a, b, c in mons], 1)
        # d/dr = (1/2) d/dx
        def dpow(v, e):
            return e * v ** (e - 1) if e > 0 else np.zeros_like(v)
        Vr = np.stack([0.5 * dpow(x, a) * y ** b * z ** c for a, b, c in mons], 1)
        Vs = np.stack([0.5 * x ** a * dpow(y, b) * z ** c for a, b, c in mons], 1)
        Vt = np.stack([0.5 * x ** a * y ** b * dpow(z, c) for a, b, c in mons], 1)
        Vi = np.linalg.inv(V)
        self.V = V
        self.Dr, self.Ds, self.Dt = Vr @ Vi, Vs @ Vi, Vt @ Vi
        # mass matrices through an orthonormal basis: with V_o the
        # Vandermonde matrix of a basis orthonormal on the element,
        # M = (V_o V_o^T)^-1 exactly (the nodal basis is V_o^-T times the
        # modal one).  Better conditioned than exact monomial moments, whose
        # Hilbert-like matrix loses about 1e-11 at P = 4.
        Vo = orthonormal_vandermonde3(P, self.r, self.s, self.t)
        self.Vo = Vo
        self.M = np.linalg.inv(Vo @ Vo.T)
        # faces: nodes by lattice condition, in increasing node order
        i, j, k = L[:, 0], L[:, 1], L[:, 2]
        conds = (k == 0, j == 0, i + j + k == P, i == 0)
        self.Fmask = np.array([np.nonzero(cnd)[0] for cnd in conds])
        # face coordinates (u, v) on the unit triangle for each face's nodes;
        # the face mass matrix of the face's Lagrange basis with respect to
        # the reference triangle of area 2 (coordinates 2u - 1, 2v - 1)
        fuv = (np.stack([x, y], 1), np.stack([x, z], 1), np.stack([y, z], 1), np.stack([y, z], 1))
        E = np.zeros((self.Np, 4 * self.Nfp))
        self.Mface = []
        for f in range(4):
            uv = fuv[f][self.Fmask[f]]
            Vf = orthonormal_vandermonde2(P, 2.0 * uv[:, 0] - 1.0, 2.0 * uv[:, 1] - 1.0)
            Mf = np.linalg.inv(Vf @ Vf.T)
            self.Mface.append(Mf)
            E[np.ix_(self.Fmask[f], np.arange(f * self.Nfp, (f + 1) * self.Nfp))] = Mf
        self.E = E
        # LIFT = M^-1 E = V_o V_o^T E
        self.LIFT = Vo @ (Vo.T @ E)


# ---------------------------------------------------------------------------
# geometry and connectivity
# ---------------------------------------------------------------------------

class TetMesh:
    """EToV (K, 4) into vertex coordinates VXYZ (Nv, 3); element k's own
    vertex coordinates X[k] (4, 3) (for periodic meshes an element may use a
    periodic image of a shared vertex); bc (K, 4): 0 interior, 1 wall."""

    def __init__(self, EToV, X, period=None):
        self.EToV = np.asarray(EToV, dtype=np.int64)
        self.X = np.asarray(X, dtype=np.float64)
        self.K = len(self.EToV)
        self.period = period
        faces = {}
        K = self.K
        self.EToE = np.tile(np.arange(K)[:, None], (1, 4))
        self.EToF = np.tile(np.arange(4)[None, :], (K, 1))
        self.bc = np.zeros((K, 4), dtype=np.int8)
        for k in range(K):
            for f, fv in enumerate(FACE_VERTS):
                key = tuple(sorted(self.EToV[k, list(fv)]))
                if key in faces:
                    k2, f2 = faces.pop(key)
                    self.EToE[k, f], self.EToF[k, f] = k2, f2
                    self.EToE[k2, f2], self.EToF[k2, f2] = k, f
                else:
                    faces[key] = (k, f)
        for (k, f) in faces.values():
            self.bc[k, f] = WALL


def node_coordinates(mesh, R):
    """Physical node coordinates (K, Np) x3 of the affine map."""
    lam = np.stack([-(1 + R.r + R.s + R.t) / 2, (1 + R.r) / 2, (1 + R.s) / 2, (1 + R.t) / 2], 1)
    xyz = np.einsum("iv,kvd->kid", lam, mesh.X)
    return xyz[..., 0], xyz[..., 1], xyz[..., 2]


class Geometry:
    def __init__(self, mesh, R):
        X = mesh.X
        A = np.stack([(X[:, 1] - X[:, 0]) / 2, (X[:, 2] - X[:, 0]) / 2, (X[:, 3] - X[:, 0]) / 2], 2)  # columns xr xs xt
        self.J = np.linalg.det(A)
        Ai = np.linalg.inv(A)          # rows: grad r, grad s, grad t
        self.drdx = Ai                  # drdx[k, a, d] = d(r_a)/d(x_d)
        K = mesh.K
        self.n = np.zeros((K, 4, 3))
        self.sJ = np.zeros((K, 4))
        for f, (a, b, c) in enumerate(FACE_VERTS):
            opp = ({0, 1, 2, 3} - {a, b, c}).pop()
            cr = np.cross(X[:, b] - X[:, a], X[:, c] - X[:, a])
            area = 0.5 * np.linalg.norm(cr, axis=1)
            nn = cr / (2 * area[:, None])
            sgn = np.sign(np.einsum("kd,kd->k", nn, X[:, opp] - X[:, a]))
            self.n[:, f] = -sgn[:, None] * nn
            self.sJ[:, f] = area / 2.0
        self.Fscale = self.sJ / self.J[:, None]


def face_maps(mesh, R, xyz, tol=1e-9):
    """For each (k, f, j): the neighbour node index (element, node) whose
    coordinates equal those of face node j (modulo the periodic box)."""
    x, y, z = xyz
    K, Nfp = mesh.K, R.Nfp
    pk = np.zeros((K, 4, Nfp), dtype=np.int64)
    pn = np.zeros((K, 4, Nfp), dtype=np.int64)
    per = mesh.period
    for k in range(K):
        for f in range(4):
            kn, fn = mesh.EToE[k, f], mesh.EToF[k, f]
            idm, idp = R.Fmask[f], R.Fmask[fn]
            pm = np.stack([x[k, idm], y[k, idm], z[k, idm]], 1)
            pp = np.stack([x[kn, idp], y[kn, idp], z[kn, idp]], 1)
            d = pm[:, None, :] - pp[None, :, :]
            if per is not None:
                d = d - np.round(d / per) * per
            dist = np.abs(d).max(2)
            jm = dist.argmin(1)
            if mesh.bc[k, f] == 0 and not (dist[np.arange(Nfp), jm] < tol).all():
                raise ValueError(f"face nodes of element {k} face {f} do not match")
            pk[k, f] = kn
            pn[k, f] = idp[jm]
    return pk, pn


# ---------------------------------------------------------------------------
# the semi-discrete operator
# ---------------------------------------------------------------------------

def pressure(U, g=GAMMA):
    return (g - 1.0) * (U[:, 4] - 0.5 * (U[:, 1] ** 2 + U[:, 2] ** 2 + U[:, 3] ** 2) / U[:, 0])


def fluxes(U, g=GAMMA):
    """F, G, H of the 3D Euler system (Section 5), each (K, 5, Np)."""
    rho, mx, my, mz, E = U[:, 0], U[:, 1], U[:, 2], U[:, 3], U[:, 4]
    u, v, w = mx / rho, my / rho, mz / rho
    p = (g - 1.0) * (E - 0.5 * (mx * u + my * v + mz * w))
    F = np.stack([mx, mx * u + p, my * u, mz * u, (E + p) * u], 1)
    G = np.stack([my, mx * v, my * v + p, mz * v, (E + p) * v], 1)
    H = np.stack([mz, mx * w, my * w, mz * w + p, (E + p) * w], 1)
    return F, G, H


def normal_flux(u, n, g=GAMMA):
    """n.F(u) and |v.n| + c for states u (..., 5) and normals n (..., 3)."""
    rho = u[..., 0]
    vel = u[..., 1:4] / rho[..., None]
    p = (g - 1.0) * (u[..., 4] - 0.5 * rho * (vel ** 2).sum(-1))
    vn = (vel * n).sum(-1)
    fn = np.stack([rho * vn,
                   u[..., 1] * vn + p * n[..., 0],
                   u[..., 2] * vn + p * n[..., 1],
                   u[..., 3] * vn + p * n[..., 2],
                   (u[..., 4] + p) * vn], -1)
    lam = np.abs(vn) + np.sqrt(g * p / rho)
    return fn, lam


class Oracle3D:
    def __init__(self, mesh, P, cfl=0.5, gamma=GAMMA):
        self.mesh, self.P, self.cfl, self.g = mesh, P, cfl, gamma
        self.R = ref(P)
        self.xyz = node_coordinates(mesh, self.R)
        self.geo = Geometry(mesh, self.R)
        self.pk, self.pn = face_maps(mesh, self.R, self.xyz)

    def rhs(self, U):
        R, geo, m = self.R, self.geo, self.mesh
        U = np.asarray(U, dtype=np.float64)
        K, Np, Nfp = m.K, R.Np, R.Nfp
        F, G, H = fluxes(U, self.g)
        a = geo.drdx            # (K, 3 [r s t], 3 [x y z])
        out = np.zeros_like(U)
        for D, row in ((R.Dr, 0), (R.Ds, 1), (R.Dt, 2)):
            for flux, col in ((F, 0), (G, 1), (H, 2)):
                out -= a[:, row, col][:, None, None] * np.einsum("ij,kcj->kci", D, flux)
        # face terms
        d = np.zeros((K, NF, 4 * Nfp))
        for f in range(4):
            idm = R.Fmask[f]
            um = np.transpose(U[:, :, idm], (0, 2, 1))                  # (K, Nfp, 5)
            up = np.transpose(U[self.pk[:, f], :, self.pn[:, f]], (0, 1, 2))  # (K, Nfp, 5)
            n = np.broadcast_to(geo.n[:, f][:, None, :], (K, Nfp, 3))
            wall = m.bc[:, f] == WALL
            if wall.any():
                g = um[wall].copy()
                mn = (g[..., 1:4] * n[wall]).sum(-1)
                g[..., 1:4] -= 2.0 * mn[..., None] * n[wall]
                up = up.copy()
                up[wall] = g
            fm, lm = normal_flux(um, n, self.g)
            fp, lp = normal_flux(up, n, self.g)
            lam = np.maximum(lm, lp)
            jump = 0.5 * (fm - fp) + 0.5 * lam[..., None] * (up - um)
            d[:, :, f * Nfp:(f + 1) * Nfp] = np.transpose(jump, (0, 2, 1)) * geo.Fscale[:, f][:, None, None]
        out += np.einsum("ij,kcj->kci", R.LIFT, d)
        return out

    def dt(self, U):
        R, geo = self.R, self.geo
        P1 = self.P + 1.0
        best = 0.0
        for f in range(4):
            u = np.transpose(U[:, :, R.Fmask[f]], (0, 2, 1))
            rho = u[..., 0]
            vel = u[..., 1:4] / rho[..., None]
            p = (self.g - 1.0) * (u[..., 4] - 0.5 * rho * (vel ** 2).sum(-1))
            lam = np.sqrt((vel ** 2).sum(-1)) + np.sqrt(self.g * p / rho)
            best = max(best, float((0.5 * P1 * P1 * geo.Fscale[:, f][:, None] * lam).max()))
        return self.cfl / best

    def totals(self, U):
        w = self.geo.J[:, None] * self.R.M.sum(0)[None, :]       # exact L2 weights of the nodal interpolant
        return np.einsum("ki,kci->c", w, U)

    def run(self, U, nsteps, dt=None):
        """LSERK(5,4) steps (Carpenter-Kennedy), dt from the state at each
        step's start unless given."""
        U = np.array(U, dtype=np.float64)
        Rk = np.zeros_like(U)
        t = 0.0
        for _ in range(nsteps):
            h = self.dt(U) if dt is None else dt
            for s in range(5):
                Rk = RK_A[s] * Rk + h * self.rhs(U)
                U = U + RK_B[s] * Rk
            t += h
        return U, t


# Carpenter-Kennedy 2N-storage (5,4) coefficients (published rationals).
RK_A = (0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0)
RK_B = (1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
        2277821191437.0 / 14882151754819.0)


# ---------------------------------------------------------------------------
# meshes and flows
# ---------------------------------------------------------------------------

def cube_mesh(N, L=1.0, jitter=0.0, seed=0, periodic=True):
    """The seeded cube mesh of the shared input generator (Kuhn split of N^3
    cubes, jittered vertices) with this module's own connectivity."""
    from meshgen.tets import cube_tets
    g = cube_tets(N, L, jitter, seed, periodic)
    return TetMesh(g.EToV, g.X, g.period)


def primitive_to_conserved(rho, u, v, w, p, g=GAMMA):
    return np.stack([rho, rho * u, rho * v, rho * w, p / (g - 1.0) + 0.5 * rho * (u * u + v * v + w * w)], 1)


def entropy_wave(xyz, t=0.0, L=1.0, amp=0.2, vel=(1.0, 0.5, 0.25)):
    """rho = 1 + amp sin(2 pi (x + y + z - (u + v + w) t) / L), constant
    velocity and pressure: an exact solution of the Euler equations."""
    x, y, z = xyz
    u, v, w = vel
    rho = 1.0 + amp * np.sin(2 * np.pi * (x + y + z - (u + v + w) * t) / L)
    one = np.ones_like(x)
    return primitive_to_conserved(rho, u * one, v * one, w * one, one)
