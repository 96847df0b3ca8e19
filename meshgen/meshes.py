"""Seeded synthetic triangle meshes for the 2D Euler test cases.

Everything here is geometry and bookkeeping: vertex grids, jitter, element
permutation, face connectivity and wall curving.  None of the DG method's
arithmetic (nodes, bases, operators, fluxes) lives here; the high-order node
positions are produced by evaluating the element map at reference points the
caller passes in.

Conventions shared with the solver interface:

* reference triangle vertices v1=(-1,-1), v2=(1,-1), v3=(-1,1);
* faces f=0: v1->v2, f=1: v2->v3, f=2: v3->v1 (counter-clockwise);
* elements are counter-clockwise (positive signed area);
* a boundary face has EToE[k,f]=k, EToF[k,f]=f and bc[k,f] != 0;
* bc codes: 0 interior (periodic seams included), 1 slip wall, 2 far field.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

BC_INTERIOR = 0
BC_WALL = 1
BC_FARFIELD = 2

# Vertex pairs (local ids) of the three faces, in counter-clockwise traversal.
FACE_VERTS = ((0, 1), (1, 2), (2, 0))


@dataclass
class Mesh:
    """Straight-sided triangle mesh plus an optional wall-curving rule."""

    VX: np.ndarray                    # (Nv,) vertex x
    VY: np.ndarray                    # (Nv,) vertex y
    EToV: np.ndarray                  # (K,3) int64, CCW vertex ids
    EToE: np.ndarray                  # (K,3) int32
    EToF: np.ndarray                  # (K,3) int32
    bc: np.ndarray                    # (K,3) int8
    name: str = ""
    # curve(k, f, t) -> (x, y) points on the exact wall for edge parameter t in
    # [-1, 1] running from the face's first vertex to its second.  None: no
    # curving (straight walls).
    curve: Optional[Callable[[int, int, np.ndarray], np.ndarray]] = None
    # smooth displacement applied to every high-order node (all elements
    # curved); a function (x, y) -> (dx, dy) that is periodic where the mesh is.
    node_displacement: Optional[Callable[[np.ndarray, np.ndarray], tuple]] = None
    info: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return int(self.EToV.shape[0])

    def vertex_xy(self):
        """(K,3) arrays of vertex coordinates per element."""
        return self.VX[self.EToV], self.VY[self.EToV]

    def signed_area(self) -> np.ndarray:
        x, y = self.vertex_xy()
        return 0.5 * ((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0])
                      - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))


# ---------------------------------------------------------------------------
# connectivity
# ---------------------------------------------------------------------------

def connect(EToV: np.ndarray, vid_key: np.ndarray, bc_of_face=None):
    """Face-to-face connectivity.

    ``vid_key`` maps each vertex id to an identification key (periodic images
    share a key).  Faces with the same unordered key pair are glued.  Faces that
    stay unmatched become boundary faces whose code ``bc_of_face(k, f)`` gives.
    """
    K = EToV.shape[0]
    EToE = np.repeat(np.arange(K, dtype=np.int32)[:, None], 3, axis=1)
    EToF = np.repeat(np.arange(3, dtype=np.int32)[None, :], K, axis=0).copy()
    bc = np.zeros((K, 3), dtype=np.int8)
    a = np.stack([vid_key[EToV[:, i]] for i, _ in FACE_VERTS], axis=1)
    b = np.stack([vid_key[EToV[:, j]] for _, j in FACE_VERTS], axis=1)
    lo = np.minimum(a, b).ravel()
    hi = np.maximum(a, b).ravel()
    nk = int(vid_key.max()) + 1
    key = lo.astype(np.int64) * nk + hi
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = np.nonzero(ks[1:] == ks[:-1])[0]
    if same.size and np.any(np.diff(same) == 1):
        raise ValueError("a face is shared by more than two elements")
    f1 = order[same]
    f2 = order[same + 1]
    k1, l1 = f1 // 3, f1 % 3
    k2, l2 = f2 // 3, f2 % 3
    EToE[k1, l1] = k2
    EToF[k1, l1] = l2
    EToE[k2, l2] = k1
    EToF[k2, l2] = l1
    matched = np.zeros(3 * K, dtype=bool)
    matched[f1] = True
    matched[f2] = True
    for ff in np.nonzero(~matched)[0]:
        k, f = divmod(int(ff), 3)
        if bc_of_face is None:
            raise ValueError(f"unmatched face ({k},{f}) on a closed mesh")
        bc[k, f] = bc_of_face(k, f)
    return EToE, EToF, bc


def permute_elements(mesh: Mesh, perm: np.ndarray) -> Mesh:
    """New mesh whose element ``i`` is old element ``perm[i]``."""
    perm = np.asarray(perm, dtype=np.int64)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    EToE = inv[mesh.EToE[perm]].astype(np.int32)
    curve = None
    if mesh.curve is not None:
        old_curve = mesh.curve
        curve = lambda k, f, t: old_curve(int(perm[k]), f, t)  # noqa: E731
    return Mesh(mesh.VX, mesh.VY, mesh.EToV[perm].copy(), EToE,
                mesh.EToF[perm].copy(), mesh.bc[perm].copy(), mesh.name,
                curve, mesh.node_displacement, dict(mesh.info, permuted=True))


# ---------------------------------------------------------------------------
# generators
# ---------------------------------------------------------------------------

def periodic_square(N: int, L: float = 10.0, jitter: float = 0.1,
                    jitter_seed: int = 1208, perm_seed: Optional[int] = 4772,
                    curved_amplitude: float = 0.0) -> Mesh:
    """Doubly periodic [0,L]^2 with 2*N*N triangles.

    Each grid cell is split along its (i,j)->(i+1,j+1) diagonal.  Interior
    vertices move independently in x and y by U(-jitter*h, jitter*h); seam
    vertices stay put so that the periodic translation is exact.  With
    ``perm_seed`` the element order is randomly permuted.  With
    ``curved_amplitude`` a every high-order node moves by
    a*h*sin(2 pi x/L) sin(2 pi y/L) in both coordinates, which curves every
    element while keeping shared faces watertight.
    """
    if N < 3:
        raise ValueError("N >= 3")
    h = L / N
    n1 = N + 1
    ii, jj = np.meshgrid(np.arange(n1), np.arange(n1), indexing="ij")
    VX = (ii * h).astype(np.float64).ravel()
    VY = (jj * h).astype(np.float64).ravel()
    rng = np.random.default_rng(jitter_seed)
    d = rng.uniform(-jitter * h, jitter * h, size=(2, n1 * n1))
    interior = ((ii > 0) & (ii < N) & (jj > 0) & (jj < N)).ravel()
    VX[interior] += d[0, interior]
    VY[interior] += d[1, interior]

    def vid(i, j):
        return i * n1 + j

    ci, cj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()
    t1 = np.stack([vid(ci, cj), vid(ci + 1, cj), vid(ci + 1, cj + 1)], axis=1)
    t2 = np.stack([vid(ci, cj), vid(ci + 1, cj + 1), vid(ci, cj + 1)], axis=1)
    EToV = np.empty((2 * N * N, 3), dtype=np.int64)
    EToV[0::2] = t1
    EToV[1::2] = t2
    key = ((ii % N) * N + (jj % N)).ravel()
    EToE, EToF, bc = connect(EToV, key)
    disp = None
    if curved_amplitude:
        a = curved_amplitude * h

        def disp(x, y):
            w = a * np.sin(2 * np.pi * x / L) * np.sin(2 * np.pi * y / L)
            return w, w
    mesh = Mesh(VX, VY, EToV, EToE, EToF, bc, f"periodic_square_N{N}", None,
                disp, dict(N=N, L=L, h=h, periodic=(L, L)))
    if perm_seed is not None:
        perm = np.random.default_rng(perm_seed).permutation(mesh.K)
        mesh = permute_elements(mesh, perm)
    return mesh


def channel(Nx: int, Ny: int, L: float = 10.0, H: float = 5.0, jitter: float = 0.1,
            jitter_seed: int = 7, perm_seed: Optional[int] = None) -> Mesh:
    """[0,L] x [0,H], periodic in x, slip walls at y=0 and y=H; 2*Nx*Ny
    triangles (cells split along the (i,j)->(i+1,j+1) diagonal).  Vertices
    off the seam and the walls move by U(-jitter*h, jitter*h) per coordinate
    (h the smaller cell side)."""
    if Nx < 3 or Ny < 2:
        raise ValueError("Nx >= 3, Ny >= 2")
    hx, hy = L / Nx, H / Ny
    h = min(hx, hy)
    nx1, ny1 = Nx + 1, Ny + 1
    ii, jj = np.meshgrid(np.arange(nx1), np.arange(ny1), indexing="ij")
    VX = (ii * hx).astype(np.float64).ravel()
    VY = (jj * hy).astype(np.float64).ravel()
    rng = np.random.default_rng(jitter_seed)
    d = rng.uniform(-jitter * h, jitter * h, size=(2, nx1 * ny1))
    interior = ((ii > 0) & (ii < Nx) & (jj > 0) & (jj < Ny)).ravel()
    VX[interior] += d[0, interior]
    VY[interior] += d[1, interior]

    def vid(i, j):
        return i * ny1 + j

    ci, cj = np.meshgrid(np.arange(Nx), np.arange(Ny), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()
    EToV = np.empty((2 * Nx * Ny, 3), dtype=np.int64)
    EToV[0::2] = np.stack([vid(ci, cj), vid(ci + 1, cj), vid(ci + 1, cj + 1)], axis=1)
    EToV[1::2] = np.stack([vid(ci, cj), vid(ci + 1, cj + 1), vid(ci, cj + 1)], axis=1)
    key = ((ii % Nx) * ny1 + jj).ravel()
    EToE, EToF, bc = connect(EToV, key, lambda k, f: BC_WALL)
    mesh = Mesh(VX, VY, EToV, EToE, EToF, bc, f"channel_{Nx}x{Ny}", None, None,
                dict(Nx=Nx, Ny=Ny, L=L, H=H, h=h, periodic=(L, None)))
    if perm_seed is not None:
        mesh = permute_elements(mesh, np.random.default_rng(perm_seed).permutation(mesh.K))
    return mesh


def _orient_ccw(VX, VY, EToV):
    x = VX[EToV]
    y = VY[EToV]
    area = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    flip = area < 0
    EToV = EToV.copy()
    EToV[flip, 1], EToV[flip, 2] = EToV[flip, 2].copy(), EToV[flip, 1].copy()
    return EToV


def _ogrid(Xs, Ys, Nt, Nr, jitter, seed, wall_curve_param, name, info,
           inner_bc=BC_WALL, mirror_split=False):
    """O-grid triangles from vertex arrays Xs/Ys of shape (Nt, Nr+1).

    Column j=0 is the wall, j=Nr the far field; index i is periodic.  Cells
    are split along their (i,j)->(i+1,j+1) diagonal; with ``mirror_split``
    the cells of the second half (i >= Nt/2) take the other diagonal, so that
    an unjittered grid that is mirror-symmetric in i -> Nt-i gives a mirror-
    symmetric triangulation.
    """
    VX = Xs.ravel().copy()
    VY = Ys.ravel().copy()
    if jitter:
        rng = np.random.default_rng(seed)
        # local spacing: the smallest distance to the 4 grid neighbours
        dxr = np.hypot(np.diff(Xs, axis=1), np.diff(Ys, axis=1))
        dxt = np.hypot(np.roll(Xs, -1, 0) - Xs, np.roll(Ys, -1, 0) - Ys)
        hloc = np.full(Xs.shape, np.inf)
        hloc[:, :-1] = np.minimum(hloc[:, :-1], dxr)
        hloc[:, 1:] = np.minimum(hloc[:, 1:], dxr)
        hloc = np.minimum(hloc, dxt)
        hloc = np.minimum(hloc, np.roll(dxt, 1, 0))
        d = rng.uniform(-jitter, jitter, size=(2,) + Xs.shape) * hloc
        d[:, :, 0] = 0.0
        d[:, :, -1] = 0.0
        VX += d[0].ravel()
        VY += d[1].ravel()
    n1 = Nr + 1

    def vid(i, j):
        return (i % Nt) * n1 + j

    ci, cj = np.meshgrid(np.arange(Nt), np.arange(Nr), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()
    t1 = np.stack([vid(ci, cj), vid(ci + 1, cj), vid(ci + 1, cj + 1)], axis=1)
    t2 = np.stack([vid(ci, cj), vid(ci + 1, cj + 1), vid(ci, cj + 1)], axis=1)
    if mirror_split:
        second = ci >= Nt // 2
        t1[second] = np.stack([vid(ci, cj), vid(ci + 1, cj), vid(ci, cj + 1)], axis=1)[second]
        t2[second] = np.stack([vid(ci + 1, cj), vid(ci + 1, cj + 1), vid(ci, cj + 1)], axis=1)[second]
    EToV = np.empty((2 * Nt * Nr, 3), dtype=np.int64)
    EToV[0::2] = t1
    EToV[1::2] = t2
    EToV = _orient_ccw(VX, VY, EToV)
    key = np.arange(Nt * n1)
    jcol = np.arange(Nt * n1) % n1

    def bc_of_face(k, f):
        a, b = FACE_VERTS[f]
        ja, jb = jcol[EToV[k, a]], jcol[EToV[k, b]]
        if ja == 0 and jb == 0:
            return inner_bc
        if ja == Nr and jb == Nr:
            return BC_FARFIELD
        raise ValueError("unmatched interior face")

    EToE, EToF, bc = connect(EToV, key, bc_of_face)
    mesh = Mesh(VX, VY, EToV, EToE, EToF, bc, name, None, None, info)
    if wall_curve_param is not None and inner_bc == BC_WALL:
        # parameter of each wall vertex; curve(k,f,t) interpolates in it
        param_of_vertex, point_of_param = wall_curve_param
        ev = EToV

        def curve(k, f, t):
            a, b = FACE_VERTS[f]
            pa = param_of_vertex(int(ev[k, a]))
            pb = param_of_vertex(int(ev[k, b]))
            if pb - pa > np.pi:       # seam of the periodic parameter
                pa += 2 * np.pi
            elif pa - pb > np.pi:
                pb += 2 * np.pi
            return point_of_param(pa + 0.5 * (1.0 + np.asarray(t)) * (pb - pa))
        mesh.curve = curve
    return mesh


def cylinder_annulus(Ntheta: int = 200, Nr: int = 50, R1: float = 1.0,
                     R2: float = 20.0, jitter: float = 0.1, seed: int = 38,
                     curved: bool = True, inner_bc: int = BC_WALL,
                     mirror_split: bool = False) -> Mesh:
    """Annulus R1<=r<=R2 around the origin, 2*Ntheta*Nr triangles.

    Radii are geometric, r_j = R1*(R2/R1)^(j/Nr).  Interior vertices get a
    seeded jitter of ``jitter`` times the local spacing.  The inner circle is a
    slip wall (curved onto the exact circle when ``curved``), the outer circle
    the far field.  ``inner_bc=BC_FARFIELD`` gives a far-field-only annulus
    (straight inner boundary).  ``mirror_split`` (with ``jitter=0`` and even
    ``Ntheta``) makes the triangulation mirror-symmetric about the x axis.
    """
    th = 2 * np.pi * np.arange(Ntheta) / Ntheta
    r = R1 * (R2 / R1) ** (np.arange(Nr + 1) / Nr)
    Xs = r[None, :] * np.cos(th)[:, None]
    Ys = r[None, :] * np.sin(th)[:, None]
    n1 = Nr + 1
    curve = None
    if curved:
        def param_of_vertex(v):
            return th[v // n1]

        def point_of_param(p):
            return np.stack([R1 * np.cos(p), R1 * np.sin(p)], axis=-1)
        curve = (param_of_vertex, point_of_param)
    return _ogrid(Xs, Ys, Ntheta, Nr, jitter, seed, curve,
                  f"cylinder_{Ntheta}x{Nr}",
                  dict(R1=R1, R2=R2, chord=2 * R1, wall="circle"), inner_bc,
                  mirror_split)


def naca4_thickness(x, t=0.12):
    """Symmetric NACA 4-digit half-thickness with the closed trailing edge."""
    x = np.clip(x, 0.0, 1.0)
    return 5.0 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2
                      + 0.2843 * x ** 3 - 0.1036 * x ** 4)


def naca_point(beta, t=0.12):
    """Airfoil surface point for the parameter beta in [0, 2 pi) (0 = trailing
    edge, pi = leading edge, upper surface for beta in (0, pi)).

    x = 1 - sin(beta/2): uniform panels at the trailing edge, quadratic
    clustering in x at the leading edge (uniform in arc length there).
    """
    beta = np.asarray(beta, dtype=np.float64)
    x = 1.0 - np.sin(0.5 * beta)
    sgn = np.where(np.sin(beta) >= 0.0, 1.0, -1.0)
    return np.stack([x, sgn * naca4_thickness(x, t)], axis=-1)


def naca4_ogrid(Ntheta: int = 600, Nr: int = 100, t: float = 0.12,
                R: float = 30.0, growth: float = 1.06, jitter: float = 0.02,
                seed: int = 80, curved: bool = True, mirror_split: bool = False) -> Mesh:
    """O-grid around a symmetric 4-digit airfoil (chord 1) inside a circular
    far field of radius R centred at (0.5, 0); 2*Ntheta*Nr triangles.

    Radial lines blend each surface point with the far-field point at the
    same angle; the blend parameter is geometrically graded (ratio
    ``growth``).  The surface parameter clusters panels at the leading edge.
    """
    beta = 2 * np.pi * np.arange(Ntheta) / Ntheta
    surf = naca_point(beta, t)
    outer = np.stack([0.5 + R * np.cos(beta), R * np.sin(beta)], axis=-1)
    j = np.arange(Nr + 1)
    s = (growth ** j - 1.0) / (growth ** Nr - 1.0)
    X = (1 - s)[None, :] * surf[:, None, 0] + s[None, :] * outer[:, None, 0]
    Y = (1 - s)[None, :] * surf[:, None, 1] + s[None, :] * outer[:, None, 1]
    n1 = Nr + 1
    curve = None
    if curved:
        def param_of_vertex(v):
            return beta[v // n1]

        def point_of_param(p):
            return naca_point(np.mod(p, 2 * np.pi), t)
        curve = (param_of_vertex, point_of_param)
    return _ogrid(X, Y, Ntheta, Nr, jitter, seed, curve,
                  f"naca00{int(round(t * 100)):02d}_{Ntheta}x{Nr}",
                  dict(R=R, chord=1.0, wall="naca", thickness=t), BC_WALL, mirror_split)


# ---------------------------------------------------------------------------
# high-order node positions
# ---------------------------------------------------------------------------

# Interior points of the order-3 Gauss-Lobatto rule on [-1, 1]; the wall edge
# is fixed by its end vertices plus these two points.
_GL3_INNER = np.array([-1.0 / np.sqrt(5.0), 1.0 / np.sqrt(5.0)])


def node_coordinates(mesh: Mesh, r: np.ndarray, s: np.ndarray):
    """Physical coordinates (x, y), each (K, Np), of reference points (r, s).

    Straight elements use the affine vertex map.  A wall face with a curve
    rule gets a cubic edge displacement d(t) = (1 - t^2)(alpha + beta t) that
    matches the exact wall at the order-3 Gauss-Lobatto points; it is blended
    into the element as 4 la lb (alpha + beta (lb - la)), where la, lb are the
    barycentric coordinates of the face's two vertices.  That blend equals
    d(t) on the wall face, vanishes on the other two faces and is a cubic
    polynomial of (r, s).
    """
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    lam = np.stack([-(r + s) / 2.0, (1.0 + r) / 2.0, (1.0 + s) / 2.0])  # (3,Np)
    vx, vy = mesh.vertex_xy()
    x = vx @ lam
    y = vy @ lam
    if mesh.curve is not None:
        ks, fs = np.nonzero(mesh.bc == BC_WALL)
        for k, f in zip(ks.tolist(), fs.tolist()):
            a, b = FACE_VERTS[f]
            pa = np.array([vx[k, a], vy[k, a]])
            pb = np.array([vx[k, b], vy[k, b]])
            tq = _GL3_INNER
            straight = pa[None, :] + 0.5 * (1.0 + tq)[:, None] * (pb - pa)[None, :]
            exact = np.asarray(mesh.curve(k, f, tq))
            g = (exact - straight) / (1.0 - tq ** 2)[:, None]   # (2, 2)
            alpha = 0.5 * (g[0] + g[1])
            beta = (g[1] - g[0]) / (tq[1] - tq[0])
            la, lb = lam[a], lam[b]
            w = 4.0 * la * lb
            x[k] += w * (alpha[0] + beta[0] * (lb - la))
            y[k] += w * (alpha[1] + beta[1] * (lb - la))
    if mesh.node_displacement is not None:
        dx, dy = mesh.node_displacement(x, y)
        x = x + dx
        y = y + dy
    return np.ascontiguousarray(x), np.ascontiguousarray(y)
