"""Seeded synthetic tetrahedral meshes of a cube for the 3D Euler cases.

Geometry and bookkeeping only (vertex grid, jitter, the split of each cube
into tetrahedra, face connectivity); none of the DG method's arithmetic.

Conventions shared with the 3D solver interface: reference tetrahedron
vertices v1..v4 = (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1); faces
f0 = (v1 v2 v3), f1 = (v1 v2 v4), f2 = (v2 v3 v4), f3 = (v1 v3 v4);
elements positively oriented; a wall face has EToE[k,f] = k, EToF[k,f] = f
and bc[k,f] = 1.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

FACE_VERTS3 = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))
BC3_INTERIOR, BC3_WALL = 0, 1

# The 6 tetrahedra of a cube that share its main diagonal (0,0,0)-(1,1,1):
# one per ordering of the axes along which the path from corner 0 climbs
# (Kuhn's triangulation; neighbouring cubes' faces match).
_KUHN = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


@dataclass
class TetGrid:
    EToV: np.ndarray                  # (K, 4) int64 global vertex ids (periodic images share an id)
    X: np.ndarray                     # (K, 4, 3) each element's own vertex coordinates
    period: Optional[np.ndarray]      # (3,) box lengths of a periodic mesh, else None
    EToE: np.ndarray = None           # (K, 4) int32
    EToF: np.ndarray = None           # (K, 4) int32
    bc: np.ndarray = None             # (K, 4) int8

    @property
    def K(self):
        return int(self.EToV.shape[0])


def connect3(EToV):
    """Face-to-face connectivity of a tetrahedral mesh: faces with the same
    vertex triple are glued; unmatched faces become walls."""
    EToV = np.asarray(EToV, dtype=np.int64)
    K = EToV.shape[0]
    EToE = np.repeat(np.arange(K, dtype=np.int32)[:, None], 4, axis=1)
    EToF = np.repeat(np.arange(4, dtype=np.int32)[None, :], K, axis=0).copy()
    bc = np.full((K, 4), BC3_WALL, dtype=np.int8)
    tri = np.sort(np.stack([EToV[:, list(fv)] for fv in FACE_VERTS3], 1), axis=2).reshape(-1, 3)
    nv = int(EToV.max()) + 1
    key = (tri[:, 0] * nv + tri[:, 1]) * nv + tri[:, 2]
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = np.nonzero(ks[1:] == ks[:-1])[0]
    if same.size and np.any(np.diff(same) == 1):
        raise ValueError("a face is shared by more than two elements")
    f1, f2 = order[same], order[same + 1]
    k1, l1 = f1 // 4, f1 % 4
    k2, l2 = f2 // 4, f2 % 4
    EToE[k1, l1], EToF[k1, l1] = k2, l2
    EToE[k2, l2], EToF[k2, l2] = k1, l1
    bc[k1, l1] = BC3_INTERIOR
    bc[k2, l2] = BC3_INTERIOR
    return EToE, EToF, bc


def cube_tets(N, L=1.0, jitter=0.0, seed=0, periodic=True):
    """N^3 cubes of side h = L/N (or, with N = (Nx, Ny, Nz), a box of
    Nx x Ny x Nz such cubes, Nx h by Ny h by Nz h), each split into 6
    tetrahedra along its main diagonal; vertices jittered uniformly by up to
    jitter * h per axis (a periodic mesh jitters each shared vertex once and
    its images by the same amount; a walled box keeps its boundary
    vertices).  Periodic meshes need at least 3 cubes per direction so that
    no two faces share a vertex triple by wrap-around."""
    dims = np.array((N, N, N) if np.isscalar(N) else tuple(N), dtype=np.int64)
    if periodic and dims.min() < 3:
        raise ValueError("a periodic box mesh needs at least 3 cubes per direction")
    h = L / dims[0]
    rng = np.random.default_rng(seed)
    nv = dims if periodic else dims + 1
    base = np.stack(np.meshgrid(np.arange(nv[0]), np.arange(nv[1]), np.arange(nv[2]), indexing="ij"),
                    -1).reshape(-1, 3)
    VXYZ = base * h
    if jitter > 0:
        J = rng.uniform(-jitter * h, jitter * h, VXYZ.shape)
        if not periodic:
            J[((base == 0) | (base == dims[None, :]))] = 0.0
        VXYZ = VXYZ + J

    def vid(c):
        if periodic:
            c = np.array(c) % dims
        return (c[0] * nv[1] + c[1]) * nv[2] + c[2]

    EToV, X = [], []
    for i in range(dims[0]):
        for j in range(dims[1]):
            for k in range(dims[2]):
                for perm in _KUHN:
                    corner = [i, j, k]
                    path = [tuple(corner)]
                    for ax in perm:
                        corner[ax] += 1
                        path.append(tuple(corner))
                    ids = [int(vid(c)) for c in path]
                    pts = []
                    for c, v in zip(path, ids):
                        p = VXYZ[v].copy()
                        if periodic:
                            p = p + (np.array(c) - np.array(c) % dims) * h
                        pts.append(p)
                    pts = np.array(pts)
                    vol = np.linalg.det(np.stack([pts[1] - pts[0], pts[2] - pts[0], pts[3] - pts[0]], 1))
                    if vol < 0:
                        ids[1], ids[2] = ids[2], ids[1]
                        pts[[1, 2]] = pts[[2, 1]]
                    EToV.append(ids)
                    X.append(pts)
    g = TetGrid(np.array(EToV, dtype=np.int64), np.array(X), dims * h if periodic else None)
    g.EToE, g.EToF, g.bc = connect3(g.EToV)
    return g


def affine_node_coordinates(grid, r, s, t):
    """Physical coordinates (K, Np) x3 of reference points (r, s, t) under
    each element's affine map (barycentric weights of the four vertices)."""
    lam = np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2], 1)
    xyz = np.einsum("iv,kvd->kid", lam, grid.X)
    return xyz[..., 0], xyz[..., 1], xyz[..., 2]


def entropy_wave3(xyz, t=0.0, L=1.0, amp=0.2, vel=(1.0, 0.5, 0.25), gamma=1.4, along=(1, 1, 1)):
    """Conserved (K, 5, Np) of rho = 1 + amp sin(2 pi a.(x - v t) / L) at
    constant velocity v and unit pressure, a = `along` (integer wave
    numbers): an exact solution of the Euler equations on a periodic box
    whose sides are multiples of L along the axes a involves."""
    x, y, z = xyz
    u, v, w = vel
    a = along
    rho = 1.0 + amp * np.sin(2 * np.pi * (a[0] * (x - u * t) + a[1] * (y - v * t) + a[2] * (z - w * t)) / L)
    one = np.ones_like(x)
    return np.stack([rho, rho * u * one, rho * v * one, rho * w * one,
                     one / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)], 1)


def smooth_state3(xyz, seed=0, gamma=1.4):
    """A seeded smooth non-uniform flow on the unit-periodic cube (all five
    fields vary), conserved variables (K, 5, Np)."""
    x, y, z = xyz
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 6)
    two = 2 * np.pi
    rho = 1.0 + 0.2 * np.sin(two * x + ph[0]) * np.cos(two * y + ph[1])
    u = 0.3 * np.sin(two * z + ph[2])
    v = 0.2 * np.cos(two * x + ph[3])
    w = -0.1 * np.sin(two * y + ph[4])
    p = 1.0 + 0.1 * np.cos(two * (x + z) + ph[5])
    return np.stack([rho, rho * u, rho * v, rho * w, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)], 1)
