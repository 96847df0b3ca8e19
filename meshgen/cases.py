"""The five synthetic workloads, with their sizes, seeds and flow parameters.

``make_case(name, r, s)`` builds the mesh, evaluates the node positions at the
caller's reference nodes (r, s) and returns the initial state.  ``scale``
shrinks a case for quick tests while keeping its structure.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import flows, meshes


@dataclass
class Case:
    name: str
    P: int
    mesh: meshes.Mesh
    x: np.ndarray
    y: np.ndarray
    U0: np.ndarray                 # (K,4,Np) float64
    freestream: np.ndarray         # (4,)
    gamma: float = flows.GAMMA
    cfl: float = 0.5
    steps: int = 100
    av: bool = False
    av_eps0: float = 0.3
    av_kappa: float = 1.0
    av_s0: float = float("nan")    # nan: -4 log10 P
    info: dict = field(default_factory=dict)

    @property
    def K(self):
        return self.mesh.K

    @property
    def Np(self):
        return (self.P + 1) * (self.P + 2) // 2

    def dofs(self):
        return 4 * self.Np * self.K


CASES = ("vortex", "cylinder", "airfoil", "roofline", "roofline_curved")


def _wall_points(mesh):
    """Vertices of the wall faces (x, y)."""
    k, f = np.nonzero(mesh.bc == meshes.BC_WALL)
    v = mesh.EToV[k[:, None], np.asarray(meshes.FACE_VERTS)[f]]
    return mesh.VX[v].ravel(), mesh.VY[v].ravel()


def _np_of(P):
    return (P + 1) * (P + 2) // 2


def make_case(name: str, r, s, scale: float = 1.0, P: int | None = None,
              mach: float | None = None, steps: int | None = None,
              start: str = "freestream") -> Case:
    """Build one of ``CASES``.  ``scale`` < 1 shrinks the element count.
    ``start`` for the cylinder and the airfoil: "freestream" (impulsive),
    "potential" (the wall-compatible potential flow: closed form for the
    cylinder, a panel solution for the airfoil) or "damped" (the freestream
    with its velocity damped to rest at the wall)."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    if name == "vortex":
        # 2x16x16 jittered, permuted periodic square; isentropic vortex; P=2.
        P = 2 if P is None else P
        N = max(3, int(round(16 * math.sqrt(scale))))
        mesh = meshes.periodic_square(N, 10.0, 0.1, 1208, 4772)
        x, y = meshes.node_coordinates(mesh, r, s)
        U0 = flows.isentropic_vortex(x, y)
        q = flows.primitive_to_conserved(1.0, 1.0, 0.0, 1.0)   # rho=1, u=1, p=1
        return Case(name, P, mesh, x, y, U0, np.asarray(q, dtype=np.float64).ravel(),
                    steps=100 if steps is None else steps)
    if name == "cylinder":
        P = 4 if P is None else P
        nt = max(8, int(round(200 * math.sqrt(scale))))
        nr = max(2, int(round(50 * math.sqrt(scale))))
        mesh = meshes.cylinder_annulus(nt, nr, 1.0, 20.0, 0.1, 38, True)
        x, y = meshes.node_coordinates(mesh, r, s)
        M = 0.38 if mach is None else mach
        q = flows.freestream_state(M, 0.0)
        if start == "potential":
            U0 = np.ascontiguousarray(flows.cylinder_potential(x, y, M))
        elif start == "damped":
            U0 = flows.wall_damped(x, y, *_wall_points(mesh), q)
        else:
            U0 = flows.uniform((mesh.K, x.shape[1]), q)
        return Case(name, P, mesh, x, y, U0, q, steps=2000 if steps is None else steps,
                    info=dict(mach=M, alpha=0.0))
    if name == "airfoil":
        P = 3 if P is None else P
        nt = max(16, int(round(600 * math.sqrt(scale))))
        nr = max(4, int(round(100 * math.sqrt(scale))))
        growth = 1.06 ** (100.0 / nr)
        mesh = meshes.naca4_ogrid(nt, nr, 0.12, 30.0, growth, 0.02, 80, True)
        x, y = meshes.node_coordinates(mesh, r, s)
        M = 0.8 if mach is None else mach
        q = flows.freestream_state(M, 1.25)
        if start == "damped":
            U0 = flows.wall_damped(x, y, *_wall_points(mesh), q)
        elif start == "potential":
            U0 = flows.airfoil_potential(x, y, M, 1.25)
        elif start == "freestream":
            U0 = flows.uniform((mesh.K, x.shape[1]), q)
        else:
            raise ValueError(f"start {start!r} is not available for the airfoil")
        return Case(name, P, mesh, x, y, U0, q, steps=2000 if steps is None else steps,
                    av=True, av_eps0=0.3, av_kappa=1.0,
                    info=dict(mach=M, alpha=1.25))
    if name in ("roofline", "roofline_curved"):
        # ~1.0e6 triangles (N=707), P=5, jittered straight (or all curved),
        # grid element order (no permutation).
        P = 5 if P is None else P
        N = max(3, int(round(707 * math.sqrt(scale))))
        amp = 0.05 if name == "roofline_curved" else 0.0
        mesh = meshes.periodic_square(N, 10.0, 0.1, 5, None, amp)
        x, y = meshes.node_coordinates(mesh, r, s)
        U0 = flows.isentropic_vortex(x, y)
        q = flows.primitive_to_conserved(1.0, 1.0, 0.0, 1.0)
        return Case(name, P, mesh, x, y, U0, np.asarray(q, dtype=np.float64).ravel(),
                    steps=200 if steps is None else steps)
    raise ValueError(f"unknown case {name!r}; one of {CASES}")
