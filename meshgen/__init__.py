"""Seeded synthetic inputs (meshes, node positions, initial states).

Shared by the solver's tests and benchmarks and by the CPU oracle's tests; it
holds no DG arithmetic.
"""
from .meshes import (BC_FARFIELD, BC_INTERIOR, BC_WALL, FACE_VERTS, Mesh,  # noqa: F401
                     channel, connect, cylinder_annulus, naca4_ogrid, naca4_thickness,
                     naca_point, node_coordinates, periodic_square,
                     permute_elements)
from .flows import (GAMMA, airfoil_panels, airfoil_potential, airfoil_velocity,  # noqa: F401
                    cylinder_potential, freestream_state,
                    isentropic_vortex, primitive_to_conserved, uniform,
                    wall_damped)
from .cases import CASES, make_case  # noqa: F401
