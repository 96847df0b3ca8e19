"""MI355X (gfx950) nodal DG solver for the 2D Euler equations on curved
triangles: HIP kernels behind the C ABI in ``include/dg.h`` and a thin
Python binding (:mod:`paper_1208_4772_amd.dg`)."""
