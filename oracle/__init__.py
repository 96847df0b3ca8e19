"""FP64 CPU oracle of the 2D curved-element nodal DG Euler solver.

TEST INFRASTRUCTURE ONLY.  Used by ``tests/``, ``__graft_entry__.smoke()`` and
the benchmark's CPU-baseline leg to check and time the solver; the solver
itself never imports it.
"""
