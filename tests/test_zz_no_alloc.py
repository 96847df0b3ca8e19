"""dg_step_static, the step that allocates nothing (its work buffer is the
library's static device area), against dg_step with a caller work buffer:
the same bits, on two meshes in a row (the second smaller, so it runs on
what the first left in the area), through the raw C ABI."""
import ctypes as C

import numpy as np
import pytest

import meshgen
from oracle.refelem import ref

pytestmark = pytest.mark.gpu


def dg():
    from paper_1208_4772_amd import dg as _dg
    return _dg


def solver(mesh, P, q, precision, av=False):
    R = ref(P)
    x, y = meshgen.node_coordinates(mesh, R.r, R.s)
    kw = dict(av=True, av_kappa=1.0, av_eps0=0.3) if av else {}
    s = dg().Solver(mesh.EToE, mesh.EToF, mesh.bc, x, y, P, precision, freestream=q, **kw)
    return s, x, y


def perturbed(x, y, q, amp=0.02):
    rho0, u0, v0 = q[0], q[1] / q[0], q[2] / q[0]
    p0 = 0.4 * (q[3] - 0.5 * rho0 * (u0 * u0 + v0 * v0))
    return meshgen.primitive_to_conserved(rho0 * (1 + amp * np.sin(x) * np.cos(0.7 * y)),
                                          u0 + amp * np.sin(0.9 * y), v0 + amp * np.cos(1.1 * x),
                                          p0 * (1 + amp * np.cos(x + 0.5 * y)))


@pytest.mark.parametrize("precision", ["fp32", "fp64", "bf16x3"])
def test_static_step_equals_step_with_work_buffer(precision):
    import torch
    L = dg().lib()
    cases = [
        (meshgen.naca4_ogrid(40, 8), 3, meshgen.freestream_state(0.7, 1.25), True),      # larger, viscous
        (meshgen.cylinder_annulus(16, 4), 2, meshgen.freestream_state(0.38), False),    # smaller
    ]
    for n, (mesh, P, q, av) in enumerate(cases):
        s, x, y = solver(mesh, P, q, precision, av)
        U0 = perturbed(x, y, q)
        a = s.state(U0)
        b = s.state(U0)
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        for _ in range(3):
            s.step(a)
            rc = L.dg_step_static(s._h, C.c_void_p(b.data_ptr()), 0.0, st)
            assert rc == 0, L.dg_last_error()
        torch.cuda.synchronize()
        print(f"[static step {precision} case {n}] K={mesh.K} bitwise {bool(torch.equal(a, b))}")
        assert torch.equal(a, b)
        s.close()


def test_static_step_rejects_a_mesh_beyond_the_area():
    import torch
    L = dg().lib()
    mesh = meshgen.periodic_square(260, perm_seed=None)
    q = np.array([1.0, 1.0, 0.0, 1.0 / 0.4 + 0.5])
    s, x, y = solver(mesh, 5, q, "fp64")
    state_b, work_b = C.c_size_t(), C.c_size_t()
    L.dg_buffer_bytes(s._h, C.byref(state_b), C.byref(work_b))
    assert work_b.value > (256 << 20)
    U = s.empty_state()
    rc = L.dg_step_static(s._h, C.c_void_p(U.data_ptr()), 0.0,
                          C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == dg().DG_EINVAL
    assert "static work area" in L.dg_last_error().decode()
    s.close()
