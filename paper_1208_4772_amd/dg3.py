"""Binding of the 3D solver (the C ABI in ``include/dg3.h``): nodal DG for
the Euler equations on straight tetrahedra, five conserved fields.

Argument marshalling only, as :mod:`paper_1208_4772_amd.dg`: the library's
HIP kernels do every step; torch provides device memory and the stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .dg import (DG_FP64_PLAIN, PRECISIONS, RunStats, Stats, _check, _p, _stream_handle, lib)


class MeshDesc3(C.Structure):
    _fields_ = [("K", C.c_int), ("P", C.c_int), ("precision", C.c_int),
                ("EToV", C.c_void_p), ("EToE", C.c_void_p), ("EToF", C.c_void_p), ("bc", C.c_void_p),
                ("X", C.c_void_p), ("gamma", C.c_double), ("cfl", C.c_double)]


def n_nodes3(P):
    return (P + 1) * (P + 2) * (P + 3) // 6


def reference_nodes3(P: int):
    Np = n_nodes3(P)
    r, s, t = np.zeros(Np), np.zeros(Np), np.zeros(Np)
    _check(lib().dg3_reference_nodes(int(P), _p(r), _p(s), _p(t)))
    return r, s, t


def reference_operators3(P: int):
    """The library's reference operators of order P (host arrays)."""
    Np, Nfp = n_nodes3(P), (P + 1) * (P + 2) // 2
    out = dict(Dr=np.zeros((Np, Np)), Ds=np.zeros((Np, Np)), Dt=np.zeros((Np, Np)),
               LIFT=np.zeros((Np, 4 * Nfp)), fmask=np.zeros((4, Nfp), dtype=np.int32))
    _check(lib().dg3_reference_operators(int(P), *(_p(out[k]) for k in ("Dr", "Ds", "Dt", "LIFT", "fmask"))))
    return out


def _desc(EToV, EToE, EToF, bc, X, P, precision, gamma, cfl):
    keep = [np.ascontiguousarray(EToV, dtype=np.int32), np.ascontiguousarray(EToE, dtype=np.int32),
            np.ascontiguousarray(EToF, dtype=np.int32), np.ascontiguousarray(bc, dtype=np.int8),
            np.ascontiguousarray(X, dtype=np.float64)]
    e2v, e2e, e2f, b, xx = keep
    K = int(e2e.shape[0])
    for a in (e2v, e2e, e2f, b):
        if a.shape != (K, 4):
            raise ValueError("connectivity arrays must be (K, 4)")
    if xx.shape != (K, 4, 3):
        raise ValueError("X must be (K, 4, 3)")
    d = MeshDesc3()
    d.K, d.P, d.precision = K, int(P), PRECISIONS[precision]
    d.EToV, d.EToE, d.EToF, d.bc, d.X = (_p(a).value for a in keep)
    d.gamma, d.cfl = float(gamma), float(cfl)
    return d, keep


def face_map3(EToV, EToE, EToF, bc, X, P, precision="fp64", gamma=1.4, cfl=0.5):
    """The library's neighbour node map (K, 4 Nfp) of a mesh (host only):
    offsets kn * 5 * Np + node into a [K][5][Np] state, -1 at walls."""
    d, keep = _desc(EToV, EToE, EToF, bc, X, P, precision, gamma, cfl)
    out = np.zeros((d.K, 4 * ((P + 1) * (P + 2) // 2)), dtype=np.int32)
    _check(lib().dg3_face_map(C.byref(d), _p(out)))
    return out


class Solver3D:
    """One tetrahedral mesh on one GPU.  States are torch tensors (K, 5, Np)
    on the device, float64 for ``fp64`` and float32 for ``fp32``.

    EToV, EToE, EToF: (K, 4) int; bc: (K, 4) with 0 interior, 1 slip wall;
    X: (K, 4, 3) vertex coordinates of each element (positively oriented)."""

    def __init__(self, EToV, EToE, EToF, bc, X, P, precision="fp32", gamma=1.4, cfl=0.5, device="cuda:0"):
        import torch
        if precision not in ("fp64", "fp64_plain", "fp32"):
            raise ValueError("precision must be fp64 or fp32")
        self.torch = torch
        self.device = torch.device(device)
        self.P = int(P)
        self.Np = n_nodes3(self.P)
        self.precision = precision
        self.dtype = torch.float64 if PRECISIONS[precision] == DG_FP64_PLAIN else torch.float32
        d, self._keep = _desc(EToV, EToE, EToF, bc, X, P, precision, gamma, cfl)
        self.K = d.K
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().dg3_mesh_setup(C.byref(d), _stream_handle(), C.byref(self._h)))
        sb, wb = C.c_size_t(), C.c_size_t()
        _check(lib().dg3_buffer_bytes(self._h, C.byref(sb), C.byref(wb)))
        self.state_bytes, self.work_bytes = sb.value, wb.value
        self.work = torch.empty(self.work_bytes, dtype=torch.uint8, device=self.device)

    @classmethod
    def from_mesh(cls, mesh, P, **kw):
        """Solver for a mesh object with EToV, EToE, EToF, bc and X."""
        return cls(mesh.EToV, mesh.EToE, mesh.EToF, mesh.bc, mesh.X, P, **kw)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dg3_mesh_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state(self, U_host):
        """Device state from a host float64 array (K, 5, Np)."""
        t = self.torch.as_tensor(np.ascontiguousarray(U_host, dtype=np.float64))
        if tuple(t.shape) != (self.K, 5, self.Np):
            raise ValueError(f"state must have shape {(self.K, 5, self.Np)}")
        return t.to(self.device).to(self.dtype).contiguous()

    def empty_state(self):
        return self.torch.empty((self.K, 5, self.Np), dtype=self.dtype, device=self.device)

    def _check_state(self, U):
        if U.dtype != self.dtype or not U.is_contiguous() or tuple(U.shape) != (self.K, 5, self.Np):
            raise ValueError(f"state must be a contiguous {self.dtype} tensor of shape {(self.K, 5, self.Np)}")
        if U.device != self.device:
            raise ValueError(f"state must live on {self.device}")

    def rhs(self, U, out=None, stream=None):
        self._check_state(U)
        out = self.empty_state() if out is None else out
        self._check_state(out)
        _check(lib().dg3_rhs(self._h, C.c_void_p(U.data_ptr()), C.c_void_p(out.data_ptr()),
                             _stream_handle(stream)))
        return out

    def run(self, U, nsteps, dt=0.0, stream=None, check=True):
        """nsteps LSERK steps of U in place (dt > 0: fixed step, else CFL)."""
        self._check_state(U)
        st = RunStats()
        rc = lib().dg3_run(self._h, C.c_void_p(U.data_ptr()), C.c_void_p(self.work.data_ptr()), int(nsteps),
                           float(dt), C.byref(st), _stream_handle(stream))
        if check:
            _check(rc)
        return Stats(st.steps, st.status, st.t, st.dt_min, st.dt_max, tuple(st.totals), tuple(st.residual),
                     st.wall_s, st.dof_updates_per_s)

    def dofs(self):
        return self.K * 5 * self.Np
