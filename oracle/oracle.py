"""Python front end of the FP64 CPU oracle (``dg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the solver.  It builds the C core with
gcc on first use (or via :func:`build`), computes the reference operators in
:mod:`oracle.refelem`, and wraps the C entry points with NumPy arrays.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

from .refelem import ref

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

NF = 4


# Second build of the same source whose floating-point expressions are
# contracted into fused multiply-adds wherever the compiler can: the same
# arithmetic in a different rounding order, used to measure how far two valid
# evaluation orders of the oracle differ on ill-conditioned meshes.
LIB_FMA = os.path.join(HERE, "liboracle_fma.so")
FMA_FLAGS = ["-mfma", "-ffp-contract=fast"]


def build(force: bool = True, fma: bool = False) -> str:
    """Compile ``dg_oracle.c`` into ``liboracle.so`` (gcc, -O2, OpenMP, no
    contraction); ``fma``: the contracted build ``liboracle_fma.so``."""
    out = LIB_FMA if fma else LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + f".tmp{os.getpid()}"
    flags = FMA_FLAGS if fma else ["-ffp-contract=off"]
    subprocess.check_call(["gcc", "-O2", *flags, "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, SRC, "-lm"])
    os.replace(tmp, out)
    return out


class _Weak(C.Structure):
    _fields_ = [("ncub", C.c_int), ("ng", C.c_int),
                ("wq", C.c_void_p), ("Icub", C.c_void_p), ("Drc", C.c_void_p), ("Dsc", C.c_void_p),
                ("wg", C.c_void_p), ("If", C.c_void_p), ("Drg", C.c_void_p), ("Dsg", C.c_void_p)]


class _Mesh(C.Structure):
    _fields_ = [
        ("K", C.c_int), ("P", C.c_int), ("Np", C.c_int), ("Nfp", C.c_int),
        ("gamma", C.c_double),
        ("Dr", C.c_void_p), ("Ds", C.c_void_p), ("LIFT", C.c_void_p),
        ("Vinv", C.c_void_p), ("Mref", C.c_void_p), ("Fmask", C.c_void_p),
        ("top_modes", C.c_void_p),
        ("EToE", C.c_void_p), ("EToF", C.c_void_p), ("bc", C.c_void_p),
        ("rx", C.c_void_p), ("sx", C.c_void_p), ("ry", C.c_void_p), ("sy", C.c_void_p),
        ("J", C.c_void_p), ("nx", C.c_void_p), ("ny", C.c_void_p), ("Fscale", C.c_void_p),
        ("freestream", C.c_double * 4),
        ("cfl", C.c_double),
        ("av_enable", C.c_int),
        ("av_eps0", C.c_double), ("av_s0", C.c_double), ("av_kappa", C.c_double),
        ("riemann", C.c_int),
        ("no_euler_flux", C.c_int),
        ("eps_override", C.c_double),
        ("eps", C.c_void_p), ("Q", C.c_void_p),
        ("weak", C.c_void_p), ("x", C.c_void_p), ("y", C.c_void_p),
    ]


_libs = {}


def lib(fma: bool = False):
    """The oracle's C core (``fma``: the contracted build)."""
    if fma not in _libs:
        path = build(force=False, fma=fma)
        L = C.CDLL(path)
        vp, d, i, l = C.c_void_p, C.c_double, C.c_int, C.c_long
        L.oracle_geometry.restype = l
        L.oracle_geometry.argtypes = [vp] + [vp] * 11
        L.oracle_rhs.argtypes = [vp, vp, vp]
        L.oracle_sensor.argtypes = [vp, vp, vp]
        L.oracle_av_gradient.argtypes = [vp, vp, vp, vp]
        L.oracle_dt.restype = d
        L.oracle_dt.argtypes = [vp, vp, vp]
        L.oracle_totals.argtypes = [vp, vp, vp]
        L.oracle_run.restype = d
        L.oracle_run.argtypes = [vp, vp, i, d, vp, vp, vp, vp]
        L.oracle_residual.argtypes = [vp, vp, vp, vp]
        L.oracle_lf_flux.argtypes = [d, vp, vp, d, d, vp]
        L.oracle_hllc_flux.argtypes = [d, vp, vp, d, d, vp]
        L.oracle_ghost.argtypes = [d, i, vp, d, d, vp, vp]
        L.oracle_rk_coefficients.argtypes = [vp, vp]
        L.oracle_set_threads.argtypes = [i]
        L.oracle_max_threads.restype = i
        _libs[fma] = L
    return _libs[fma]


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def set_threads(n: int):
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def rk_coefficients():
    a = np.zeros(5)
    b = np.zeros(5)
    lib().oracle_rk_coefficients(_p(a), _p(b))
    return a, b


def lf_flux(um, up, nx, ny, gamma=1.4):
    um = np.ascontiguousarray(um, dtype=np.float64)
    up = np.ascontiguousarray(up, dtype=np.float64)
    out = np.zeros(4)
    lib().oracle_lf_flux(gamma, _p(um), _p(up), float(nx), float(ny), _p(out))
    return out


def hllc_flux(um, up, nx, ny, gamma=1.4):
    um = np.ascontiguousarray(um, dtype=np.float64)
    up = np.ascontiguousarray(up, dtype=np.float64)
    out = np.zeros(4)
    lib().oracle_hllc_flux(gamma, _p(um), _p(up), float(nx), float(ny), _p(out))
    return out


def ghost(code, um, nx, ny, qinf, gamma=1.4):
    um = np.ascontiguousarray(um, dtype=np.float64)
    qinf = np.ascontiguousarray(qinf, dtype=np.float64)
    out = np.zeros(4)
    lib().oracle_ghost(gamma, int(code), _p(um), float(nx), float(ny), _p(qinf), _p(out))
    return out


def prolong(U, P, Q):
    """State (K, 4, Np(P)) prolonged to order Q (p-refinement)."""
    from .refelem import prolongation
    U = np.ascontiguousarray(U, dtype=np.float64)
    return np.ascontiguousarray(U @ prolongation(P, Q).T)


class Oracle:
    """FP64 oracle bound to one mesh and order.

    ``x``, ``y`` are the (K, Np) node coordinates in this module's node order
    (:func:`oracle.refelem.nodes`).  States are (K, 4, Np) float64 arrays.
    ``fma``: evaluate with the contracted build of the same source.
    ``riemann``: the numerical flux, "lf" (local Lax-Friedrichs) or "hllc".
    ``weak``: the paper's over-integrated weak form (cubature and face Gauss
    rules, per-element mass matrices) instead of the nodal strong form.
    """

    def __init__(self, mesh, P, x, y, freestream=(1.0, 0.0, 0.0, 2.5), gamma=1.4,
                 cfl=0.5, av=False, av_eps0=0.3, av_s0=None, av_kappa=1.0,
                 no_euler_flux=False, eps_override=-1.0, fma=False, riemann="lf", weak=False):
        R = ref(P)
        self._L = lib(fma)
        self.ref = R
        self.P, self.Np, self.Nfp = P, R.Np, R.Nfp
        self.K = int(mesh.K)
        K, Np, Nfp = self.K, self.Np, self.Nfp
        self._keep = []

        def keep(a, dtype):
            a = np.ascontiguousarray(a, dtype=dtype)
            self._keep.append(a)
            return a

        self.Dr = keep(R.Dr, np.float64)
        self.Ds = keep(R.Ds, np.float64)
        self.LIFT = keep(R.LIFT, np.float64)
        self.Vinv = keep(R.Vinv, np.float64)
        self.Mref = keep(R.M, np.float64)
        self.Fmask = keep(R.Fmask, np.int32)
        self.top = keep(R.top_modes, np.int32)
        self.EToE = keep(mesh.EToE, np.int32)
        self.EToF = keep(mesh.EToF, np.int32)
        self.bc = keep(mesh.bc, np.int8)
        x = keep(x, np.float64)
        y = keep(y, np.float64)
        assert x.shape == (K, Np) and y.shape == (K, Np)
        self.x, self.y = x, y
        g = {n: np.zeros((K, Np)) for n in ("rx", "sx", "ry", "sy", "J")}
        fgeo = {n: np.zeros((K, 3 * Nfp)) for n in ("nx", "ny", "sJ", "Fscale")}
        self.geo = {**g, **fgeo}
        self.eps = np.zeros(K)
        self.Q = np.zeros((K, 2, NF, Np))
        m = _Mesh()
        m.K, m.P, m.Np, m.Nfp = K, P, Np, Nfp
        m.gamma = gamma
        m.Dr, m.Ds, m.LIFT = _p(self.Dr).value, _p(self.Ds).value, _p(self.LIFT).value
        m.Vinv, m.Mref, m.Fmask = _p(self.Vinv).value, _p(self.Mref).value, _p(self.Fmask).value
        m.top_modes = _p(self.top).value
        m.EToE, m.EToF, m.bc = _p(self.EToE).value, _p(self.EToF).value, _p(self.bc).value
        for n in ("rx", "sx", "ry", "sy", "J", "nx", "ny", "Fscale"):
            setattr(m, n, _p(self.geo[n]).value)
        for c in range(4):
            m.freestream[c] = float(freestream[c])
        m.cfl = cfl
        m.av_enable = 1 if av else 0
        m.av_eps0 = av_eps0
        m.av_s0 = -4.0 * math.log10(P) if av_s0 is None or (isinstance(av_s0, float) and math.isnan(av_s0)) else av_s0
        m.av_kappa = av_kappa
        if riemann not in ("lf", "hllc"):
            raise ValueError("riemann must be 'lf' or 'hllc'")
        m.riemann = 1 if riemann == "hllc" else 0
        m.no_euler_flux = 1 if no_euler_flux else 0
        m.eps_override = eps_override
        m.eps, m.Q = _p(self.eps).value, _p(self.Q).value
        self.weak = bool(weak)
        if weak:
            if av or eps_override >= 0.0 or no_euler_flux:
                raise ValueError("the weak form is inviscid")
            from .refelem import weak_ops
            W = weak_ops(P)
            wk = _Weak()
            wk.ncub, wk.ng = W.ncub, W.ng
            for name in ("wq", "Icub", "Drc", "Dsc", "wg", "If", "Drg", "Dsg"):
                setattr(wk, name, _p(keep(getattr(W, name), np.float64)).value)
            self._weak = wk
            m.weak = C.addressof(wk)
            m.x, m.y = _p(x).value, _p(y).value
        self.m = m
        self.bad_jacobians = self._L.oracle_geometry(
            C.byref(m), _p(x), _p(y), *(_p(self.geo[n]) for n in
                                         ("rx", "sx", "ry", "sy", "J", "nx", "ny", "sJ", "Fscale")))

    @classmethod
    def for_case(cls, case, **kw):
        """Oracle for a :class:`meshgen.cases.Case` built at this module's nodes."""
        args = dict(freestream=case.freestream, gamma=case.gamma, cfl=case.cfl,
                    av=case.av, av_eps0=case.av_eps0, av_kappa=case.av_kappa,
                    av_s0=None if math.isnan(case.av_s0) else case.av_s0)
        args.update(kw)
        return cls(case.mesh, case.P, case.x, case.y, **args)

    def _state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (self.K, NF, self.Np)
        return U

    def rhs(self, U):
        U = self._state(U)
        out = np.empty_like(U)
        self._L.oracle_rhs(C.byref(self.m), _p(U), _p(out))
        return out

    def sensor(self, U):
        U = self._state(U)
        eps = np.empty(self.K)
        self._L.oracle_sensor(C.byref(self.m), _p(U), _p(eps))
        return eps

    def av_gradient(self, U, eps):
        U = self._state(U)
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        Q = np.empty((self.K, 2, NF, self.Np))
        self._L.oracle_av_gradient(C.byref(self.m), _p(U), _p(eps), _p(Q))
        return Q

    def dt(self, U):
        U = self._state(U)
        flag = C.c_int(0)
        d = self._L.oracle_dt(C.byref(self.m), _p(U), C.byref(flag))
        return d, flag.value

    def totals(self, U):
        U = self._state(U)
        out = np.zeros(4)
        self._L.oracle_totals(C.byref(self.m), _p(U), _p(out))
        return out

    def residual(self, U):
        U = self._state(U)
        scratch = np.empty_like(U)
        out = np.zeros(4)
        self._L.oracle_residual(C.byref(self.m), _p(U), _p(scratch), _p(out))
        return out

    def run(self, U, nsteps, dt=0.0):
        """Advance a copy of U by nsteps LSERK steps; returns (U, info)."""
        U = self._state(U).copy()
        R = np.zeros_like(U)
        scratch = np.zeros_like(U)
        mm = np.zeros(2)
        flag = C.c_int(0)
        t = self._L.oracle_run(C.byref(self.m), _p(U), int(nsteps), float(dt), _p(R),
                             _p(scratch), _p(mm), C.byref(flag))
        return U, dict(t=t, dt_min=mm[0], dt_max=mm[1], flag=flag.value)
