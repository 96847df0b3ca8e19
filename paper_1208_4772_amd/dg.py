"""Thin Python binding of ``libdg.so`` (the C ABI in ``include/dg.h``).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch provides device memory (``torch.Tensor.data_ptr()``)
and the stream (``torch.cuda.current_stream().cuda_stream``).  Loading fails
loudly if the library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# DG_LIBRARY may point at another build of the same library (same ABI).
LIB_PATH = os.environ.get("DG_LIBRARY") or os.path.join(HERE, "libdg.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EGEOM, DG_ENONFINITE, DG_EDEVICE, DG_EBUSY = 0, -1, -2, -3, -4, -5, -6
DG_FP64_PLAIN, DG_FP32, DG_FP32_BF16X3 = 0, 2, 3
PRECISIONS = {"fp64": DG_FP64_PLAIN, "fp64_plain": DG_FP64_PLAIN, "fp32": DG_FP32,
              "bf16x3": DG_FP32_BF16X3}
DG_RIEMANN_LF, DG_RIEMANN_HLLC = 0, 1
RIEMANN = {"lf": DG_RIEMANN_LF, "hllc": DG_RIEMANN_HLLC}
DG_FORM_NODAL, DG_FORM_WEAK = 0, 1
FORMS = {"nodal": DG_FORM_NODAL, "weak": DG_FORM_WEAK}

# Every symbol include/dg.h declares.
EXPORTS = ("dg_last_error", "dg_version", "dg_reference_nodes", "dg_face_nodes",
           "dg_reference_operators", "dg_mesh_setup", "dg_mesh_destroy", "dg_buffer_bytes",
           "dg_rhs", "dg_step", "dg_run", "dg_totals", "dg_residual", "dg_viscosity",
           "dg_set_graphs", "dg_set_kernel_timing", "dg_kernel_time", "dg_autotune", "dg_mesh_footprint",
           "dg_estimate_footprint", "dg_batch_create", "dg_batch_destroy", "dg_batch_admit",
           "dg_batch_advance", "dg_batch_poll", "dg_batch_slot_stats", "dg_batch_release",
           "dg_status", "dg_step_static", "dg_prolong_operator", "dg_prolong", "dg_weak_operators",
           "dg_batch_info", "dg_tuning_set", "dg_tuning_lookup", "dg_tuning_clear", "dg_tuning_save",
           "dg_tuning_load", "dg_device_arch", "dg_mesh_curved")
# Every symbol include/dg3.h declares.
EXPORTS3 = ("dg3_reference_nodes", "dg3_reference_operators", "dg3_face_map", "dg3_mesh_setup",
            "dg3_mesh_destroy", "dg3_buffer_bytes", "dg3_rhs", "dg3_run")


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("K", C.c_int), ("P", C.c_int), ("precision", C.c_int),
                ("gamma", C.c_double), ("cfl", C.c_double),
                ("EToE", C.c_void_p), ("EToF", C.c_void_p), ("bc", C.c_void_p),
                ("x", C.c_void_p), ("y", C.c_void_p),
                ("freestream", C.c_double * 4),
                ("av_enable", C.c_int), ("av_eps0", C.c_double), ("av_s0", C.c_double),
                ("av_kappa", C.c_double), ("riemann", C.c_int), ("form", C.c_int)]


class RunStats(C.Structure):
    _fields_ = [("steps", C.c_int), ("status", C.c_int), ("t", C.c_double),
                ("dt_min", C.c_double), ("dt_max", C.c_double),
                ("totals", C.c_double * 4), ("residual", C.c_double * 4),
                ("wall_s", C.c_double), ("dof_updates_per_s", C.c_double)]


_lib = None


def lib():
    """Load ``libdg.so`` (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1208_4772_amd.build`")
        # torch first: the library then binds to the HIP runtime torch has
        # already loaded (same soname) instead of bringing a second one into
        # the process, which would not see the device
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        L.dg_last_error.restype = C.c_char_p
        L.dg_version.restype = i
        L.dg_reference_nodes.argtypes = [i, vp, vp]
        L.dg_face_nodes.argtypes = [i, vp]
        L.dg_reference_operators.argtypes = [i, vp, vp, vp, vp]
        L.dg_mesh_setup.argtypes = [C.POINTER(MeshDesc), vp, C.POINTER(vp)]
        L.dg_mesh_destroy.argtypes = [vp]
        L.dg_buffer_bytes.argtypes = [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.dg_rhs.argtypes = [vp, vp, vp, d, vp]
        L.dg_step.argtypes = [vp, vp, vp, d, vp]
        L.dg_step_static.argtypes = [vp, vp, d, vp]
        L.dg_prolong_operator.argtypes = [i, i, vp]
        L.dg_weak_operators.argtypes = [i, C.POINTER(i), C.POINTER(i), vp, vp, vp, vp, vp, vp]
        L.dg_prolong.argtypes = [vp, vp, vp, vp, vp]
        L.dg_run.argtypes = [vp, vp, vp, i, C.POINTER(RunStats), vp]
        L.dg_totals.argtypes = [vp, vp, vp, vp]
        L.dg_residual.argtypes = [vp, vp, vp, vp, vp]
        L.dg_viscosity.argtypes = [vp, vp, vp, vp]
        L.dg_status.argtypes = [vp, vp, C.POINTER(i)]
        L.dg_set_kernel_timing.argtypes = [vp, i]
        L.dg_set_graphs.argtypes = [vp, i]
        sz = C.c_size_t
        L.dg_mesh_footprint.argtypes = [vp, C.POINTER(sz)]
        L.dg_estimate_footprint.argtypes = [i, i, i, i, C.POINTER(sz)]
        L.dg_batch_create.argtypes = [sz, i, C.POINTER(vp)]
        L.dg_batch_destroy.argtypes = [vp]
        L.dg_batch_admit.argtypes = [vp, vp, vp, vp, i, vp, C.POINTER(i)]
        L.dg_batch_advance.argtypes = [vp, i, vp, C.POINTER(i)]
        L.dg_batch_poll.argtypes = [vp, vp, vp, i, C.POINTER(i)]
        L.dg_batch_slot_stats.argtypes = [vp, i, vp, C.POINTER(RunStats)]
        L.dg_batch_release.argtypes = [vp, i]
        L.dg_batch_info.argtypes = [vp, C.POINTER(i), C.POINTER(i)]
        L.dg_kernel_time.argtypes = [vp, vp, C.POINTER(d), C.POINTER(C.c_long)]
        L.dg_autotune.argtypes = [vp, vp, vp, vp, C.POINTER(i), C.POINTER(d)]
        cp = C.c_char_p
        L.dg_tuning_set.argtypes = [cp, i, i, i, i]
        L.dg_tuning_lookup.argtypes = [cp, i, i, i, C.POINTER(i)]
        L.dg_tuning_clear.argtypes = []
        L.dg_tuning_save.argtypes = [cp, C.POINTER(i)]
        L.dg_tuning_load.argtypes = [cp, C.POINTER(i)]
        L.dg_device_arch.argtypes = [C.c_char_p, sz]
        L.dg_mesh_curved.argtypes = [vp, C.POINTER(i)]
        # the 3D ABI (include/dg3.h)
        L.dg3_reference_nodes.argtypes = [i, vp, vp, vp]
        L.dg3_reference_operators.argtypes = [i, vp, vp, vp, vp, vp]
        L.dg3_face_map.argtypes = [vp, vp]
        L.dg3_mesh_setup.argtypes = [vp, vp, C.POINTER(vp)]
        L.dg3_mesh_destroy.argtypes = [vp]
        L.dg3_buffer_bytes.argtypes = [vp, C.POINTER(sz), C.POINTER(sz)]
        L.dg3_rhs.argtypes = [vp, vp, vp, vp]
        L.dg3_run.argtypes = [vp, vp, vp, i, d, C.POINTER(RunStats), vp]
        for name in EXPORTS + EXPORTS3:
            getattr(L, name).restype = getattr(L, name).restype or i
        _lib = L
    return _lib


def _check(rc):
    if rc != DG_OK:
        msg = lib().dg_last_error().decode(errors="replace")
        raise DGError(rc, msg)
    return rc


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def n_nodes(P):
    return (P + 1) * (P + 2) // 2


def reference_nodes(P: int):
    Np = n_nodes(P)
    r = np.zeros(Np)
    s = np.zeros(Np)
    _check(lib().dg_reference_nodes(P, _p(r), _p(s)))
    return r, s


def face_nodes(P: int):
    fm = np.zeros(3 * (P + 1), dtype=np.int32)
    _check(lib().dg_face_nodes(P, _p(fm)))
    return fm.reshape(3, P + 1)


def reference_operators(P: int):
    Np, Nfp = n_nodes(P), P + 1
    Dr = np.zeros((Np, Np))
    Ds = np.zeros((Np, Np))
    LIFT = np.zeros((Np, 3 * Nfp))
    Vinv = np.zeros((Np, Np))
    _check(lib().dg_reference_operators(P, _p(Dr), _p(Ds), _p(LIFT), _p(Vinv)))
    return dict(Dr=Dr, Ds=Ds, LIFT=LIFT, Vinv=Vinv)


def weak_operators(P: int):
    """The library's weak-form operators of order P (host arrays)."""
    nq, ng = C.c_int(), C.c_int()
    _check(lib().dg_weak_operators(int(P), C.byref(nq), C.byref(ng), None, None, None, None, None, None))
    Np, Nfp = n_nodes(P), P + 1
    out = dict(wq=np.zeros(nq.value), Icub=np.zeros((nq.value, Np)), Drc=np.zeros((nq.value, Np)),
               Dsc=np.zeros((nq.value, Np)), wg=np.zeros(ng.value), If=np.zeros((ng.value, Nfp)))
    _check(lib().dg_weak_operators(int(P), C.byref(nq), C.byref(ng), *(_p(out[k]) for k in
                                                                       ("wq", "Icub", "Drc", "Dsc", "wg", "If"))))
    return out


def prolong_operator(P: int, Q: int):
    """(Np(Q), Np(P)) prolongation matrix of the library (p-refinement)."""
    I = np.zeros((n_nodes(Q), n_nodes(P)))
    _check(lib().dg_prolong_operator(int(P), int(Q), _p(I)))
    return I


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class Stats:
    steps: int
    status: int
    t: float
    dt_min: float
    dt_max: float
    totals: tuple
    residual: tuple
    wall_s: float
    dof_updates_per_s: float


class Solver:
    """One mesh on one GPU.  States are torch tensors (K, 4, Np) on the
    device in the handle's precision (float64 for ``fp64``, float32 for
    ``fp32``)."""

    def __init__(self, EToE, EToF, bc, x, y, P, precision="fp32", gamma=1.4, cfl=0.5,
                 freestream=(1.0, 0.0, 0.0, 2.5), av=False, av_eps0=0.3, av_s0=float("nan"),
                 av_kappa=1.0, riemann="lf", form="nodal", device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.P = int(P)
        self.Np = n_nodes(self.P)
        self.precision = precision
        self.dtype = torch.float64 if PRECISIONS[precision] == DG_FP64_PLAIN else torch.float32
        self._keep = [np.ascontiguousarray(EToE, dtype=np.int32),
                      np.ascontiguousarray(EToF, dtype=np.int32),
                      np.ascontiguousarray(bc, dtype=np.int8),
                      np.ascontiguousarray(x, dtype=np.float64),
                      np.ascontiguousarray(y, dtype=np.float64)]
        e2e, e2f, b, xx, yy = self._keep
        self.K = int(e2e.shape[0])
        assert xx.shape == (self.K, self.Np) and yy.shape == (self.K, self.Np)
        d = MeshDesc()
        d.K, d.P, d.precision = self.K, self.P, PRECISIONS[precision]
        d.gamma, d.cfl = gamma, cfl
        d.EToE, d.EToF, d.bc = _p(e2e).value, _p(e2f).value, _p(b).value
        d.x, d.y = _p(xx).value, _p(yy).value
        for c in range(4):
            d.freestream[c] = float(freestream[c])
        d.av_enable = 1 if av else 0
        d.av_eps0 = av_eps0
        d.av_s0 = av_s0 if av_s0 is not None else float("nan")
        d.av_kappa = av_kappa
        if riemann not in RIEMANN:
            raise ValueError(f"riemann must be one of {sorted(RIEMANN)}")
        d.riemann = RIEMANN[riemann]
        if form not in FORMS:
            raise ValueError(f"form must be one of {sorted(FORMS)}")
        d.form = FORMS[form]
        self.av = bool(av)
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().dg_mesh_setup(C.byref(d), _stream_handle(), C.byref(self._h)))
        sb, wb = C.c_size_t(), C.c_size_t()
        _check(lib().dg_buffer_bytes(self._h, C.byref(sb), C.byref(wb)))
        self.state_bytes, self.work_bytes = sb.value, wb.value
        self.work = torch.empty(self.work_bytes, dtype=torch.uint8, device=self.device)

    @classmethod
    def from_case(cls, case, precision="fp32", x=None, y=None, **kw):
        """Solver for a :class:`meshgen.cases.Case` (its x, y unless given)."""
        m = case.mesh
        args = dict(gamma=case.gamma, cfl=case.cfl, freestream=case.freestream, av=case.av,
                    av_eps0=case.av_eps0, av_kappa=case.av_kappa, av_s0=case.av_s0)
        args.update(kw)
        return cls(m.EToE, m.EToF, m.bc, case.x if x is None else x, case.y if y is None else y,
                   case.P, precision, **args)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dg_mesh_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- states -------------------------------------------------------------
    def state(self, U_host):
        """Device state from a host float64 array (K, 4, Np)."""
        t = self.torch.as_tensor(np.ascontiguousarray(U_host, dtype=np.float64))
        assert tuple(t.shape) == (self.K, 4, self.Np)
        return t.to(self.device).to(self.dtype).contiguous()

    def empty_state(self):
        return self.torch.empty((self.K, 4, self.Np), dtype=self.dtype, device=self.device)

    def _check_state(self, U):
        if U.dtype != self.dtype or not U.is_contiguous() or tuple(U.shape) != (self.K, 4, self.Np):
            raise ValueError(f"state must be a contiguous {self.dtype} tensor of shape "
                             f"{(self.K, 4, self.Np)}")
        if U.device != self.device:
            raise ValueError(f"state must live on {self.device}")

    # -- solver calls -------------------------------------------------------
    def rhs(self, U, out=None, stream=None):
        self._check_state(U)
        out = self.empty_state() if out is None else out
        self._check_state(out)
        _check(lib().dg_rhs(self._h, C.c_void_p(U.data_ptr()), C.c_void_p(out.data_ptr()), 0.0,
                            _stream_handle(stream)))
        return out

    def step(self, U, dt=0.0, stream=None):
        self._check_state(U)
        _check(lib().dg_step(self._h, C.c_void_p(U.data_ptr()), C.c_void_p(self.work.data_ptr()),
                             float(dt), _stream_handle(stream)))
        return U

    def step_static(self, U, dt=0.0, stream=None):
        """One step with the library's static work area instead of this
        solver's work buffer (dg_step_static)."""
        self._check_state(U)
        _check(lib().dg_step_static(self._h, C.c_void_p(U.data_ptr()), float(dt), _stream_handle(stream)))
        return U

    def prolong_from(self, other, U_other, stream=None):
        """This solver's state (order Q) prolonged from the state of `other`
        (same elements, order P <= Q)."""
        other._check_state(U_other)
        out = self.empty_state()
        _check(lib().dg_prolong(other._h, C.c_void_p(U_other.data_ptr()), self._h, C.c_void_p(out.data_ptr()),
                                _stream_handle(stream)))
        return out

    def run(self, U, nsteps, stream=None, check=True):
        self._check_state(U)
        st = RunStats()
        rc = lib().dg_run(self._h, C.c_void_p(U.data_ptr()), C.c_void_p(self.work.data_ptr()),
                          int(nsteps), C.byref(st), _stream_handle(stream))
        if check:
            _check(rc)
        return Stats(st.steps, st.status, st.t, st.dt_min, st.dt_max, tuple(st.totals),
                     tuple(st.residual), st.wall_s, st.dof_updates_per_s)

    def totals(self, U, stream=None):
        self._check_state(U)
        out = np.zeros(4)
        _check(lib().dg_totals(self._h, C.c_void_p(U.data_ptr()), _p(out), _stream_handle(stream)))
        return out

    def residual(self, U, stream=None):
        self._check_state(U)
        out = np.zeros(4)
        _check(lib().dg_residual(self._h, C.c_void_p(U.data_ptr()), C.c_void_p(self.work.data_ptr()),
                                 _p(out), _stream_handle(stream)))
        return out

    def viscosity(self, U, stream=None):
        self._check_state(U)
        eps = self.torch.empty(self.K, dtype=self.torch.float64, device=self.device)
        _check(lib().dg_viscosity(self._h, C.c_void_p(U.data_ptr()), C.c_void_p(eps.data_ptr()),
                                  _stream_handle(stream)))
        return eps

    def autotune(self, U, stream=None):
        """Pick the stage kernel's workgroup shape (2, 4 or 8 wavefronts) by
        timing (matrix-core path only), or take the tuning table's entry for
        this kind of handle (then the time is 0); returns (waves_per_block,
        us per launch)."""
        self._check_state(U)
        b, us = C.c_int(0), C.c_double(0.0)
        _check(lib().dg_autotune(self._h, C.c_void_p(U.data_ptr()), C.c_void_p(self.work.data_ptr()),
                                 _stream_handle(stream), C.byref(b), C.byref(us)))
        return b.value, us.value

    def set_graphs(self, enable=True):
        _check(lib().dg_set_graphs(self._h, 1 if enable else 0))

    def set_kernel_timing(self, enable=True):
        _check(lib().dg_set_kernel_timing(self._h, 1 if enable else 0))

    def kernel_time(self, stream=None):
        """(total ms, launches) of the stage kernel since the last call."""
        ms, n = C.c_double(0), C.c_long(0)
        _check(lib().dg_kernel_time(self._h, _stream_handle(stream), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def status(self, stream=None):
        f = C.c_int(0)
        _check(lib().dg_status(self._h, _stream_handle(stream), C.byref(f)))
        return f.value

    def dofs(self):
        return 4 * self.Np * self.K

    def curved_elements(self):
        """Elements the library treats as curved (-1: FP64 nodal handle)."""
        n = C.c_int(0)
        _check(lib().dg_mesh_curved(self._h, C.byref(n)))
        return n.value

    def footprint(self):
        b = C.c_size_t()
        _check(lib().dg_mesh_footprint(self._h, C.byref(b)))
        return b.value


class Tuning:
    """The process-wide tuning table of workgroup shapes (``dg_tuning_*``)."""

    @staticmethod
    def set(arch, P, precision, av, waves):
        _check(lib().dg_tuning_set(arch.encode(), int(P), PRECISIONS[precision], 1 if av else 0, int(waves)))

    @staticmethod
    def lookup(arch, P, precision, av):
        w = C.c_int(0)
        _check(lib().dg_tuning_lookup(arch.encode(), int(P), PRECISIONS[precision], 1 if av else 0,
                                      C.byref(w)))
        return w.value

    @staticmethod
    def clear():
        _check(lib().dg_tuning_clear())

    @staticmethod
    def save(path):
        n = C.c_int(0)
        _check(lib().dg_tuning_save(str(path).encode(), C.byref(n)))
        return n.value

    @staticmethod
    def load(path):
        n = C.c_int(0)
        _check(lib().dg_tuning_load(str(path).encode(), C.byref(n)))
        return n.value

    @staticmethod
    def device_arch():
        buf = C.create_string_buffer(64)
        _check(lib().dg_device_arch(buf, 64))
        return buf.value.decode()


def estimate_footprint(K, P, precision="fp32", av=False):
    b = C.c_size_t()
    _check(lib().dg_estimate_footprint(int(K), int(P), PRECISIONS[precision], 1 if av else 0,
                                       C.byref(b)))
    return b.value


class Batch:
    """Continuous batching of independent solves on one device (the
    ``dg_batch_*`` ABI).  ``admit`` returns a slot id or None when the budget
    or the slots are exhausted."""

    def __init__(self, hbm_budget_bytes, max_slots):
        self._h = C.c_void_p()
        _check(lib().dg_batch_create(int(hbm_budget_bytes), int(max_slots), C.byref(self._h)))
        self.max_slots = int(max_slots)
        self._members = {}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dg_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, solver, U, nsteps, stream=None):
        solver._check_state(U)
        slot = C.c_int(-1)
        rc = lib().dg_batch_admit(self._h, solver._h, C.c_void_p(U.data_ptr()),
                                  C.c_void_p(solver.work.data_ptr()), int(nsteps),
                                  _stream_handle(stream), C.byref(slot))
        if rc == DG_EBUSY:
            return None
        _check(rc)
        self._members[slot.value] = (solver, U)
        return slot.value

    def advance(self, max_steps, stream=None):
        n = C.c_int(0)
        _check(lib().dg_batch_advance(self._h, int(max_steps), _stream_handle(stream), C.byref(n)))
        return n.value

    def poll(self, stream=None):
        buf = (C.c_int * self.max_slots)()
        n = C.c_int(0)
        _check(lib().dg_batch_poll(self._h, _stream_handle(stream), buf, self.max_slots, C.byref(n)))
        return [buf[i] for i in range(min(n.value, self.max_slots))]

    def stats(self, slot, stream=None):
        st = RunStats()
        _check(lib().dg_batch_slot_stats(self._h, int(slot), _stream_handle(stream), C.byref(st)))
        return Stats(st.steps, st.status, st.t, st.dt_min, st.dt_max, tuple(st.totals),
                     tuple(st.residual), st.wall_s, st.dof_updates_per_s)

    def info(self):
        """(graphs captured so far, kinds of solve with tables)."""
        c, g = C.c_int(), C.c_int()
        _check(lib().dg_batch_info(self._h, C.byref(c), C.byref(g)))
        return c.value, g.value

    def release(self, slot):
        _check(lib().dg_batch_release(self._h, int(slot)))
        return self._members.pop(slot, None)
