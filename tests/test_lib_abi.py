"""The C-ABI library loads, exports every symbol the header declares, and its
host-side reference element agrees with the oracle's (no GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.refelem import ref
from paper_1208_4772_amd import dg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 10
    L = C.CDLL(dg.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert sorted(dg.EXPORTS) == names


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5])
def test_library_nodes_and_operators_match_oracle(P):
    R = ref(P)
    r, s = dg.reference_nodes(P)
    np.testing.assert_allclose(r, R.r, atol=1e-15)
    np.testing.assert_allclose(s, R.s, atol=1e-15)
    np.testing.assert_array_equal(dg.face_nodes(P), R.Fmask)
    ops = dg.reference_operators(P)
    for name, ref_op in (("Dr", R.Dr), ("Ds", R.Ds), ("LIFT", R.LIFT), ("Vinv", R.Vinv)):
        np.testing.assert_allclose(ops[name], ref_op, atol=1e-13 * max(1.0, np.abs(ref_op).max()))


def test_bad_order_is_rejected():
    with pytest.raises(dg.DGError) as e:
        dg.reference_nodes(6)
    assert e.value.code == dg.DG_EINVAL
    assert "1..5" in str(e.value)


def test_setup_rejects_bad_input_before_touching_the_device():
    """Validation failures return DG_EINVAL with a message (host checks)."""
    L = dg.lib()

    def setup(**over):
        K, P = 2, 1
        e2e = np.array([[1, 1, 1], [0, 0, 0]], dtype=np.int32)
        e2f = np.array([[0, 1, 2], [0, 1, 2]], dtype=np.int32)
        bc = np.zeros((K, 3), dtype=np.int8)
        x = np.zeros((K, 3))
        y = np.zeros((K, 3))
        arrs = dict(EToE=e2e, EToF=e2f, bc=bc, x=x, y=y)
        arrs.update({k: v for k, v in over.items() if k in arrs})
        d = dg.MeshDesc()
        d.K = over.get("K", K)
        d.P = over.get("P", P)
        d.precision = over.get("precision", dg.DG_FP64_PLAIN)
        d.gamma = over.get("gamma", 1.4)
        d.cfl = 0.5
        keep = {k: np.ascontiguousarray(v) for k, v in arrs.items()}
        for k, v in keep.items():
            setattr(d, k, v.ctypes.data)
        d.av_kappa = 1.0
        h = C.c_void_p()
        rc = L.dg_mesh_setup(C.byref(d), None, C.byref(h))
        return rc, L.dg_last_error().decode(), h.value

    rc, msg, h = setup(P=0)
    assert rc == dg.DG_EINVAL and h is None
    rc, msg, _ = setup(K=0)
    assert rc == dg.DG_EINVAL
    rc, msg, _ = setup(precision=7)
    assert rc == dg.DG_EINVAL
    rc, msg, _ = setup(gamma=1.0)
    assert rc == dg.DG_EINVAL
    # element 0 face 0 says neighbour 1 face 0, but element 1 face 0 points to 0 face 0:
    # reciprocal; break it
    rc, msg, _ = setup(EToF=np.array([[1, 1, 2], [0, 1, 2]], dtype=np.int32))
    assert rc == dg.DG_EINVAL and "reciprocal" in msg
    rc, msg, _ = setup(bc=np.array([[0, 0, 3], [0, 0, 0]], dtype=np.int8))
    assert rc == dg.DG_EINVAL and "bc code" in msg
    rc, msg, _ = setup(EToE=np.array([[5, 1, 1], [0, 0, 0]], dtype=np.int32))
    assert rc == dg.DG_EINVAL and "out of range" in msg
    rc, msg, _ = setup(bc=np.array([[1, 0, 0], [0, 0, 0]], dtype=np.int8))
    assert rc == dg.DG_EINVAL


def test_one_hip_runtime_in_process():
    """Loading the library must not bring a second HIP runtime next to the
    one torch uses (a second copy does not see the device)."""
    import subprocess
    import sys
    code = ("from paper_1208_4772_amd import dg; dg.lib(); import torch; "
            "m = open('/proc/self/maps').read().splitlines(); "
            "print(len({l.split()[-1] for l in m if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True,
                         cwd=ROOT)
    assert out.stdout.strip().splitlines()[-1] == "1"


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5])
def test_library_weak_operators_match_oracle(P):
    """The library's cubature rule and weak-form operators (C++ Newton roots,
    Christoffel weights) against the oracle's (SciPy Gauss rules)."""
    from oracle.refelem import weak_ops
    L = dg.weak_operators(P)
    W = weak_ops(P)
    for name in ("wq", "Icub", "Drc", "Dsc", "wg", "If"):
        ref_op = getattr(W, name)
        np.testing.assert_allclose(L[name], ref_op, atol=1e-13 * max(1.0, np.abs(ref_op).max()))
