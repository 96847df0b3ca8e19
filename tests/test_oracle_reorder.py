"""How far two valid evaluation orders of the FP64 oracle differ (no GPU).

The oracle is built twice from the same source: once with every operation
rounded separately, once with products and sums contracted into fused
multiply-adds wherever the compiler can.  Both are correct FP64
evaluations of the same discretisation; their difference is the spread any
other FP64 implementation (the GPU's, with its own operation order) must be
expected to show against the oracle.  On the one-million-element P=5 mesh the
flux derivatives cancel about 1,800-fold in the rhs, and the spread exceeds
1e-12 relative L2: the FP64 parity bar there is stated as a multiple of this
measured spread instead.  A second source of the same size is the rounding
of the reference operators themselves: Dr and Ds re-rounded so that their
rows sum to zero exactly (as the exact matrices do) are another valid FP64
representation.  A third is the rounding of the metric terms (the same
geometry translated per element)."""
import numpy as np
import pytest

import meshgen
from oracle import oracle as orc
from oracle.refelem import ref


def perturbed(case, amp=0.05):
    """The same smooth perturbation of the freestream the GPU parity test of
    this mesh uses."""
    x, y, q = case.x, case.y, case.freestream
    rho0, u0, v0 = q[0], q[1] / q[0], q[2] / q[0]
    p0 = 0.4 * (q[3] - 0.5 * rho0 * (u0 * u0 + v0 * v0))
    rho = rho0 * (1 + amp * np.sin(x) * np.cos(0.7 * y))
    u = u0 + amp * np.sin(0.9 * y)
    v = v0 + amp * np.cos(1.1 * x)
    p = p0 * (1 + amp * np.cos(x + 0.5 * y))
    return meshgen.primitive_to_conserved(rho, u, v, p)


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_contracted_build_is_a_different_rounding_of_the_same_rhs():
    """On a small mesh the two builds agree to a few units in the last
    place (same arithmetic) but not bit for bit (different rounding)."""
    R = ref(3)
    case = meshgen.make_case("vortex", R.r, R.s, P=3)
    a = orc.Oracle.for_case(case).rhs(case.U0)
    b = orc.Oracle.for_case(case, fma=True).rhs(case.U0)
    err = rel_l2(b, a)
    assert 0.0 < err < 1e-13


def exact_row_sums(o):
    """Re-round the oracle's Dr and Ds in place so that every row sums to
    zero in FP64 (diagonal = minus the sum of the off-diagonal entries): a
    second FP64 representation of the same exact matrices, which annihilate
    constants."""
    for A in (o.Dr, o.Ds):
        n = A.shape[0]
        A[np.arange(n), np.arange(n)] = 0.0
        A[np.arange(n), np.arange(n)] = -A.sum(axis=1)
    return o


def oracle_spread(case, U):
    """Largest relative L2 difference between the rhs of U from valid FP64
    evaluations of the oracle: as built, with contraction, with the
    operators re-rounded to exact zero row sums, and with every element's
    node coordinates translated by its first node (the discrete operator is
    invariant under a per-element translation; only the rounding of the
    metric terms, which cancel ~1,000-fold in Dr x on these small elements
    far from the origin, changes)."""
    rhs = [orc.Oracle.for_case(case).rhs(U),
           orc.Oracle.for_case(case, fma=True).rhs(U),
           exact_row_sums(orc.Oracle.for_case(case)).rhs(U)]
    xs, ys = case.x - case.x[:, :1], case.y - case.y[:, :1]
    rhs.append(orc.Oracle(case.mesh, case.P, xs, ys, freestream=case.freestream,
                          gamma=case.gamma).rhs(U))
    return max(rel_l2(a, b) for i, a in enumerate(rhs) for b in rhs[:i])


@pytest.mark.slow
def test_roofline_mesh_spread_exceeds_the_plain_bar():
    R = ref(5)
    case = meshgen.make_case("roofline", R.r, R.s)
    spread = oracle_spread(case, perturbed(case))
    print(f"oracle self-spread on the roofline mesh: {spread:.3e}")
    assert spread > 1e-12
