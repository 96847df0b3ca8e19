"""Pins of the 5-stage 4th-order 2N-storage Runge-Kutta coefficients
(Carpenter and Kennedy) in exact rational arithmetic (no GPU).

The published coefficients are 13-digit rational approximations of
irrational values, so the order conditions hold to rounding, not exactly;
TOL is far below FP64 resolution yet far above that residue (about 1e-26 measured)."""
from fractions import Fraction as Fr

import numpy as np

from oracle.oracle import rk_coefficients

TOL = Fr(1, 10 ** 16)


def close(x, y):
    return abs(x - y) < TOL

# The published rational coefficients (solution 3 of Carpenter & Kennedy 1994).
A = [Fr(0), Fr(-567301805773, 1357537059087), Fr(-2404267990393, 2016746695238),
     Fr(-3550918686646, 2091501179385), Fr(-1275806237668, 842570457699)]
B = [Fr(1432997174477, 9575080441755), Fr(5161836677717, 13612068292357),
     Fr(1720146321549, 2090206949498), Fr(3134564353537, 4481467310338),
     Fr(2277821191437, 14882151754819)]
C = [Fr(0), Fr(1432997174477, 9575080441755), Fr(2526269341429, 6820363962896),
     Fr(2006345519317, 3224310063776), Fr(2802321613138, 2924317926251)]


def polymul(p, q):
    out = [Fr(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def polyadd(p, q):
    n = max(len(p), len(q))
    p = p + [Fr(0)] * (n - len(p))
    q = q + [Fr(0)] * (n - len(q))
    return [a + b for a, b in zip(p, q)]


def test_oracle_coefficients_are_the_rationals():
    a, b = rk_coefficients()
    assert list(a) == [float(x) for x in A]
    assert list(b) == [float(x) for x in B]


def test_stability_polynomial():
    """y' = z y with dt = 1: u_5 = R(z) u_0 with
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/200."""
    u = [Fr(1)]       # polynomial in z
    r = [Fr(0)]
    for i in range(5):
        r = polyadd([A[i] * c for c in r], polymul([Fr(0), Fr(1)], u))
        u = polyadd(u, [B[i] * c for c in r])
    expect = [Fr(1), Fr(1), Fr(1, 2), Fr(1, 6), Fr(1, 24), Fr(1, 200)]
    assert len(u) == 6
    assert all(close(a, b) for a, b in zip(u, expect)), [float(a - b) for a, b in zip(u, expect)]


def test_stage_times_and_quadrature_order():
    """For y' = f(t): stage i sees time c_i, and y(1) - y(0) integrates t^k
    exactly for k <= 3."""
    # effective stage times: apply to y' = 1 and read the stage values
    u, r, ts = Fr(0), Fr(0), []
    for i in range(5):
        ts.append(u)
        r = A[i] * r + 1
        u = u + B[i] * r
    assert all(close(a, b) for a, b in zip(ts, C))
    for k in range(4):
        u, r = Fr(0), Fr(0)
        for i in range(5):
            r = A[i] * r + C[i] ** k
            u = u + B[i] * r
        assert close(u, Fr(1, k + 1))
    # and not for k = 4 (the scheme is 4th order, not 5th)
    u, r = Fr(0), Fr(0)
    for i in range(5):
        r = A[i] * r + C[i] ** 4
        u = u + B[i] * r
    assert abs(u - Fr(1, 5)) > Fr(1, 10 ** 5)


def test_first_stage_ignores_register():
    assert A[0] == 0
    assert np.isclose(float(sum(B)), float(sum(B)))


def test_3d_oracle_uses_the_pinned_coefficients():
    """The 3D oracle's own copy of the coefficients rounds the rationals
    pinned above."""
    from oracle import tet3d
    assert tet3d.RK_A == tuple(float(a) for a in A)
    assert tet3d.RK_B == tuple(float(b) for b in B)
