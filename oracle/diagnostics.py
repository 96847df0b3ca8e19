"""FP64 diagnostics of a solution state, for the CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the solver.  Every
quantity is evaluated from the oracle's own geometric factors
(:class:`oracle.oracle.Oracle`) and reference element
(:mod:`oracle.refelem`); nothing here is shared with the solver's host code.

Definitions (the paper reports its cases through these quantities without
defining them discretely; Section 5, the cylinder, airfoil and sphere
paragraphs):

* conserved-variable mass weights w_ki = sum_j M_ij J_kj (exact L2 weights of
  the nodal interpolant on a straight element);
* entropy error e = (p / rho^gamma) / (p_inf / rho_inf^gamma) - 1 and its L2
  norm over the domain, normalised by the domain area (an RMS value);
* pressure force on the slip walls, F = sum over wall faces of the integral
  of p n ds, n the element's outward normal (it points into the body), by
  the face's Gauss-Lobatto rule (the row sums of the 1D face mass matrix);
  drag and lift coefficients with respect to the freestream direction,
  C_D = (F_x cos a + F_y sin a) / (q_inf c), C_L = (-F_x sin a + F_y cos a) /
  (q_inf c), q_inf = rho_inf |v_inf|^2 / 2;
* shock position: on the upper surface (wall nodes with y > 0), ordered by
  x, the last place where the pressure coefficient rises through the
  critical value C_p* = 2 / (gamma M^2) [((2 + (gamma-1) M^2) / (gamma+1))
  ^(gamma/(gamma-1)) - 1], linearly interpolated between the two nodes.
"""
from __future__ import annotations

import math

import numpy as np

WALL = 1


def _pressure(U, gamma):
    rho, mx, my, E = U[..., 0, :], U[..., 1, :], U[..., 2, :], U[..., 3, :]
    return (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)


def _freestream(q, gamma):
    q = np.asarray(q, dtype=np.float64)
    rho, u, v = q[0], q[1] / q[0], q[2] / q[0]
    p = (gamma - 1.0) * (q[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def mass_weights(o):
    """(K, Np) weights w_ki = sum_j M_ij J_kj."""
    return o.geo["J"] @ o.ref.M.T


def entropy_error(o, U, freestream, gamma=1.4):
    """RMS over the domain of (s - s_inf) / s_inf, s = p / rho^gamma."""
    U = np.asarray(U, dtype=np.float64)
    rho0, _, _, p0 = _freestream(freestream, gamma)
    s0 = p0 / rho0 ** gamma
    e = _pressure(U, gamma) / U[:, 0, :] ** gamma / s0 - 1.0
    w = mass_weights(o)
    return math.sqrt(float((w * e * e).sum()) / float(w.sum()))


def _wall_nodes(o):
    """Element, face-node index and quadrature weight (times sJ) of every
    wall face node."""
    R = o.ref
    Nfp = R.Nfp
    wq = np.concatenate([R.Emat[R.Fmask[f], f * Nfp:(f + 1) * Nfp].sum(axis=1) for f in range(3)])
    ks, fs = np.nonzero(np.asarray(o.bc) == WALL)
    ek, eq, ew = [], [], []
    for k, f in zip(ks.tolist(), fs.tolist()):
        for j in range(Nfp):
            q = f * Nfp + j
            ek.append(k)
            eq.append(q)
            ew.append(wq[q] * o.geo["sJ"][k, q])
    return np.array(ek, dtype=np.int64), np.array(eq, dtype=np.int64), np.array(ew)


def wall_force(o, U, gamma=1.4):
    """(F_x, F_y): pressure integrated over the wall faces along the element
    outward normals (the force the fluid exerts on the body)."""
    U = np.asarray(U, dtype=np.float64)
    ek, eq, ew = _wall_nodes(o)
    if ek.size == 0:
        return 0.0, 0.0
    v = o.ref.Fmask.ravel()[eq]
    u = U[ek, :, v]                                   # (n, 4)
    rho, mx, my, E = u[:, 0], u[:, 1], u[:, 2], u[:, 3]
    p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)
    nx, ny = o.geo["nx"][ek, eq], o.geo["ny"][ek, eq]
    return float((p * nx * ew).sum()), float((p * ny * ew).sum())


def lift_drag(o, U, freestream, gamma=1.4, chord=1.0):
    """(C_L, C_D) of the wall pressure force."""
    rho0, u0, v0, _ = _freestream(freestream, gamma)
    V2 = u0 * u0 + v0 * v0
    qdyn = 0.5 * rho0 * V2 * chord
    ca, sa = u0 / math.sqrt(V2), v0 / math.sqrt(V2)
    Fx, Fy = wall_force(o, U, gamma)
    return (-Fx * sa + Fy * ca) / qdyn, (Fx * ca + Fy * sa) / qdyn


def critical_cp(mach, gamma=1.4):
    """Pressure coefficient at which the local Mach number is one."""
    g = gamma
    return 2.0 / (g * mach * mach) * (((2.0 + (g - 1.0) * mach * mach) / (g + 1.0)) ** (g / (g - 1.0)) - 1.0)


def upper_surface_cp(o, U, freestream, gamma=1.4):
    """(x, C_p) at the upper-surface wall nodes (y > 0), sorted by x, with
    nodes shared by two wall faces counted once."""
    U = np.asarray(U, dtype=np.float64)
    rho0, u0, v0, p0 = _freestream(freestream, gamma)
    qdyn = 0.5 * rho0 * (u0 * u0 + v0 * v0)
    ek, eq, _ = _wall_nodes(o)
    v = o.ref.Fmask.ravel()[eq]
    xw, yw = o.x[ek, v], o.y[ek, v]
    u = U[ek, :, v]
    p = (gamma - 1.0) * (u[:, 3] - 0.5 * (u[:, 1] ** 2 + u[:, 2] ** 2) / u[:, 0])
    cp = (p - p0) / qdyn
    up = yw > 0.0
    order = np.argsort(xw[up], kind="stable")
    xs, cs = xw[up][order], cp[up][order]
    keep = np.concatenate([[True], np.diff(xs) > 1e-12]) if xs.size else np.zeros(0, bool)
    return xs[keep], cs[keep]


def shock_position(o, U, freestream, mach, gamma=1.4):
    """x of the last upward crossing of C_p* on the upper surface, linear
    between wall nodes (NaN if the pressure coefficient never rises through
    it).  Behind the shock the flow stays subsonic to the trailing edge;
    earlier crossings are pressure wiggles near the leading edge."""
    xs, cs = upper_surface_cp(o, U, freestream, gamma)
    cstar = critical_cp(mach, gamma)
    x = float("nan")
    for i in range(xs.size - 1):
        if cs[i] < cstar <= cs[i + 1]:
            x = float(xs[i] + (cstar - cs[i]) / (cs[i + 1] - cs[i]) * (xs[i + 1] - xs[i]))
    return x
