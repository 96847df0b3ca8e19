"""Initial and reference states (conserved variables rho, rho u, rho v, E).

These are inputs: closed-form flow fields evaluated at given points.  The
state layout matches the solver's: an array (K, 4, Np) of float64.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def primitive_to_conserved(rho, u, v, p, gamma=GAMMA):
    rho, u, v, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, u, v, p)))
    axis = -2 if rho.ndim >= 1 else 0
    return np.stack([rho, rho * u, rho * v,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)], axis=axis)


def freestream_state(mach: float, alpha_deg: float = 0.0, gamma=GAMMA):
    """(rho, rho u, rho v, E) with rho=1, sound speed 1, velocity M(cos a, sin a)."""
    a = np.deg2rad(alpha_deg)
    u = mach * np.cos(a)
    v = mach * np.sin(a)
    p = 1.0 / gamma
    return np.array([1.0, u, v, p / (gamma - 1.0) + 0.5 * (u * u + v * v)])


def cylinder_potential(x, y, mach: float, radius: float = 1.0, gamma=GAMMA):
    """Wall-compatible start for flow past a cylinder of the given radius at
    the origin: the incompressible potential-flow velocity (freestream
    (mach, 0), zero normal velocity on the wall) with density and pressure
    from the isentropic energy relation c^2 = 1 + (gamma-1)/2 (M^2 - |v|^2)
    (rho = c^(2/(gamma-1)), p = rho^gamma / gamma; freestream rho = c = 1)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r2 = (x * x + y * y) / (radius * radius)
    th = np.arctan2(y, x)
    ur = mach * (1.0 - 1.0 / r2) * np.cos(th)
    ut = -mach * (1.0 + 1.0 / r2) * np.sin(th)
    u = ur * np.cos(th) - ut * np.sin(th)
    v = ur * np.sin(th) + ut * np.cos(th)
    c2 = 1.0 + 0.5 * (gamma - 1.0) * (mach * mach - (u * u + v * v))
    if np.any(c2 <= 0):
        raise ValueError("Mach number too high for the isentropic potential start")
    rho = c2 ** (1.0 / (gamma - 1.0))
    return primitive_to_conserved(rho, u, v, rho ** gamma / gamma, gamma)


def wall_damped(x, y, wall_x, wall_y, q, delta: float = 0.2, gamma=GAMMA):
    """Smooth start for flow past a body: the freestream q with its velocity
    scaled by 1 - exp(-(d / delta)^2), d the distance to the nearest of the
    given wall points, at the freestream density and pressure.  The fluid at
    the wall starts at rest (compatible with the slip wall) and the flow
    reaches the freestream a few delta away, so the start launches no
    impulsive wave from the wall."""
    from scipy.spatial import cKDTree
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d, _ = cKDTree(np.c_[np.ravel(wall_x), np.ravel(wall_y)]).query(np.c_[x.ravel(), y.ravel()])
    f = 1.0 - np.exp(-(d.reshape(x.shape) / delta) ** 2)
    q = np.asarray(q, dtype=np.float64)
    rho, u, v = q[0], q[1] / q[0], q[2] / q[0]
    p = (gamma - 1.0) * (q[3] - 0.5 * rho * (u * u + v * v))
    return np.ascontiguousarray(primitive_to_conserved(rho + 0 * x, u * f, v * f, p + 0 * x, gamma))


def uniform(shape_KNp, q):
    """Fill (K,4,Np) with the constant state q (4,)."""
    K, Np = shape_KNp
    return np.ascontiguousarray(np.broadcast_to(np.asarray(q, dtype=np.float64)[None, :, None],
                                                (K, 4, Np)).copy())


def isentropic_vortex(x, y, t=0.0, beta=5.0, x0=5.0, y0=5.0, L=10.0,
                      u_inf=1.0, gamma=GAMMA):
    """Isentropic vortex advected with (u_inf, 0) on a periodic box of side L.

    Velocity perturbation beta*(-ybar, xbar)*exp(1-r^2)/(2 pi) and temperature
    drop (gamma-1) beta^2 exp(2(1-r^2))/(16 gamma pi^2); p = rho^gamma.  This
    pair satisfies radial equilibrium exactly, so the field is a steady vortex
    carried by the uniform flow.  xbar is wrapped to the nearest periodic
    image of the moving centre.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xb = x - x0 - u_inf * t
    xb = xb - L * np.round(xb / L)
    yb = y - y0
    r2 = xb * xb + yb * yb
    e1 = np.exp(1.0 - r2)
    u = u_inf - beta * yb * e1 / (2 * np.pi)
    v = beta * xb * e1 / (2 * np.pi)
    T = 1.0 - (gamma - 1.0) * beta * beta * e1 * e1 / (16.0 * gamma * np.pi ** 2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return np.ascontiguousarray(primitive_to_conserved(rho, u, v, p, gamma))
